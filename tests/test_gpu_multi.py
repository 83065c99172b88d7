"""GPU parity of the multi-database search (one plan over ragged query
batches against several indexes) against the CPU float64 oracle, through the
C ABI: every query's index bit-exact and its sim within 1e-12 of the oracle's
branch-and-bound on its own database, eagerly and through the captured HIP
graph (replayed several times with eager work and new queries in between)."""
import numpy as np
import pytest

import hn_inputs
import oracle

pytestmark = pytest.mark.gpu

SIM_TOL = 1e-12


@pytest.fixture(scope="module")
def hn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2606_27280_amd as hn
    hn._lib.lib()
    return hn


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def say(msg):
    print(msg, flush=True)


# (n, k, alpha, queries): ragged sizes, mixed K and alpha, an empty batch,
# a one-entry database and ties from duplicated rows
SPECS = [(5000, 8, 1 / 32, 70), (1, 16, 1 / 8, 3), (300, 16, 1 / 8, 0), (20000, 16, 1 / 8, 301),
         (4096, 8, 1 / 8, 1), (777, 8, 0.0, 40), (12345, 16, 1 / 32, 129)]


def _dbs(seed0, specs=SPECS):
    out = []
    for t, (n, k, a, q) in enumerate(specs):
        db = hn_inputs.make_db(n, k, a, max(1, n // 200), seed0 + t)
        if n >= 8:
            db[n - 1] = db[2]
        qs = hn_inputs.make_queries(db, k, a, q - q // 5, q // 5, seed0 + 100 + t)
        out.append((db, qs, k, a))
    return out


def _reference(dbs):
    idx, sim = [], []
    for db, qs, k, a in dbs:
        if len(qs):
            r = oracle.bnb_top1(db, qs, k, a)
            idx.append(r["idx"])
            sim.append(r["sim"])
    return np.concatenate(idx), np.concatenate(sim)


def _check(idx, sim, ref, what):
    ri, rs = ref
    idx = idx.cpu().numpy()
    sim = sim.cpu().numpy()
    bad = np.nonzero(idx != ri)[0]
    assert bad.size == 0, "%s: %d mismatches, first %d" % (what, bad.size, bad[0])
    assert (np.abs(sim - rs) <= SIM_TOL).all(), what


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8", "int8"])
def test_multi_matches_oracle(hn, precision):
    dbs = _dbs(7000)
    ref = _reference(dbs)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    qs = np.concatenate([q for _, q, _, _ in dbs])
    say("multi plan: %d databases, %d queries, %s" % (len(dbs), len(qs), precision))
    plan = hn.MultiPlan(ixs, [len(q) for _, q, _, _ in dbs], precision=precision)
    info = plan.info()
    assert info["total_queries"] == len(qs)
    # fp32 groups K=8 and K=16 streams (two widths); bf16/fp8 share one
    assert info["scan_launches"] == (4 if precision == "fp32" else 2)
    dq = dev(qs)
    for use_graph in (False, True):
        say("multi search graph=%s" % use_graph)
        idx, sim = plan.search(dq, use_graph=use_graph)
        _check(idx, sim, ref, "%s graph=%s" % (precision, use_graph))
    plan.close()
    for ix in ixs:
        ix.close()


def test_multi_graph_replays_and_new_queries(hn):
    import torch
    dbs = _dbs(7100)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    counts = [len(q) for _, q, _, _ in dbs]
    plan = hn.MultiPlan(ixs, counts, precision="bf16")
    buf = torch.empty((sum(counts), 128), dtype=torch.float32, device="cuda:0")
    idx = torch.empty(sum(counts), dtype=torch.int64, device="cuda:0")
    sim = torch.empty(sum(counts), dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        # fresh queries each replay (same layout), eager work in between
        fresh = [(db, hn_inputs.make_queries(db, k, a, len(q), 0, 7200 + 10 * rep + t), k, a)
                 for t, (db, q, k, a) in enumerate(dbs)]
        buf.copy_(dev(np.concatenate([q for _, q, _, _ in fresh])))
        say("graph replay %d" % rep)
        plan.search(buf, use_graph=True, out=(idx, sim))
        torch.cuda.synchronize()
        _check(idx, sim, _reference(fresh), "replay %d" % rep)
        e_idx, e_sim = plan.search(buf, use_graph=False)
        assert torch.equal(e_idx, idx) and torch.equal(e_sim, sim)
        _ = torch.ones(1000, device="cuda:0").sum().item()
    # other output buffers: captured again
    idx2, sim2 = plan.search(buf, use_graph=True)
    assert torch.equal(idx2, idx) and torch.equal(sim2, sim)
    plan.close()
    for ix in ixs:
        ix.close()


def test_multi_equals_single_searches(hn):
    """Same results as one hn_search_top1 per database (any configuration)."""
    import torch
    dbs = _dbs(7300)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    qs = [q for _, q, _, _ in dbs]
    singles = [ix.search(dev(q)) if len(q) else None for ix, q in zip(ixs, qs)]
    s_idx = torch.cat([r[0] for r in singles if r is not None])
    s_sim = torch.cat([r[1] for r in singles if r is not None])
    for qt, cb in ((1, 0), (2, 8), (0, 64)):
        say("multi query_tiles=%d chunk_blocks=%d" % (qt, cb))
        plan = hn.MultiPlan(ixs, [len(q) for q in qs], query_tiles=qt, chunk_blocks=cb)
        idx, sim = plan.search(dev(np.concatenate(qs)))
        assert torch.equal(idx, s_idx) and torch.equal(sim, s_sim)
        plan.close()
    for ix in ixs:
        ix.close()


def test_multi_rejects(hn):
    db = hn_inputs.make_db(500, 64, 1 / 8, 4, 1)
    ix64 = hn.Index(dev(db), 64, 1 / 8)
    db2 = hn_inputs.make_db(500, 16, 1 / 8, 4, 2)
    ix16 = hn.Index(dev(db2), 16, 1 / 8)
    say("multi rejects")
    with pytest.raises(hn.HNError) as e:
        hn.MultiPlan([ix16, ix64], [3, 3])
    assert e.value.code == -5
    with pytest.raises(hn.HNError):
        hn.MultiPlan([ix16], [-1])
    import paper_2606_27280_amd._lib as L
    o = L.SearchOpts(0, 1, 0, 0, 0, -1.0)  # learned seed
    import ctypes
    h = ctypes.c_void_p()
    hs = (ctypes.c_void_p * 1)(ix16._h.value)
    qc = (ctypes.c_int64 * 1)(2)
    rc = L.lib().hn_multi_plan_create(hs, 1, qc, ctypes.byref(o), ctypes.byref(h))
    assert rc == -5
    plan = hn.MultiPlan([ix16], [0])
    import torch
    i, s = plan.search(torch.empty((0, 128), dtype=torch.float32, device="cuda:0"))
    assert i.numel() == 0
    plan.close()
    ix64.close()
    ix16.close()


def _self_queries(db, k, alpha, count):
    """q = x_i, rows whose stored minor norm exceeds sqrt(alpha) first."""
    x = db.astype(np.float64)
    over = np.nonzero((x[:, k:] ** 2).sum(1) > alpha)[0]
    rest = np.setdiff1d(np.arange(len(db)), over)
    pick = np.concatenate([over[: count // 2], rest])[:count]
    return db[pick].copy()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "int8"])
def test_multi_self_and_minor_heavy_queries(hn, precision):
    """Exact self-queries (including rows with a float32 minor-norm excess)
    and queries whose minor block is scaled up (the bound needs the slack's
    norm term) in every database of a plan: results equal the oracle's."""
    dbs = []
    for db, qs, k, a in _dbs(7400):
        if len(qs):
            heavy = qs.astype(np.float64)
            heavy[:, k:] *= 2.0
            qs = np.concatenate([qs, heavy.astype(np.float32),
                                 _self_queries(db, k, a, min(len(db), 6))])
        dbs.append((db, qs, k, a))
    ref = _reference(dbs)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    qs = np.concatenate([q for _, q, _, _ in dbs])
    say("multi plan with self and minor-heavy queries: %d queries, %s" % (len(qs), precision))
    plan = hn.MultiPlan(ixs, [len(q) for _, q, _, _ in dbs], precision=precision)
    for use_graph in (False, True):
        idx, sim = plan.search(dev(qs), use_graph=use_graph)
        _check(idx, sim, ref, "%s self/heavy graph=%s" % (precision, use_graph))
    plan.close()
    for ix in ixs:
        ix.close()


def test_multi_batch_times_from_the_replay(hn):
    """Device timestamps inside the replayed graph: one time per database,
    positive where the database has queries, 0 where it has none, and no
    later than the search's own length."""
    import torch
    dbs = _dbs(7500)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    counts = [len(q) for _, q, _, _ in dbs]
    plan = hn.MultiPlan(ixs, counts, precision="bf16")
    dq = dev(np.concatenate([q for _, q, _, _ in dbs]))
    out = (torch.empty(len(dq), dtype=torch.int64, device="cuda:0"),
           torch.empty(len(dq), dtype=torch.float64, device="cuda:0"))
    plan.search(dq, use_graph=True, out=out)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    plan.search(dq, use_graph=True, out=out)
    b.record()
    torch.cuda.synchronize()
    total = a.elapsed_time(b)
    ms = plan.batch_times()
    say("batch times (ms): %s; whole replay %.4f ms" % (["%.4f" % v for v in ms], total))
    assert len(ms) == len(counts)
    for c, v in zip(counts, ms):
        if c:
            assert 0.0 < v <= total * 1.05 + 0.01
        else:
            assert v == 0.0
    _check(*out, _reference(dbs), "timed replay")
    plan.close()
    for ix in ixs:
        ix.close()


def test_autotuner_single_and_multi(hn, tmp_path):
    """The tuner times every candidate launch shape, rejects any shape that
    changes a result (all are bit-identical by construction), keeps the
    fastest and caches it."""
    from paper_2606_27280_amd.autotune import Tuner
    import hn_inputs
    dbs = _dbs(7600)
    ixs = [hn.Index(dev(db), k, a) for db, _, k, a in dbs]
    counts = [len(q) for _, q, _, _ in dbs]
    dq = dev(np.concatenate([q for _, q, _, _ in dbs]))
    t = Tuner(str(tmp_path / "tune.json"))
    say("tune multi")
    best, table = t.tune_multi(ixs, counts, dq, precision="bf16", query_tiles=(1, 2),
                               chunk_blocks=(0, 16), reps=2)
    assert set(table) == {(1, 0), (1, 16), (2, 0), (2, 16)}
    assert best in table and table[best] == min(table.values())
    w = hn_inputs.workload(1)
    db = w.db()
    qs = dev(w.queries(db))
    ix = hn.Index(dev(db), w.k, w.alpha)
    say("tune single")
    best1, table1 = t.tune(ix, qs, precision="fp32", query_tiles=(1, 2), chunk_blocks=(0, 32),
                           reps=2)
    assert len(table1) == 4 and table1[best1] == min(table1.values())
    import torch
    t2 = Tuner(str(tmp_path / "tune.json"))
    assert t2.lookup(torch.cuda.get_device_name(0), ix.n, ix.k, "fp32", len(qs)) == best1
    i_b, s_b = ix.search(qs, query_tiles=best1[0], chunk_blocks=best1[1])
    i_0, s_0 = ix.search(qs)
    assert torch.equal(i_b, i_0) and torch.equal(s_b, s_0)
    ix.close()
    for x in ixs:
        x.close()
