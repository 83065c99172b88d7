"""Full-size parity of the three larger workloads, in the launch
configurations the benchmark times, through the C ABI.

* N = 4,194,304, K = 8, alpha = 1/32, Q = 65,536 perturbed queries (16,384
  clusters): every precision's result equals the exhaustive GPU search on
  every query, and a strided sample of 512 queries equals the oracle's
  branch-and-bound (Theorem 1), the exhaustive search included.
* The learned seed at N = 4,194,304, K = 16, alpha = 1/8 (512 k-means++
  anchors, 200,000 training queries): the single pass with the trained
  model returns exactly the plain two-pass results on all 65,536 held-out
  queries and the oracle's on a sample; the pruned fractions of both seeds
  are reported and the plain seed's survivor counts are bracketed by the
  oracle's exact sets.
* 64 databases (N_d log-uniform in [4,096, 2,097,152], ragged batches of 1 to
  4,096 queries, K_d and alpha_d mixed): the multi-database plan replayed
  from its HIP graph equals one hn_search_top1 per database on every query,
  in every precision, and the oracle on sampled queries of every database.

Inputs come from hn_inputs (the benchmark's generators); indices are
bit-exact and similarities equal to the oracle's canonical float64 sums.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import hn_inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

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


def assert_exact(gi, gs, ri, rs, what):
    bad = np.nonzero(np.asarray(gi) != ri)[0]
    assert bad.size == 0, "%s: %d index mismatches, first at %d" % (what, bad.size, bad[0])
    d = np.abs(np.asarray(gs) - rs)
    assert (d <= SIM_TOL).all(), "%s: max |dsim| = %g" % (what, d.max())


def same(a, b):
    import torch
    return bool(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]))


def test_workload3_full_size_every_precision(hn):
    t0 = time.perf_counter()
    w = hn_inputs.workload(3)
    db = w.db()
    qs = w.queries(db)
    say("workload3: N=%d K=%d alpha=%g Q=%d generated in %.0f s" % (
        w.n, w.k, w.alpha, len(qs), time.perf_counter() - t0))
    d_db, dq = dev(db), dev(qs)
    ix = hn.Index(d_db, w.k, w.alpha)
    bf = hn.bruteforce_top1(d_db, dq)
    sample = np.arange(0, len(qs), len(qs) // 512)
    ref = oracle.bnb_top1(db, qs[sample], w.k, w.alpha)
    bi, bs = bf[0].cpu().numpy(), bf[1].cpu().numpy()
    assert_exact(bi[sample], bs[sample], ref["idx"], ref["sim"], "workload3 exhaustive")
    for prec in ("fp32", "bf16", "fp8", "int8"):
        say("workload3: %s search" % prec)
        idx, sim, aux, st = ix.search(dq, precision=prec, aux=True, stats=True)
        assert same((idx, sim), bf), prec
        assert_exact(idx.cpu().numpy()[sample], sim.cpu().numpy()[sample], ref["idx"],
                     ref["sim"], "workload3 " + prec)
        surv = aux["survivors"].double()
        say("workload3 %s: pruned %.4f%%, %.1f survivors/query, %d overflow queries" % (
            prec, 100.0 * (1 - float(surv.mean()) / w.n), float(surv.mean()),
            st["overflow_queries"]))
    say("workload3: %.0f s" % (time.perf_counter() - t0))
    ix.close()


def test_workload5_full_size_learned_seed(hn):
    import torch
    t0 = time.perf_counter()
    w = hn_inputs.workload(5)
    db = w.db()
    qs = w.queries(db)
    qt = w.train_queries(db)
    say("workload5: N=%d, %d held-out + %d training queries generated in %.0f s" % (
        w.n, len(qs), len(qt), time.perf_counter() - t0))
    d_db, dq = dev(db), dev(qs)
    ix = hn.Index(d_db, w.k, w.alpha)
    u = dev(hn_inputs.uniform_draws(w.extra["n_anchor"], w.extra["anchor_seed"]))
    anchors = ix.kmeanspp(w.extra["n_anchor"], u)
    labels = ix.seed_labels(anchors, dev(qt))
    params = dev(hn_inputs.mlp_init(w.extra["train_seed"] + 1))
    losses = hn.seed_train(params, dev(qt), labels, batch=1024, epochs=4, lr=2e-3)
    ls = losses.cpu().numpy()
    per_epoch = len(ls) // 4
    say("workload5: model trained, loss %.3f -> %.3f" % (ls[:per_epoch].mean(),
                                                         ls[-per_epoch:].mean()))
    assert ls[-per_epoch:].mean() < ls[:per_epoch].mean()
    ix.set_seed_model(params, anchors)
    plain = ix.search(dq, precision="bf16", aux=True)
    learned = ix.search(dq, precision="bf16", seed="learned", aux=True)
    assert same(plain[:2], learned[:2])
    sample = np.arange(0, len(qs), len(qs) // 256)
    ref = oracle.bnb_top1(db, qs[sample], w.k, w.alpha)
    assert_exact(plain[0].cpu().numpy()[sample], plain[1].cpu().numpy()[sample], ref["idx"],
                 ref["sim"], "workload5")
    # pruned fractions of both seeds; the plain seed's survivor counts lie
    # between the oracle's exact sets at its own L
    pa, la = plain[2], learned[2]
    sp, sl_ = pa["survivors"].double(), la["survivors"].double()
    L = pa["seed_sim"].cpu().numpy()
    eps = pa["slack"].cpu().numpy()
    lo, hi = oracle.survivor_counts(db, qs[sample], w.k, w.alpha,
                                    L[sample] - 2 * eps[sample] - 2.0 ** -20,
                                    L[sample] + 2.0 ** -40)
    s_plain = pa["survivors"].cpu().numpy()[sample]
    assert (hi <= s_plain).all() and (s_plain <= lo).all()
    # the two bounds judged by the oracle: exact survivor sets S(q, L) at
    # the plain seed's L and at the learned seed's L
    Lq = la["seed_sim"].cpu().numpy()[sample]
    Lq = np.where(np.isfinite(Lq), Lq, -np.inf)
    at_plain, _ = oracle.survivor_counts(db, qs[sample], w.k, w.alpha, L[sample], L[sample])
    at_learned, _ = oracle.survivor_counts(db, qs[sample], w.k, w.alpha, Lq, Lq)
    assert (Lq <= plain[1].cpu().numpy()[sample]).all()  # a real entry's sim: admissible
    say("workload5 oracle |S(q, L)| per query: plain L %.1f, learned L %.1f" % (
        at_plain.mean(), at_learned.mean()))
    Ll = torch.nan_to_num(la["seed_sim"], neginf=float("nan"))
    say("workload5 pruned: plain seed %.4f%% (%.1f survivors/query, mean L %.3f), learned "
        "single pass %.4f%% (%.1f survivors/query, mean L %.3f)" % (
            100.0 * (1 - float(sp.mean()) / w.n), float(sp.mean()), float(pa["seed_sim"].mean()),
            100.0 * (1 - float(sl_.mean()) / w.n), float(sl_.mean()), float(Ll.nanmean())))
    say("workload5: %.0f s" % (time.perf_counter() - t0))
    ix.close()


def test_workload4_full_size_batched_plans(hn):
    import torch
    t0 = time.perf_counter()
    specs = hn_inputs.batched_set()

    def gen(sp):
        db = sp.db()
        return db, sp.queries(db)

    with ThreadPoolExecutor(16) as ex:
        data = list(ex.map(gen, specs))
    say("workload4: %d databases, %d entries, %d queries generated in %.0f s" % (
        len(specs), sum(sp.n for sp in specs), sum(sp.q for sp in specs),
        time.perf_counter() - t0))
    ixs = [hn.Index(dev(db), sp.k, sp.alpha) for sp, (db, _) in zip(specs, data)]
    counts = [len(q) for _, q in data]
    dq = dev(np.concatenate([q for _, q in data]))
    offs = np.concatenate([[0], np.cumsum(counts)])
    # oracle on sampled queries of every database: first, last and up to 4 more
    picks, refs = [], []
    for d, ((db, q), sp) in enumerate(zip(data, specs)):
        s = np.unique(np.concatenate([[0, len(q) - 1], np.linspace(0, len(q) - 1, 6).astype(int)]))
        r = oracle.bnb_top1(db, q[s], sp.k, sp.alpha)
        picks.append(offs[d] + s)
        refs.append((r["idx"], r["sim"]))
    picks = np.concatenate(picks)
    ref_i = np.concatenate([r[0] for r in refs])
    ref_s = np.concatenate([r[1] for r in refs])
    say("workload4: oracle on %d sampled queries (%.0f s)" % (len(picks), time.perf_counter() - t0))
    for prec in ("fp32", "bf16", "fp8", "int8"):
        singles = [ix.search(dq[offs[d]:offs[d + 1]], precision=prec)
                   for d, ix in enumerate(ixs) if counts[d]]
        s_idx = torch.cat([s[0] for s in singles])
        s_sim = torch.cat([s[1] for s in singles])
        plan = hn.MultiPlan(ixs, counts, precision=prec)
        out = (torch.empty(len(dq), dtype=torch.int64, device="cuda:0"),
               torch.empty(len(dq), dtype=torch.float64, device="cuda:0"))
        for rep in range(3):  # the captured graph, replayed
            out[0].fill_(-5)
            plan.search(dq, use_graph=True, out=out)
            torch.cuda.synchronize()
            assert same(out, (s_idx, s_sim)), (prec, rep)
        assert_exact(out[0].cpu().numpy()[picks], out[1].cpu().numpy()[picks], ref_i, ref_s,
                     "workload4 " + prec)
        say("workload4 %s: plan (graph, 3 replays) == single searches == oracle sample" % prec)
        plan.close()
    say("workload4: %.0f s" % (time.perf_counter() - t0))
    for ix in ixs:
        ix.close()
