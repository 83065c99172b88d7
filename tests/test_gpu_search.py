"""GPU parity of the HIP path against the CPU float64 oracle, through the C ABI.

Indices must be bit-exact and similarities equal to the oracle's canonical
float64 sim (tolerance 1e-12; the kernels reproduce the canonical sum, so the
expected difference is 0).  Survivor sets are checked against the oracle's
exact seed-threshold sets S(q, L) with the GPU's own L.
"""
import math

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


def assert_exact(gi, gs, ri, rs, what=""):
    gi = np.asarray(gi)
    gs = np.asarray(gs)
    bad = np.nonzero(gi != ri)[0]
    assert bad.size == 0, "%s: %d index mismatches, first q=%d gpu=%d oracle=%d" % (
        what, bad.size, bad[0], gi[bad[0]], ri[bad[0]])
    d = np.abs(gs - rs)
    assert (d <= SIM_TOL).all(), "%s: max |dsim| = %g" % (what, d.max())


def exact_must(db, q, L):
    """{i : sim(q, x_i) >= L} with the canonical float64 sim: the entries an
    exact search must rescore (the bound of Eq. 3 is only a means to this).
    A float64 matmul screens; entries within 1e-9 of L are decided by the
    oracle's canonical sim."""
    s = db.astype(np.float64) @ q.astype(np.float64)
    near = np.nonzero(s >= L - 1e-9)[0]
    return {int(i) for i in near if oracle.sim(q, db[i]) >= L}


def self_queries(db, k, alpha, count):
    """Rows of the database as queries (q = x_i), the rows whose stored minor
    block exceeds sqrt(alpha) in norm (float32 rounding) first: for them the
    literal Eq. 3 bound fails on the self pair."""
    x = db.astype(np.float64)
    over = np.nonzero((x[:, k:] ** 2).sum(1) > alpha)[0]
    rest = np.setdiff1d(np.arange(len(db)), over)
    pick = np.concatenate([over[: count // 2], rest[: count - min(len(over), count // 2)]])
    return db[pick[:count]].copy(), int(min(len(over), count // 2))


# ------------------------------------------------------------ scan numerics

@pytest.mark.parametrize("k", [1, 5, 8, 16, 40, 127])
def test_scan_scores_fp32_within_rounding_bound(hn, k):
    alpha = 1 / 8
    db = hn_inputs.make_db(1005, k, alpha, 7, 100 + k)
    qs = hn_inputs.make_queries(db, k, alpha, 30, 7, 200 + k)
    say("scan_scores fp32 k=%d n=1005 q=37" % k)
    ix = hn.Index(dev(db), k, alpha)
    got = ix.scan_scores(dev(qs), "fp32").cpu().numpy().astype(np.float64)
    ref = qs[:, :k].astype(np.float64) @ db[:, :k].astype(np.float64).T
    absprod = np.abs(qs[:, :k]).astype(np.float64) @ np.abs(db[:, :k]).astype(np.float64).T
    gam = k * 2.0 ** -23 / (1 - k * 2.0 ** -23)
    err = np.abs(got - ref)
    assert (err <= gam * absprod + k * 2.0 ** -125 + 1e-15).all(), err.max()
    ix.close()


@pytest.mark.parametrize("k", [8, 16, 30, 64])
def test_scan_scores_bf16_within_rounding_bound(hn, k):
    alpha = 1 / 32
    db = hn_inputs.make_db(999, k, alpha, 5, 300 + k)
    qs = hn_inputs.make_queries(db, k, alpha, 20, 5, 400 + k)
    say("scan_scores bf16 k=%d n=999 q=25" % k)
    ix = hn.Index(dev(db), k, alpha)
    got = ix.scan_scores(dev(qs), "bf16").cpu().numpy().astype(np.float64)
    ref = qs[:, :k].astype(np.float64) @ db[:, :k].astype(np.float64).T
    absprod = np.abs(qs[:, :k]).astype(np.float64) @ np.abs(db[:, :k]).astype(np.float64).T
    ub = 2.0 ** -8
    bound = absprod * ((2 * ub + ub * ub) + k * 2.0 ** -23 / (1 - k * 2.0 ** -23) * (1 + ub) ** 2)
    err = np.abs(got - ref)
    assert (err <= bound + k * 2.0 ** -125 + 1e-15).all(), (err - bound).max()
    # and the rounding really happened (this is not the float32 path)
    assert err.max() > 1e-5
    # the matrix core sums the exact products of the rounded operands with
    # float32-sized error (torch's round-to-nearest-even bf16 cast)
    import torch
    q16 = torch.from_numpy(qs[:, :k]).to(torch.bfloat16).double().numpy()
    x16 = torch.from_numpy(db[:, :k]).to(torch.bfloat16).double().numpy()
    gam = k * 2.0 ** -23 / (1 - k * 2.0 ** -23)
    d = np.abs(got - q16 @ x16.T)
    assert (d <= gam * (np.abs(q16) @ np.abs(x16).T) + 1e-30).all(), d.max()
    ix.close()


def _fp8_copy(a):
    """OCP E4M3FN copy (round to nearest even, torch's CPU cast) of a float32
    matrix with the power-of-two scale 2^(e - 8), amax = f 2^e, 0.5 <= f < 1:
    returns (scale, float64 values of the scaled codes times the scale)."""
    import torch
    amax = float(np.abs(a).max())
    scale = 1.0 if amax == 0 else math.ldexp(1.0, math.frexp(amax)[1] - 8)
    codes = torch.from_numpy(np.ascontiguousarray(a / np.float32(scale), dtype=np.float32))
    back = codes.to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.isfinite(back).all()
    return scale, back * scale


@pytest.mark.parametrize("k", [1, 8, 16, 30, 32])
def test_scan_scores_fp8_exact_products_and_bound(hn, k):
    """The fp8 scan score is the float32 sum of exact E4M3 products, rescaled
    (the codes are contracted on the bf16 matrix core):
    it matches the float64 dot of the quantised operands up to float32
    accumulation, and the true prefix dot within the residual-norm bound the
    search's slack uses."""
    alpha = 1 / 8
    db = hn_inputs.make_db(1003, k, alpha, 9, 500 + k)
    qs = hn_inputs.make_queries(db, k, alpha, 28, 9, 600 + k)
    qs[0, :k] *= 1e-4  # a query with tiny components: subnormal fp8 codes
    say("scan_scores fp8 k=%d n=1003 q=37" % k)
    ix = hn.Index(dev(db), k, alpha, flags=hn.HN_BUILD_NO_VALIDATE)
    got = ix.scan_scores(dev(qs), "fp8").cpu().numpy().astype(np.float64)
    _, x8 = _fp8_copy(db[:, :k])
    q8 = np.stack([_fp8_copy(q[None, :k])[1][0] for q in qs])
    quant = q8 @ x8.T  # exact: products of E4M3 values, few terms
    acc = np.abs(q8) @ np.abs(x8).T
    gam = k * 2.0 ** -23 / (1 - k * 2.0 ** -23)
    d = np.abs(got - quant)
    assert (d <= gam * acc + 1e-30).all(), d.max()
    ref = qs[:, :k].astype(np.float64) @ db[:, :k].astype(np.float64).T
    rx = np.sqrt(((x8 - db[:, :k]) ** 2).sum(1)).max()
    mu8 = np.sqrt((x8 ** 2).sum(1)).max()
    rq = np.sqrt(((q8 - qs[:, :k]) ** 2).sum(1))
    nq = np.sqrt((qs[:, :k].astype(np.float64) ** 2).sum(1))
    bound = rq[:, None] * mu8 + nq[:, None] * rx + gam * (nq + rq)[:, None] * mu8
    assert (np.abs(got - ref) <= bound + 1e-15).all()
    if k > 1:
        assert np.abs(got - ref).max() > 1e-4  # the quantisation really happened
    ix.close()


def _int8_codes(a, amax):
    """round(a / s) clipped to [-127, 127], s = 2^(e - 7) for amax = f 2^e,
    0.5 <= f < 1 (numpy's rint: nearest, ties to even)."""
    s = 1.0 if amax == 0 else math.ldexp(1.0, math.frexp(amax)[1] - 7)
    c = np.clip(np.rint(np.asarray(a, dtype=np.float64) / s), -127, 127).astype(np.int64)
    return s, c


@pytest.mark.parametrize("k", [1, 8, 16, 30, 32])
def test_scan_scores_int8_exact_and_bound(hn, k):
    """The int8 scan score is s_q s_x times the exact integer dot of the codes
    (bit for bit), and within the residual-norm bound of the true prefix dot."""
    alpha = 1 / 32
    db = hn_inputs.make_db(1007, k, alpha, 9, 700 + k)
    qs = hn_inputs.make_queries(db, k, alpha, 28, 9, 800 + k)
    qs[0, :k] *= 1e-3
    say("scan_scores int8 k=%d n=1007 q=37" % k)
    ix = hn.Index(dev(db), k, alpha, flags=hn.HN_BUILD_NO_VALIDATE)
    got = ix.scan_scores(dev(qs), "int8").cpu().numpy()
    sx, xc = _int8_codes(db[:, :k], float(np.abs(db[:, :k]).max()))
    exp = np.empty((len(qs), len(db)), dtype=np.float64)
    rq = np.empty(len(qs))
    for i, q in enumerate(qs):
        sq, qc = _int8_codes(q[:k], float(np.abs(q[:k]).max()))
        exp[i] = (xc @ qc).astype(np.float64) * sq * sx
        rq[i] = np.sqrt(((qc * sq - q[:k].astype(np.float64)) ** 2).sum())
    assert np.array_equal(got.astype(np.float64), exp)
    ref = qs[:, :k].astype(np.float64) @ db[:, :k].astype(np.float64).T
    xr = xc * sx
    rx = np.sqrt(((xr - db[:, :k]) ** 2).sum(1)).max()
    mux = np.sqrt((xr ** 2).sum(1)).max()
    nq = np.sqrt((qs[:, :k].astype(np.float64) ** 2).sum(1))
    bound = rq[:, None] * mux + nq[:, None] * rx
    assert (np.abs(got - ref) <= bound + 1e-15).all()
    ix.close()


# ------------------------------------------------------------ exact search

def _check_search(hn, db, qs, k, alpha, precision="fp32", what="", **kw):
    say("search %s: n=%d k=%d alpha=%g q=%d precision=%s %s" % (
        what, len(db), k, alpha, len(qs), precision, kw))
    ix = hn.Index(dev(db), k, alpha, **({"flags": kw.pop("flags")} if "flags" in kw else {}))
    idx, sim, aux, st = ix.search(dev(qs), precision=precision, aux=True, stats=True, **kw)
    ref = oracle.bnb_top1(db, qs, k, alpha)
    assert_exact(idx.cpu().numpy(), sim.cpu().numpy(), ref["idx"], ref["sim"], what)
    out = {n: t.cpu().numpy() for n, t in aux.items()}
    ix.close()
    return ref, out, st


def test_workload1_all_precisions_exact(hn):
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    bi, bs = oracle.bruteforce_top1(db, qs)
    for prec in ("fp32", "bf16", "fp8", "int8"):
        ref, aux, st = _check_search(hn, db, qs, w.k, w.alpha, prec, "workload1")
        assert (ref["idx"] == bi).all()
        assert st["overflow_queries"] == 0
        # the seed bound is the canonical sim of a real entry
        for qi in range(0, len(qs), 17):
            assert aux["seed_sim"][qi] == oracle.sim(qs[qi], db[aux["seed_idx"][qi]])
        # survivor counts bracketed by the oracle's exact sets at the GPU's L
        L = aux["seed_sim"]
        lo, hi = oracle.survivor_counts(db, qs, w.k, w.alpha,
                                        L - 2 * aux["slack"] - 2.0 ** -20, L + 2.0 ** -40)
        assert (hi <= aux["survivors"]).all() and (aux["survivors"] <= lo).all()
        assert st["survivors"] == int(aux["survivors"].sum())


@pytest.mark.parametrize("n,k,alpha,nq", [
    (1, 8, 1 / 32, 5), (2, 16, 1 / 8, 4), (17, 16, 1 / 8, 3), (100, 1, 0.25, 20),
    (300, 127, 0.5, 33), (1000, 16, 0.0, 50), (4097, 16, 1 / 8, 1), (5000, 8, 1 / 32, 600),
    (3001, 40, 1 / 16, 70), (2000, 64, 1 / 4, 17)])
def test_edge_shapes_exact(hn, n, k, alpha, nq):
    db = hn_inputs.make_db(n, k, alpha, max(1, n // 64), 1000 + n + k)
    qs = hn_inputs.make_queries(db, k, alpha, nq - nq // 4, nq // 4, 2000 + n + k)
    if n >= 8:  # exact ties: duplicated rows
        db[n - 1] = db[0]
        db[n // 2] = db[3]
    # exact self-queries (q = x_i), rows with a float32 minor-norm excess first
    sq, _ = self_queries(db, k, alpha, min(n, 8))
    qs = np.concatenate([qs, sq])
    for prec in ("fp32", "bf16", "fp8", "int8"):
        if prec in ("fp8", "int8") and k > 32:
            continue  # no fp8 / int8 copy above k = 32 (checked in test_invalid_inputs)
        _check_search(hn, db, qs, k, alpha, prec, "edge")


def test_tie_rule_golden_on_gpu(hn):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tie_rule.json")))
    db = np.zeros((3, 128), dtype=np.float32)
    db[:, :4] = np.array(g["db"], dtype=np.float32)
    q = np.zeros((1, 128), dtype=np.float32)
    q[0, :4] = g["query"]
    for prec in ("fp32", "bf16", "fp8", "int8"):
        ref, aux, _ = _check_search(hn, db, q, g["k"], g["alpha"], prec, "tie-golden",
                                    flags=hn.HN_BUILD_NO_VALIDATE)
        assert ref["idx"][0] == g["expected_idx"]
        # the GPU seed rescoring may pick any admissible entry (here the whole
        # winning 4-entry group, so entry 0 itself); its bound is its own sim
        assert aux["seed_sim"][0] == oracle.sim(q[0], db[aux["seed_idx"][0]])
    say("bruteforce tie-golden")
    bi, bs = hn.bruteforce_top1(dev(db), dev(q))
    assert int(bi.cpu()[0]) == g["expected_idx"] and float(bs.cpu()[0]) == g["expected_sim"]


def test_duplicates_everywhere_and_overflow_fallback(hn):
    k, alpha = 16, 1 / 8
    base = hn_inputs.make_db(64, k, alpha, 2, 77)
    db = np.tile(base, (40, 1))  # every row repeated 40 times
    qs = hn_inputs.make_queries(base, k, alpha, 24, 8, 78)
    ref, aux, st = _check_search(hn, db, qs, k, alpha, "fp32", "dup", survivor_cap=500)
    assert st["overflow_queries"] > 0
    assert (ref["idx"] < 64).all()  # smallest index among the copies
    ref2, aux2, st2 = _check_search(hn, db, qs, k, alpha, "fp32", "dup-nocap")
    assert st2["overflow_queries"] == 0


def test_invalid_inputs(hn):
    import torch
    k, alpha = 8, 1 / 32
    db = hn_inputs.make_db(500, k, alpha, 4, 5)
    bad = db.copy()
    bad[123, :k] *= 1.01
    say("build with an off-norm row")
    with pytest.raises(hn.HNError) as e:
        hn.Index(dev(bad), k, alpha)
    assert e.value.code == -2 and "123" in str(e.value)
    ix = hn.Index(dev(bad), k, alpha, flags=hn.HN_BUILD_NO_VALIDATE)  # stays exact
    qs = hn_inputs.make_queries(db, k, alpha, 40, 10, 6)
    idx, sim = ix.search(dev(qs))
    ref = oracle.bnb_top1(bad, qs, k, alpha)
    assert_exact(idx.cpu().numpy(), sim.cpu().numpy(), ref["idx"], ref["sim"], "off-norm")
    ix.close()
    nan = db.copy()
    nan[7, 50] = np.nan
    say("build with a NaN row")
    for fl in (0, hn.HN_BUILD_NO_VALIDATE):
        with pytest.raises(hn.HNError):
            hn.Index(dev(nan), k, alpha, flags=fl)
    say("search with a NaN query")
    ix = hn.Index(dev(db), k, alpha)
    q2 = qs.copy()
    q2[3, 0] = np.inf
    idx, sim = ix.search(dev(q2))
    idx, sim = idx.cpu().numpy(), sim.cpu().numpy()
    assert idx[3] == -1 and math.isnan(sim[3])
    ok = np.arange(len(q2)) != 3
    ref = oracle.bnb_top1(db, q2[ok], k, alpha)
    assert_exact(idx[ok], sim[ok], ref["idx"], ref["sim"], "nan-query")
    e0 = torch.empty(0, 128, dtype=torch.float32, device="cuda:0")
    i0, s0 = ix.search(e0)
    assert i0.numel() == 0
    with pytest.raises(ValueError):
        ix.search(dev(qs).double())
    with pytest.raises(hn.HNError):
        ix.search(dev(qs), precision=7)
    with pytest.raises(hn.HNError):
        ix.search(dev(qs), beta=0.5)
    say("misaligned row pointers")
    buf = torch.zeros(len(qs) * 128 + 1, dtype=torch.float32, device="cuda:0")
    shifted = buf[1:].view(len(qs), 128)  # contiguous, 4 bytes past a 16-byte boundary
    shifted.copy_(dev(qs))
    with pytest.raises(hn.HNError) as e:
        ix.search(shifted)
    assert e.value.code == -1 and "aligned" in str(e.value)
    with pytest.raises(hn.HNError):
        hn.bruteforce_top1(dev(db), shifted)
    with pytest.raises(hn.HNError):
        hn.hn_layer(shifted, k, alpha)
    ix.close()
    say("fp8 on k = 40 (no fp8 copy)")
    db40 = hn_inputs.make_db(300, 40, alpha, 3, 8)
    ix = hn.Index(dev(db40), 40, alpha)
    with pytest.raises(hn.HNError) as e:
        ix.search(dev(hn_inputs.make_queries(db40, 40, alpha, 4, 1, 9)), precision="fp8")
    assert e.value.code == -5
    ix.close()
    with pytest.raises(ValueError):  # the binding checks the width
        hn.Index(dev(db[:, :64]), k, alpha)


def test_determinism_configs_and_batch_invariance(hn):
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    ix = hn.Index(dev(db), w.k, w.alpha)
    dq = dev(qs)
    say("determinism: default config x3")
    base = ix.search(dq, aux=True)
    b_idx, b_sim = base[0].cpu().numpy(), base[1].cpu().numpy()
    b_surv = base[2]["survivors"].cpu().numpy()
    for rep in range(2):
        r = ix.search(dq, aux=True)
        assert (r[0].cpu().numpy() == b_idx).all()
        assert np.array_equal(r[1].cpu().numpy().view(np.int64), b_sim.view(np.int64))
        assert (r[2]["survivors"].cpu().numpy() == b_surv).all()
    for qt in (1, 2, 4, 8):
        for cb in (0, 8, 37, 1024):
            say("determinism: query_tiles=%d chunk_blocks=%d" % (qt, cb))
            r = ix.search(dq, query_tiles=qt, chunk_blocks=cb, aux=True)
            assert (r[0].cpu().numpy() == b_idx).all()
            assert np.array_equal(r[1].cpu().numpy().view(np.int64), b_sim.view(np.int64))
            assert (r[2]["survivors"].cpu().numpy() == b_surv).all()
    for lo, hi in ((37, 150), (0, 1), (255, 256), (100, 117)):
        say("batch invariance: queries[%d:%d]" % (lo, hi))
        r = ix.search(dev(qs[lo:hi]), aux=True)
        assert (r[0].cpu().numpy() == b_idx[lo:hi]).all()
        assert (r[2]["survivors"].cpu().numpy() == b_surv[lo:hi]).all()
    ix.close()


def test_filter_survivor_sets_match_oracle(hn):
    import torch
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)[:24]
    ix = hn.Index(dev(db), w.k, w.alpha)
    say("filter survivors: 24 queries, L from the GPU seed")
    _, _, aux = ix.search(dev(qs), aux=True)
    L = aux["seed_sim"]
    pairs, cnt, slack = ix.filter_survivors(dev(qs), L, cap=1 << 20)
    assert cnt == pairs.shape[0]
    pairs = pairs.cpu().numpy()
    L = L.cpu().numpy()
    slack = slack.cpu().numpy()
    need = [exact_must(db, qs[qi], L[qi]) for qi in range(len(qs))]
    for qi in range(len(qs)):
        got = set(pairs[pairs[:, 0] == qi, 1].tolist())
        must = set(oracle.survivor_list(db, qs[qi], w.k, w.alpha, L[qi] + 2.0 ** -40).tolist())
        may = set(oracle.survivor_list(db, qs[qi], w.k, w.alpha,
                                       L[qi] - 2 * slack[qi] - 2.0 ** -20).tolist())
        assert must <= got <= may, qi
        # what exactness needs: every entry whose full sim reaches L
        assert need[qi] <= got, qi
    # the low-precision filters against the same sets, within their own slack
    for prec in ("bf16", "fp8", "int8"):
        say("filter survivors: %s" % prec)
        pp, pc, ps = ix.filter_survivors(dev(qs), dev(L), cap=1 << 20, precision=prec)
        pp, ps = pp[:pc].cpu().numpy(), ps.cpu().numpy()
        for qi in range(len(qs)):
            got = set(pp[pp[:, 0] == qi, 1].tolist())
            must = set(oracle.survivor_list(db, qs[qi], w.k, w.alpha, L[qi] + 2.0 ** -40).tolist())
            may = set(oracle.survivor_list(db, qs[qi], w.k, w.alpha,
                                           L[qi] - 2 * ps[qi] - 2.0 ** -20).tolist())
            assert must <= got <= may, (prec, qi)
            assert need[qi] <= got, (prec, qi)
    # a lower bound of -inf keeps everything; +inf keeps nothing
    lo = torch.full((3,), -math.inf, dtype=torch.float64, device="cuda:0")
    _, c_all, _ = ix.filter_survivors(dev(qs[:3]), lo, cap=0)
    assert c_all == 3 * len(db)
    _, c_none, _ = ix.filter_survivors(dev(qs[:3]), -lo, cap=0)
    assert c_none == 0
    for prec in ("bf16", "fp8", "int8"):
        _, c_all, _ = ix.filter_survivors(dev(qs[:3]), lo, cap=0, precision=prec)
        assert c_all == 3 * len(db), prec
        _, c_none, _ = ix.filter_survivors(dev(qs[:3]), -lo, cap=0, precision=prec)
        assert c_none == 0, prec
    ix.close()


def test_int8_filter_equals_thresholded_scores(hn):
    """The int8 filter compares exact integer sums with integer thresholds;
    its pairs are exactly the entries whose int8 scan score (from the score
    buffer, the same sums as float32) reaches the search's threshold."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)[:40]
    ix = hn.Index(dev(db), w.k, w.alpha)
    say("int8 filter vs thresholded int8 scan scores: 40 queries")
    _, _, aux = ix.search(dev(qs), aux=True, precision="int8")
    L = aux["seed_sim"]
    thr = aux["threshold"].cpu().numpy()  # in int8 scan units
    scores = ix.scan_scores(dev(qs), precision="int8").cpu().numpy()
    pp, pc, _ = ix.filter_survivors(dev(qs), L, cap=1 << 20, precision="int8")
    pp = pp[:pc].cpu().numpy()
    def scale(v):  # the power-of-two int8 scale 2^(e-7) of max |v[:k]| = f 2^e
        return np.ldexp(1.0, np.frexp(np.float32(np.abs(v[..., :w.k]).max()))[1] - 7)

    sx = scale(db)
    n_checked = 0
    for qi in range(len(qs)):
        # the score buffer holds the sums times s_q s_x (powers of two: exact)
        units = scores[qi].astype(np.float64) / (scale(qs[qi]) * sx)
        got = set(pp[pp[:, 0] == qi, 1].tolist())
        want = set(np.nonzero(units >= thr[qi])[0].tolist())
        assert got == want, qi
        n_checked += len(want)
    assert n_checked > 0
    ix.close()


@pytest.mark.parametrize("scale", [1.0, 2.0, 3.0])
def test_minor_heavy_and_self_queries_need_the_norm_slack(hn, scale):
    """Queries need not be HN-normalised.  With the minor block of q scaled up
    (||q_m|| = scale sqrt(alpha)) the bound dot_K + alpha of Eq. 3 no longer
    holds (the minor product reaches scale * alpha), and the search stays
    exact only through the slack's norm term max(0, ||q_m|| mu_m - alpha).
    Self-queries add the float32 case of the same term (rows whose stored
    minor norm exceeds sqrt(alpha)).  Every precision must return the
    oracle's result, and every entry whose full sim reaches the GPU's L must
    survive the filter."""
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(6000, k, alpha, 20, 5600)
    qs = hn_inputs.make_queries(db, k, alpha, 40, 8, 5601).astype(np.float64)
    qs[:, k:] *= scale
    qs = qs.astype(np.float32)
    sq, n_over = self_queries(db, k, alpha, 16)
    assert n_over > 0
    qs = np.concatenate([qs, sq])
    say("minor-heavy queries: scale=%g, %d self-queries (%d with norm excess)" % (
        scale, len(sq), n_over))
    ix = hn.Index(dev(db), k, alpha)
    ref = oracle.bnb_top1(db, qs, k, alpha)
    for prec in ("fp32", "bf16", "fp8", "int8"):
        idx, sim, aux = ix.search(dev(qs), precision=prec, aux=True)
        assert_exact(idx.cpu().numpy(), sim.cpu().numpy(), ref["idx"], ref["sim"],
                     "minor x%g %s" % (scale, prec))
        L = aux["seed_sim"]
        pairs, cnt, _ = ix.filter_survivors(dev(qs), L, cap=1 << 22, precision=prec)
        assert cnt == pairs.shape[0]
        pairs = pairs.cpu().numpy()
        Lh = L.cpu().numpy()
        for qi in range(0, len(qs), 3):
            got = set(pairs[pairs[:, 0] == qi, 1].tolist())
            assert exact_must(db, qs[qi], Lh[qi]) <= got, (prec, qi)
    ix.close()


def test_seed_scan_precision_does_not_change_results(hn):
    """The plain seed's argmax scan on the float32 prefix (the all-float32
    search) and on the bf16 copy give the same exact results in every filter
    precision; only the seed and the survivor counts may differ."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    ix = hn.Index(dev(db), w.k, w.alpha)
    ref = oracle.bnb_top1(db, qs, w.k, w.alpha)
    for prec in ("fp32", "bf16", "fp8", "int8"):
        for ss in ("fp32", "bf16"):
            say("seed scan %s, filter %s" % (ss, prec))
            idx, sim, aux = ix.search(dev(qs), precision=prec, seed_scan=ss, aux=True)
            assert_exact(idx.cpu().numpy(), sim.cpu().numpy(), ref["idx"], ref["sim"],
                         "seed_scan=%s %s" % (ss, prec))
            si = aux["seed_idx"].cpu().numpy()
            sv = aux["seed_sim"].cpu().numpy()
            for qi in range(0, len(qs), 31):
                assert sv[qi] == oracle.sim(qs[qi], db[si[qi]])
    with pytest.raises(hn.HNError):
        ix.search(dev(qs), seed_scan=5)
    ix.close()


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("n,nq", [(1, 3), (15, 4), (1000, 33), (4103, 70), (16384, 256)])
def test_bruteforce_exact(hn, n, nq):
    db = hn_inputs.make_db(n, 16, 1 / 8, max(1, n // 128), 3000 + n)
    qs = hn_inputs.make_queries(db, 16, 1 / 8, nq - nq // 3, nq // 3, 3100 + n)
    if n >= 8:
        db[n - 2] = db[1]
    say("bruteforce n=%d q=%d" % (n, nq))
    gi, gs = hn.bruteforce_top1(dev(db), dev(qs))
    ri, rs = oracle.bruteforce_top1(db, qs)
    assert_exact(gi.cpu().numpy(), gs.cpu().numpy(), ri, rs, "bruteforce")


def test_bruteforce_all_identical_rows_fallback(hn):
    row = hn_inputs.make_db(1, 16, 1 / 8, 1, 9)
    db = np.tile(row, (70000, 1))
    qs = hn_inputs.make_queries(row, 16, 1 / 8, 2, 1, 10)
    say("bruteforce identical rows n=70000 q=3 (candidate overflow)")
    gi, gs = hn.bruteforce_top1(dev(db), dev(qs))
    assert (gi.cpu().numpy() == 0).all()
    for qi in range(3):
        assert gs.cpu().numpy()[qi] == oracle.sim(qs[qi], row[0])


# ------------------------------------------------------------ full size

def torch_equal(i1, s1, i2, s2):
    import torch
    return bool(torch.equal(i1, i2) and torch.equal(s1, s2))


def test_workload2_full_size_sampled(hn):
    """N = 1,048,576, K = 16, alpha = 1/8, Q = 10,000 in the benchmark's launch
    configuration.  Every query: HN result == exhaustive GPU result and the
    sim equals the oracle's canonical sim of the returned entry; a strided
    sample of 500 queries against the oracle's branch-and-bound."""
    w = hn_inputs.workload(2)
    db = w.db()
    qs = w.queries(db)
    say("workload2 full: build + search fp32/bf16/fp8 + bruteforce")
    ix = hn.Index(dev(db), w.k, w.alpha)
    dq = dev(qs)
    i32, s32, aux, st = ix.search(dq, aux=True, stats=True)
    i16, s16 = ix.search(dq, precision="bf16")
    i8, s8 = ix.search(dq, precision="fp8")
    ii, si_ = ix.search(dq, precision="int8")
    assert torch_equal(ii, si_, i32, s32)
    bi, bs = hn.bruteforce_top1(dev(db), dq)
    i32, s32, i16, s16, i8, s8 = (t.cpu().numpy() for t in (i32, s32, i16, s16, i8, s8))
    bi, bs = bi.cpu().numpy(), bs.cpu().numpy()
    assert (i32 == bi).all() and np.array_equal(s32, bs)
    assert (i16 == bi).all() and np.array_equal(s16, bs)
    assert (i8 == bi).all() and np.array_equal(s8, bs)
    assert st["overflow_queries"] == 0
    sample = np.arange(0, len(qs), 20)
    ref = oracle.bnb_top1(db, qs[sample], w.k, w.alpha)
    assert_exact(i32[sample], s32[sample], ref["idx"], ref["sim"], "workload2-sample")
    rng = np.random.default_rng(0)
    for qi in rng.choice(len(qs), 200, replace=False):
        assert s32[qi] == oracle.sim(qs[qi], db[i32[qi]])
    sb = np.arange(3, len(qs), 625)
    ri, rs = oracle.bruteforce_top1(db, qs[sb])
    assert_exact(bi[sb], bs[sb], ri, rs, "workload2-bruteforce-sample")
    surv = aux["survivors"].cpu().numpy()
    L = aux["seed_sim"].cpu().numpy()
    sl = aux["slack"].cpu().numpy()
    lo, hi = oracle.survivor_counts(db, qs[sample], w.k, w.alpha,
                                    L[sample] - 2 * sl[sample] - 2.0 ** -20, L[sample] + 2.0 ** -40)
    assert (hi <= surv[sample]).all() and (surv[sample] <= lo).all()
    pruned = 1.0 - surv.mean() / len(db)
    say("workload2: pruned %.4f%%, survivors/query %.1f" % (100 * pruned, surv.mean()))
    assert pruned > 0.99
    ix.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8", "int8"])
def test_overflow_paths_exact(hn, precision):
    """Two clusters over 30,000 entries: a query keeps thousands of
    survivors, more than a list of 2,048 pairs per query holds, so most
    queries overflow the first pass.  The fp32 and bf16 searches finish them
    with the exhaustive float64 pass (no synchronisation); the fp8 and int8
    searches search them again with a float32 filter pass seeded with their
    best candidate and a list sized from the first pass's pair count; the
    noalloc form takes the exhaustive pass.  All exact."""
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(30000, k, alpha, 2, 6100)
    qs = hn_inputs.make_queries(db, k, alpha, 40, 4, 6101)
    ref = oracle.bnb_top1(db, qs, k, alpha)
    ix = hn.Index(dev(db), k, alpha)
    say("overflow paths %s: n=30000, 2 clusters" % precision)
    cap = 2048 * len(qs)
    idx, sim, st = ix.search(dev(qs), precision=precision, stats=True, survivor_cap=cap)
    assert st["overflow_queries"] > len(qs) // 2
    assert_exact(idx.cpu().numpy(), sim.cpu().numpy(), ref["idx"], ref["sim"], "overflow")
    if precision in ("fp32", "bf16"):
        ni, ns = ix.search_noalloc(dev(qs), precision=precision, survivor_cap=cap)
        assert_exact(ni.cpu().numpy(), ns.cpu().numpy(), ref["idx"], ref["sim"], "noalloc")
    ix.close()


def test_fp8_overflow_rerun_exact(hn):
    """fp8 scans keep many more pairs; a list far too small sends the
    overflowing queries through a float32 filter pass seeded with the best
    candidate each reached."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    ref, aux, st = _check_search(hn, db, qs, w.k, w.alpha, "fp8", "fp8-rerun", survivor_cap=700)
    assert st["overflow_queries"] > 0


@pytest.mark.parametrize("frac", [0.75, 0.5, 0.0])
def test_soft_beta_mode(hn, frac):
    """Soft mode (Section 7): beta < alpha replaces alpha in the skip test.
    The result is a real entry (sim <= the exact best), it is at least as good
    as every entry the weakened test must keep (dot_K + beta >= L), and the
    first-pass survivors only shrink as beta falls."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)[:64]
    beta = frac * w.alpha
    say("soft mode beta=%g" % beta)
    ix = hn.Index(dev(db), w.k, w.alpha)
    ei, es, ea = ix.search(dev(qs), aux=True)
    si, ss, sa = ix.search(dev(qs), beta=beta, aux=True)
    ei, es, si, ss = (t.cpu().numpy() for t in (ei, es, si, ss))
    L = sa["seed_sim"].cpu().numpy()
    assert (ss <= es).all()
    assert (sa["survivors"].cpu().numpy() <= ea["survivors"].cpu().numpy()).all()
    # Algorithm 1 with beta in the skip test (the oracle's running-best form)
    soft = oracle.bnb_top1(db, qs, w.k, w.alpha, beta=beta)
    assert (soft["sim"] <= es).all()
    for qi in range(len(qs)):
        assert ss[qi] == oracle.sim(qs[qi], db[si[qi]])
        must = oracle.survivor_list(db, qs[qi], w.k, beta, L[qi] + 2.0 ** -40)
        if len(must):
            best_must = max(oracle.sim(qs[qi], db[j]) for j in must)
            assert ss[qi] >= best_must
        # both results r are fixed points of the weakened bound: no entry
        # whose major score plus beta reaches r beats it
        for r in (ss[qi], soft["sim"][qi]):
            reach = oracle.survivor_list(db, qs[qi], w.k, beta, r + 2.0 ** -40)
            if len(reach):
                assert max(oracle.sim(qs[qi], db[j]) for j in reach) <= r
    recall = float((si == ei).mean())
    say("recall@1 at beta=%g: GPU (seed threshold) %.3f, Algorithm 1 (running best) %.3f" % (
        beta, recall, float((soft["idx"] == ei).mean())))
    ix.close()


def test_filter_lower_minus_inf_ragged(hn):
    """L = -inf keeps every real entry and nothing past the database end
    (a size that is not a multiple of the scan's row blocks)."""
    import torch
    db = hn_inputs.make_db(1001, 16, 1 / 8, 10, 5150)
    qs = hn_inputs.make_queries(db, 16, 1 / 8, 5, 0, 5151)
    ix = hn.Index(dev(db), 16, 1 / 8)
    lo = torch.full((5,), -math.inf, dtype=torch.float64, device="cuda:0")
    say("filter with L = -inf, n = 1001")
    for prec in ("fp32", "bf16", "int8"):
        pairs, c_all, _ = ix.filter_survivors(dev(qs), lo, cap=1 << 16, precision=prec)
        assert c_all == 5 * 1001
        assert int(pairs[:, 1].max()) == 1000
    ix.close()


def test_concurrent_streams_and_threads(hn):
    """One index searched from three host threads at once, each on its own
    stream and precision (per-stream scratch): every result equals the
    single-stream search."""
    import threading

    import torch
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    ix = hn.Index(dev(db), w.k, w.alpha)
    dq = dev(qs)
    ref_i, ref_s = ix.search(dq)
    torch.cuda.synchronize()
    precs = ("fp32", "bf16", "int8")
    streams = [torch.cuda.Stream() for _ in precs]
    results, errors = [None] * len(precs), []

    def work(t):
        try:
            with torch.cuda.stream(streams[t]):
                outs = [ix.search(dq, precision=precs[t]) for _ in range(4)]
            streams[t].synchronize()
            results[t] = outs
        except Exception as e:  # reported below
            errors.append(e)

    say("3 threads x 4 searches on 3 streams")
    threads = [threading.Thread(target=work, args=(t,)) for t in range(len(precs))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for t in range(len(precs)):
        for i, s in results[t]:
            assert torch.equal(i, ref_i) and torch.equal(s, ref_s), precs[t]
    ix.close()
