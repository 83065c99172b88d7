"""GPU parity of the learned seed (seed model, anchors, labels, single-pass
search forms) against the CPU float64 oracle, through the C ABI.

Tolerances of the seed model (float32 MFMA accumulation, float32 exact-erf
GELU, weights rounded to bf16 on both sides): every dot product sums at most
max(256, b) float32 products, so its rounding is below ~2^-24 * 256 of the sum
of magnitudes; the tests allow 1e-4 relative to the largest magnitude of each
tensor (max-norm) and 1e-4 relative in Frobenius norm, two orders above the
expected error and far below what a dropped term, transposed operand or wrong
index gives (O(1)).  Integer outputs (anchors, labels, indices) are bit-exact.
"""
import numpy as np
import pytest

import hn_inputs
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-4
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


SHAPES = [(256, 128), (256,), (256, 256), (256,), (512, 256), (512,)]


def split(p):
    out, o = [], 0
    for sh in SHAPES:
        n = int(np.prod(sh))
        out.append(np.asarray(p[o:o + n], dtype=np.float64).reshape(sh))
        o += n
    assert o == len(p)
    return out


def bf16_weights(p):
    """The oracle's parameters with the weights rounded to bf16 (torch's CPU
    round-to-nearest-even cast) and the biases as given."""
    import torch
    parts = split(p)
    for i in (0, 2, 4):
        parts[i] = torch.from_numpy(parts[i].astype(np.float32)).to(torch.bfloat16).double().numpy()
    return parts


def close(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(np.abs(ref).max(), 1e-30)
    assert np.abs(got - ref).max() <= REL * scale, "%s: max |d| %g vs scale %g" % (
        what, np.abs(got - ref).max(), scale)
    assert np.linalg.norm(got - ref) <= REL * max(np.linalg.norm(ref), 1e-30), what


# ------------------------------------------------------------ seed model

@pytest.mark.parametrize("b", [1, 37, 200])
def test_mlp_forward_matches_oracle(hn, b):
    p = hn_inputs.mlp_init(11 + b)
    x = hn_inputs.make_queries(hn_inputs.make_db(500, 16, 1 / 8, 5, 12), 16, 1 / 8, b, 0, 13)
    say("mlp forward b=%d" % b)
    got = hn.mlp_forward(dev(p), dev(x)).cpu().numpy()
    ref, _ = oracle.mlp_forward(bf16_weights(p), x)
    close(got, ref, "logits")


@pytest.mark.parametrize("b", [1, 100, 333])
def test_mlp_grad_matches_oracle(hn, b):
    p = hn_inputs.mlp_init(21 + b)
    x = hn_inputs.make_queries(hn_inputs.make_db(700, 16, 1 / 8, 5, 22), 16, 1 / 8, b, 0, 23)
    labels = np.random.Generator(np.random.PCG64(24 + b)).integers(0, 512, size=b)
    say("mlp grad b=%d" % b)
    g, loss = hn.mlp_grad(dev(p), dev(x), dev(labels.astype(np.int32)))
    g = g.cpu().numpy()
    params = bf16_weights(p)
    logits, cache = oracle.mlp_forward(params, x)
    ref_loss, dlog = oracle.softmax_ce(logits, labels)
    refs = oracle.mlp_backward(params, cache, dlog)
    gs = split(g)
    for name, a, r in zip(("dW1", "db1", "dW2", "db2", "dW3", "db3"), gs, refs):
        close(a, r, name)
    assert abs(float(loss.cpu()[0]) - ref_loss) <= REL * max(1.0, abs(ref_loss))


def test_mlp_bad_label_gives_nan_loss(hn):
    p = hn_inputs.mlp_init(3)
    x = hn_inputs.make_queries(hn_inputs.make_db(100, 16, 1 / 8, 2, 4), 16, 1 / 8, 4, 0, 5)
    say("mlp grad with an out-of-range label")
    _, loss = hn.mlp_grad(dev(p), dev(x), dev(np.array([1, 2, 512, 3], dtype=np.int32)))
    assert np.isnan(float(loss.cpu()[0]))


def test_adamw_matches_oracle(hn):
    import torch
    rng = np.random.Generator(np.random.PCG64(31))
    n = 5003
    w = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n)
    v = np.zeros(n)
    dw, dm, dv = dev(w), torch.zeros(n, device="cuda:0"), torch.zeros(n, device="cuda:0")
    wr = w.astype(np.float64)
    for t in (1, 2, 3):
        g = rng.normal(size=n).astype(np.float32)
        say("adamw step %d" % t)
        hn.mlp_adamw(dw, dev(g), dm, dv, t, lr=1e-2, weight_decay=0.01)
        wr, m, v = oracle.adamw_step(wr, g.astype(np.float64), m, v, t, 1e-2, wd=0.01)
        close(dw.cpu().numpy(), wr, "w step %d" % t)
        close(dm.cpu().numpy(), m, "m step %d" % t)
        close(dv.cpu().numpy(), v, "v step %d" % t)


def test_seed_train_equals_manual_steps_and_learns(hn):
    """hn_seed_train = the same grad + AdamW steps in order (bit-identical),
    and the loss falls on a learnable task."""
    import torch
    db = hn_inputs.make_db(2000, 16, 1 / 8, 16, 41)
    x = hn_inputs.make_queries(db, 16, 1 / 8, 300, 0, 42)
    # labels: the cluster-ish structure of the first 8 coordinates' signs
    labels = np.packbits(x[:, :8] > 0, axis=1)[:, 0].astype(np.int32)
    p0 = hn_inputs.mlp_init(43)
    pa = dev(p0)
    say("seed_train 3 epochs, batch 64")
    losses = hn.seed_train(pa, dev(x), dev(labels), batch=64, epochs=3, lr=3e-3).cpu().numpy()
    pb = dev(p0)
    m = torch.zeros_like(pb)
    v = torch.zeros_like(pb)
    t = 0
    manual = []
    for ep in range(3):
        for s in range(0, 300, 64):
            g, loss = hn.mlp_grad(pb, dev(x[s:s + 64]), dev(labels[s:s + 64]))
            t += 1
            hn.mlp_adamw(pb, g, m, v, t, lr=3e-3)
            manual.append(float(loss.cpu()[0]))
    assert torch.equal(pa, pb)
    assert np.array_equal(losses, np.array(manual, dtype=np.float32))
    assert losses[-5:].mean() < 0.8 * losses[:5].mean()


# ------------------------------------------------------------ anchors, labels

@pytest.mark.parametrize("n,n_anchor", [(1, 3), (300, 17), (3001, 64), (5000, 512)])
def test_kmeanspp_matches_oracle(hn, n, n_anchor):
    db = hn_inputs.make_db(n, 16, 1 / 8, max(1, n // 50), 50 + n)
    u = hn_inputs.uniform_draws(n_anchor, 51 + n)
    say("kmeans++ n=%d anchors=%d" % (n, n_anchor))
    ix = hn.Index(dev(db), 16, 1 / 8)
    got = ix.kmeanspp(n_anchor, dev(u)).cpu().numpy()
    ref = oracle.kmeanspp(db, n_anchor, u)
    assert np.array_equal(got, ref), np.nonzero(got != ref)[0][:5]
    ix.close()


def test_kmeanspp_all_duplicates(hn):
    # float32 rows: sim(x, x) is 1 only up to rounding, so D > 0 can remain
    row = hn_inputs.make_db(1, 8, 1 / 32, 1, 60)
    db = np.tile(row, (700, 1))
    u = hn_inputs.uniform_draws(6, 61)
    say("kmeans++ on 700 identical rows")
    ix = hn.Index(dev(db), 8, 1 / 32)
    got = ix.kmeanspp(6, dev(u)).cpu().numpy()
    assert np.array_equal(got, oracle.kmeanspp(db, 6, u))
    ix.close()
    # exact unit rows (alpha = 0): D = 0 everywhere, zero total weight, every
    # later pick is the last entry
    db = np.zeros((700, 128), dtype=np.float32)
    db[:, 0] = 1.0
    say("kmeans++ on 700 identical unit rows")
    ix = hn.Index(dev(db), 8, 0.0)
    got = ix.kmeanspp(6, dev(u)).cpu().numpy()
    assert np.array_equal(got, oracle.kmeanspp(db, 6, u))
    assert (got[1:] == 699).all()
    ix.close()


def test_seed_labels_match_oracle(hn):
    db = hn_inputs.make_db(4000, 16, 1 / 8, 40, 70)
    qs = hn_inputs.make_queries(db, 16, 1 / 8, 150, 30, 71)
    anchors = oracle.kmeanspp(db, 64, hn_inputs.uniform_draws(64, 72))
    say("seed labels q=180 anchors=64")
    ix = hn.Index(dev(db), 16, 1 / 8)
    got = ix.seed_labels(dev(anchors), dev(qs)).cpu().numpy()
    nn, _ = oracle.bruteforce_top1(db, qs)
    for i in range(len(qs)):
        sims = [oracle.sim(db[nn[i]], db[a]) for a in anchors]
        best = max(range(len(anchors)), key=lambda a: (sims[a], -a))
        assert got[i] == best, i
    bad = dev(np.array([0, 4000], dtype=np.int64))
    with pytest.raises(hn.HNError):
        ix.seed_labels(bad, dev(qs[:2]))
    with pytest.raises(ValueError):
        ix.set_seed_model(dev(hn_inputs.mlp_init(1)), dev(anchors))  # 64 != 512 anchors
    with pytest.raises(hn.HNError):
        ix.search(dev(qs[:3]), seed="learned")  # no model installed
    ix.close()


# ------------------------------------------------------------ single-pass forms

def _trained_index(hn, db, k, alpha, qs_train, steps_epochs=4):
    ix = hn.Index(dev(db), k, alpha)
    anchors = ix.kmeanspp(512, dev(hn_inputs.uniform_draws(512, 80)))
    labels = ix.seed_labels(anchors, dev(qs_train))
    params = dev(hn_inputs.mlp_init(81))
    losses = hn.seed_train(params, dev(qs_train), labels, batch=256, epochs=steps_epochs,
                           lr=2e-3).cpu().numpy()
    ix.set_seed_model(params, anchors)
    return ix, anchors, params, losses


def test_single_pass_forms_exact(hn):
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    qs_train = hn_inputs.make_queries(db, w.k, w.alpha, 3000, 0, 90)
    say("train the seed model on workload 1 (3000 queries)")
    ix, anchors, params, losses = _trained_index(hn, db, w.k, w.alpha, qs_train)
    assert losses[-3:].mean() < losses[:3].mean()
    ref = oracle.bnb_top1(db, qs, w.k, w.alpha)
    surv = {}
    for seed in ("learned", "window"):
        for prec in ("fp32", "bf16", "fp8", "int8"):
            say("single pass seed=%s precision=%s" % (seed, prec))
            idx, sim, aux, st = ix.search(dev(qs), precision=prec, seed=seed, aux=True,
                                          stats=True)
            idx, sim = idx.cpu().numpy(), sim.cpu().numpy()
            assert (idx == ref["idx"]).all(), (seed, prec)
            assert (np.abs(sim - ref["sim"]) <= SIM_TOL).all()
            assert st["overflow_queries"] == 0
            surv[(seed, prec)] = aux["survivors"].cpu().numpy()
            if seed == "learned":
                si = aux["seed_idx"].cpu().numpy()
                ss = aux["seed_sim"].cpu().numpy()
                assert np.isin(si, anchors.cpu().numpy()).all()
                for qi in range(0, len(qs), 9):
                    assert ss[qi] == oracle.sim(qs[qi], db[si[qi]])
    # the seed only raises the window's floor: never more survivors
    for prec in ("fp32", "bf16", "fp8", "int8"):
        assert (surv[("learned", prec)] <= surv[("window", prec)]).all()
    ix.close()


@pytest.mark.parametrize("frac", [0.5, 0.0])
def test_single_pass_soft_mode_returns_real_entries(hn, frac):
    """The window-only single pass with beta < alpha (Section 7's soft mode):
    the result is a real entry with its canonical sim, never better than the
    exact best, and its re-filter threshold (raised to the bound at the sim
    of the entry that scored the final maximum, capped at that maximum)
    leaves the pass's own maximum rescored: every query gets an entry."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)[:96]
    ix = hn.Index(dev(db), w.k, w.alpha)
    ref = oracle.bnb_top1(db, qs, w.k, w.alpha)
    beta = frac * w.alpha
    for prec in ("fp32", "bf16"):
        say("window single pass, soft mode beta=%g, %s" % (beta, prec))
        idx, sim = ix.search(dev(qs), precision=prec, seed="window", beta=beta)
        idx, sim = idx.cpu().numpy(), sim.cpu().numpy()
        assert (idx >= 0).all() and (idx < len(db)).all()
        assert (sim <= ref["sim"]).all()
        for qi in range(len(qs)):
            assert sim[qi] == oracle.sim(qs[qi], db[idx[qi]])
    ix.close()


def test_learned_seed_top4_rescoring(hn):
    """The learned L is the best canonical sim among the anchors of the 4
    largest logits; checked on queries whose top-4 set is unambiguous under
    the oracle's float64 logits (margin to the 5th above the forward's
    tolerance); elsewhere L must be the sim of one of the top-5 anchors."""
    db = hn_inputs.make_db(6000, 16, 1 / 8, 60, 100)
    qs_train = hn_inputs.make_queries(db, 16, 1 / 8, 1500, 0, 101)
    qs = hn_inputs.make_queries(db, 16, 1 / 8, 90, 10, 102)
    say("learned seed top-4 on n=6000")
    ix, anchors, params, _ = _trained_index(hn, db, 16, 1 / 8, qs_train, 2)
    _, _, aux = ix.search(dev(qs), seed="learned", aux=True)
    ss = aux["seed_sim"].cpu().numpy()
    logits, _ = oracle.mlp_forward(bf16_weights(params.cpu().numpy()), qs)
    an = anchors.cpu().numpy()
    order = np.argsort(-logits, axis=1, kind="stable")
    checked = 0
    for i in range(len(qs)):
        z = logits[i]
        margin = z[order[i, 3]] - z[order[i, 4]]
        cands = [oracle.sim(qs[i], db[an[a]]) for a in order[i, :5]]
        if margin > 1e-3 * max(1.0, np.abs(z).max()):
            assert ss[i] == max(cands[:4]), i
            checked += 1
        else:
            assert ss[i] in cands
    assert checked >= len(qs) // 2
    ix.close()


def test_trained_seed_gains_over_untrained(hn):
    """What training buys: the trained model's seed bound is tighter than an
    untrained model's (same anchors) and the single pass keeps fewer
    survivors; both stay exact."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    qs_train = hn_inputs.make_queries(db, w.k, w.alpha, 4000, 0, 110)
    say("trained vs untrained seed model, workload 1")
    ix, anchors, params, _ = _trained_index(hn, db, w.k, w.alpha, qs_train, 6)
    idx_t, _, aux_t = ix.search(dev(qs), seed="learned", aux=True)
    ix.set_seed_model(dev(hn_inputs.mlp_init(81)), anchors)  # the untrained start
    idx_u, _, aux_u = ix.search(dev(qs), seed="learned", aux=True)
    assert (idx_t.cpu() == idx_u.cpu()).all()
    L_t = aux_t["seed_sim"].cpu().numpy().mean()
    L_u = aux_u["seed_sim"].cpu().numpy().mean()
    s_t = aux_t["survivors"].cpu().numpy().astype(np.float64).mean()
    s_u = aux_u["survivors"].cpu().numpy().astype(np.float64).mean()
    say("mean L trained %.4f untrained %.4f; survivors %.1f vs %.1f" % (L_t, L_u, s_t, s_u))
    assert L_t > L_u
    assert s_t < s_u
    ix.close()


def test_single_pass_overflow_rerun_exact(hn):
    """A pair list far too small for the window: the overflowing queries are
    finished by a filter pass seeded with the best candidate they reached."""
    w = hn_inputs.workload(1)
    db = w.db()
    qs = w.queries(db)
    ix = hn.Index(dev(db), w.k, w.alpha)
    ref = oracle.bnb_top1(db, qs, w.k, w.alpha)
    for prec in ("fp32", "bf16"):
        say("window form with survivor_cap=3000, precision=%s" % prec)
        idx, sim, st = ix.search(dev(qs), precision=prec, seed="window", survivor_cap=3000,
                                 stats=True)
        assert st["overflow_queries"] > 0
        assert (idx.cpu().numpy() == ref["idx"]).all()
        assert (np.abs(sim.cpu().numpy() - ref["sim"]) <= SIM_TOL).all()
    ix.close()
