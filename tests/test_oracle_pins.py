"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rational arithmetic, closed forms, theorems used as invariants, special cases
and the paper's printed figures.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import hn_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U53 = 2.0 ** -53


def gamma(n, u):
    return n * u / (1 - n * u)


def exact_dot(q, x, lo=0, hi=None):
    hi = len(q) if hi is None else hi
    return sum((Fraction(float(q[j])) * Fraction(float(x[j])) for j in range(lo, hi)), Fraction(0))


def tiny_hn(n, nq, k, alpha, seed, clusters=4):
    db = hn_inputs.make_db(n, k, alpha, clusters, seed)
    qs = hn_inputs.make_queries(db, k, alpha, nq - nq // 3, nq // 3, seed + 1)
    return db, qs


# ------------------------------------------------------------ canonical sim

def test_sim_is_the_ascending_float64_sum(orc):
    # 2^60 + 1 rounds back to 2^60 in float64, so the order of the additions
    # decides the result: ascending sequential gives 1, a pairwise or reversed
    # order gives 0, and the exact value is 2.
    big = 2.0 ** 60
    q = np.ones(4, dtype=np.float32)
    x = np.array([big, 1.0, -big, 1.0], dtype=np.float32)
    assert orc.sim(q, x) == 1.0
    x2 = np.array([big, -big, 1.0, 1.0], dtype=np.float32)
    assert orc.sim(q, x2) == 2.0


def test_sim_within_float64_error_bound_of_exact(orc):
    rng = np.random.default_rng(11)
    for _ in range(50):
        q = rng.standard_normal(128).astype(np.float32)
        x = rng.standard_normal(128).astype(np.float32)
        ex = exact_dot(q, x)
        absum = sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(q, x))
        err = abs(Fraction(orc.sim(q, x)) - ex)
        assert err <= Fraction(gamma(128, U53)) * absum


# ------------------------------------------------------------ HN layer, Eq. 1

@pytest.mark.parametrize("k,alpha", [(8, 1 / 32), (16, 1 / 8), (16, 0.0), (1, 0.25), (127, 0.5)])
def test_block_norms_closed_form(orc, k, alpha):
    rng = np.random.default_rng(3)
    f = rng.standard_normal((20, 128)) * rng.uniform(0.1, 10.0, (20, 1))
    y = orc.hn_normalize(f, k, alpha)
    nM = np.sqrt((y[:, :k] ** 2).sum(1))
    nm = np.sqrt((y[:, k:] ** 2).sum(1))
    assert np.allclose(nM, math.sqrt(1 - alpha), rtol=0, atol=4e-16)
    assert np.allclose(nm, math.sqrt(alpha), rtol=0, atol=4e-16)
    assert np.allclose(np.sqrt((y ** 2).sum(1)), 1.0, rtol=0, atol=4e-16)
    if alpha == 0.0:
        assert (y[:, k:] == 0.0).all()
    # direction of each block is kept
    cos = (y[:, :k] * f[:, :k]).sum(1) / (nM * np.sqrt((f[:, :k] ** 2).sum(1)))
    assert np.allclose(cos, 1.0, atol=1e-14)


def test_generator_rows_are_hn_normalised():
    for k, alpha in [(8, 1 / 32), (16, 1 / 8), (16, 0.0)]:
        db = hn_inputs.make_db(3000, k, alpha, 12, 5)
        x = db.astype(np.float64)
        nM = np.sqrt((x[:, :k] ** 2).sum(1))
        nm = np.sqrt((x[:, k:] ** 2).sum(1))
        # float32 storage of a float64-normalised block: relative drift at
        # most about sqrt(dim) half-ulps
        assert np.abs(nM / math.sqrt(1 - alpha) - 1).max() < 2.0 ** -20
        if alpha > 0:
            assert np.abs(nm / math.sqrt(alpha) - 1).max() < 2.0 ** -20
        else:
            assert (db[:, k:] == 0).all()


def test_db_max_norms_exact_integer_rows(orc):
    """Block-norm maxima on rows built from Pythagorean triples, so every norm
    is an exact integer and each maximum comes from a different row.  With
    k = 16: row 0 major (3, 4) = 5, minor 12, full 13; row 1 major (5, 12) =
    13, minor 0; row 2 major 8, minor 15, full 17; row 3 has 9 at j = 15 (the
    last major coordinate) and 40 at j = 16 (the first minor one): major 9,
    minor 40, full 41.  A block boundary off by one, or an inflated norm,
    changes a result."""
    k = 16
    db = np.zeros((4, 128), dtype=np.float32)
    db[0, 0], db[0, 1], db[0, 16] = 3, 4, 12
    db[1, 2], db[1, 3] = 5, 12
    db[2, 5], db[2, 100] = 8, 15
    db[3, 15], db[3, 16] = 9, 40
    assert orc.db_max_norms(db, k) == (13.0, 40.0, 41.0)
    # the same rows split at k = 15 and 17 move row 3's coordinates
    assert orc.db_max_norms(db, 15) == (13.0, 41.0, 41.0)
    assert orc.db_max_norms(db, 17) == (41.0, 15.0, 41.0)


@pytest.mark.parametrize("k,alpha", [(8, 1 / 32), (16, 1 / 8), (16, 0.0), (64, 0.5)])
def test_db_max_norms_closed_form_on_hn_rows(orc, k, alpha):
    """On HN rows the maxima are the closed forms of Eq. 1: sqrt(1 - alpha),
    sqrt(alpha) and 1, up to the float32 storage of the rows (a relative
    2^-20), from above and from below."""
    db = hn_inputs.make_db(2000, k, alpha, 16, 4242 + k)
    mM, mm, mf = orc.db_max_norms(db, k)
    tol = 2.0 ** -20
    for got, want in ((mM, math.sqrt(1 - alpha)), (mm, math.sqrt(alpha)), (mf, 1.0)):
        if want == 0.0:
            assert got == 0.0
        else:
            assert abs(got / want - 1.0) <= tol, (got, want)


# --------------------------------------------------------- bound, Eq. 3

@pytest.mark.parametrize("k,alpha", [(8, 1 / 32), (16, 1 / 8), (4, 1 / 4)])
def test_bound_admissible_on_every_pair_exact(orc, k, alpha):
    """Eq. 3 via Cauchy-Schwarz, checked exactly on every (query, entry) pair
    of a tiny input: the minor product never exceeds ||q_m|| ||x_m||, and the
    oracle's widened float64 bound never falls below the float64 sim."""
    db, qs = tiny_hn(14, 9, k, alpha, seed=100 + k)
    mu = orc.db_max_norms(db, k)
    for q in qs:
        slack = orc.lib().or_bnb_slack(np.ascontiguousarray(q), 128, k, alpha, *mu)
        qm2 = exact_dot(q, q, k, 128)
        for x in db:
            minor = exact_dot(q, x, k, 128)
            xm2 = exact_dot(x, x, k, 128)
            assert minor <= 0 or minor * minor <= qm2 * xm2
            s64 = orc.sim(q[:k], x[:k])
            assert orc.sim(q, x) <= s64 + alpha + slack
            # with exact reals the bound is sqrt(alpha)^2 up to float32 storage
            assert float(minor) <= alpha * (1 + 2.0 ** -20)


def test_bound_tight_when_minors_identical(orc):
    k, alpha = 16, 1 / 8
    db, qs = tiny_hn(6, 6, k, alpha, seed=7)
    for q in qs:
        x = q.copy()
        x[:k] = db[0, :k]  # any major, identical minor
        gap = orc.sim(q, x) - orc.sim(q[:k], x[:k])
        assert abs(gap - alpha) < 1e-6


# ----------------------------------------------------------- top-1

def test_bruteforce_matches_exact_rational_argmax(orc):
    db, qs = tiny_hn(40, 12, 8, 1 / 32, seed=21)
    idx, sv = orc.bruteforce_top1(db, qs, threads=2)
    for qi, q in enumerate(qs):
        ex = [exact_dot(q, x) for x in db]
        m = max(ex)
        i_star = ex.index(m)
        second = max(v for i, v in enumerate(ex) if i != i_star)
        if m - second > Fraction(1, 10 ** 12):
            assert idx[qi] == i_star
        assert abs(Fraction(sv[qi]) - ex[idx[qi]]) < Fraction(1, 10 ** 13)


def test_bruteforce_ties_go_to_smallest_index(orc):
    db, qs = tiny_hn(60, 10, 16, 1 / 8, seed=31)
    idx0, _ = orc.bruteforce_top1(db, qs)
    db2 = db.copy()
    for qi in range(len(qs)):
        b = idx0[qi]
        # copies of the best row placed after it must never win
        for pos in range(b + 1, min(b + 4, len(db2))):
            db2[pos] = db[b]
    idx2, sv2 = orc.bruteforce_top1(db2, qs)
    for qi in range(len(qs)):
        sims = [orc.sim(qs[qi], x) for x in db2]
        assert sv2[qi] == max(sims)
        assert idx2[qi] == sims.index(max(sims))  # first occurrence


def test_tie_rule_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "tie_rule.json")))
    db = np.array(g["db"], dtype=np.float32)
    q = np.array([g["query"]], dtype=np.float32)
    r = orc.bnb_top1(db, q, g["k"], g["alpha"])
    assert r["seed_idx"][0] == g["expected_seed"]
    assert r["idx"][0] == g["expected_idx"]
    assert r["sim"][0] == g["expected_sim"]
    bi, bs = orc.bruteforce_top1(db, q)
    assert bi[0] == g["expected_idx"] and bs[0] == g["expected_sim"]


# ------------------------------------------------- Theorem 1 (exactness)

def _cases():
    rng = np.random.default_rng(2024)
    out = []
    for t in range(120):
        n = int(rng.choice([1, 2, 3, 17, 64, 300, 1000]))
        k = int(rng.choice([1, 4, 8, 16, 32, 127]))
        alpha = float(rng.choice([0.0, 1 / 32, 1 / 8, 1 / 4, 0.9]))
        out.append((t, n, k, alpha))
    return out


def test_bnb_equals_bruteforce_seeded(orc):
    """Theorem 1: index and sim of Algorithm 1 equal exhaustive search."""
    for t, n, k, alpha in _cases():
        clusters = max(1, n // 16)
        db = hn_inputs.make_db(n, k, alpha, clusters, 9000 + t)
        qs = hn_inputs.make_queries(db, k, alpha, 6, 3, 9500 + t)
        # duplicate rows to create exact ties
        if n >= 4:
            db[n - 1] = db[0]
            db[n // 2] = db[1]
        bi, bs = orc.bruteforce_top1(db, qs, threads=3)
        r = orc.bnb_top1(db, qs, k, alpha, threads=3)
        assert (r["idx"] == bi).all(), (t, n, k, alpha)
        assert (r["sim"].view(np.int64) == bs.view(np.int64)).all()


def test_bnb_adversarial_equal_sim_smaller_index(orc):
    """An entry before the seed with the same full sim but a smaller major
    score (minor compensates) must win.  Built from dyadic values so that the
    sims tie exactly, inside a larger random database."""
    g = json.load(open(os.path.join(GOLDEN, "tie_rule.json")))
    rng = np.random.default_rng(5)
    base = np.array(g["db"], dtype=np.float32)
    filler = (rng.standard_normal((200, 4)) * 0.1).astype(np.float32)
    db = np.concatenate([filler[:50], base, filler[50:]])
    q = np.array([g["query"]], dtype=np.float32)
    r = orc.bnb_top1(db, q, g["k"], g["alpha"])
    bi, bs = orc.bruteforce_top1(db, q)
    assert r["idx"][0] == 50 and bi[0] == 50
    assert r["seed_idx"][0] == 51


def test_alpha0_needs_no_phase2(orc):
    """At alpha = 0 the minor block is exactly zero: the major score is the
    full sim and Phase 2 evaluates nothing beyond exact major-score ties
    (Table 3, alpha = 0 rows)."""
    g = json.load(open(os.path.join(GOLDEN, "alpha0.json")))
    for k in (8, 16):
        db = hn_inputs.make_db(4000, k, 0.0, 40, 77 + k)
        qs = hn_inputs.make_queries(db, k, 0.0, 30, 10, 78 + k)
        r = orc.bnb_top1(db, qs, k, 0.0)
        pct = 100.0 * r["phase2"].sum() / (len(qs) * len(db))
        # the float64 slack admits only entries within ~1e-14 of the best
        assert pct == g["phase2_percent"]
        assert (r["seed_idx"] == r["idx"]).all()


# -------------------------------------------- Theorem 2 (determinism)

def test_deterministic_across_thread_counts(orc):
    db, qs = tiny_hn(3000, 37, 16, 1 / 8, seed=404, clusters=20)
    ref = orc.bnb_top1(db, qs, 16, 1 / 8, threads=1)
    refb = orc.bruteforce_top1(db, qs, threads=1)
    for t in (2, 3, 5, 8, 16):
        r = orc.bnb_top1(db, qs, 16, 1 / 8, threads=t)
        for key in ref:
            assert ref[key].tobytes() == r[key].tobytes(), (t, key)
        b = orc.bruteforce_top1(db, qs, threads=t)
        assert b[0].tobytes() == refb[0].tobytes() and b[1].tobytes() == refb[1].tobytes()


# ------------------------------------------------------- survivor sets

def test_survivor_list_matches_exact_rational(orc):
    k, alpha = 8, 1 / 32
    db, qs = tiny_hn(80, 6, k, alpha, seed=55)
    for q in qs:
        sm = [exact_dot(q, x, 0, k) for x in db]
        L = float(max(sm)) + alpha - 0.05
        got = orc.survivor_list(db, q, k, alpha, L)
        want = [i for i, s in enumerate(sm) if s + Fraction(alpha) >= Fraction(L)]
        near = {i for i, s in enumerate(sm) if abs(s + Fraction(alpha) - Fraction(L)) < Fraction(1, 10 ** 12)}
        assert set(got) - near == set(want) - near
        assert list(got) == sorted(got)


def test_survivor_counts_consistent(orc):
    k, alpha = 16, 1 / 8
    db, qs = tiny_hn(2000, 20, k, alpha, seed=66, clusters=10)
    r = orc.bnb_top1(db, qs, k, alpha)
    L = r["seed_sim"] - r["slack"]
    lo, hi = orc.survivor_counts(db, qs, k, alpha, L, r["seed_sim"])
    for qi in range(len(qs)):
        assert lo[qi] == len(orc.survivor_list(db, qs[qi], k, alpha, L[qi]))
        assert hi[qi] <= lo[qi]
        # Algorithm 1 evaluates only entries whose widened bound reaches the
        # running best, which never falls below the seed's sim
        assert r["phase2"][qi] <= lo[qi] - 1
    a, _ = orc.survivor_counts(db, qs, k, alpha, np.full(len(qs), -np.inf), L)
    assert (a == len(db)).all()


# ----------------------------------------------------------- top-k

def test_topk_consistent_with_top1_and_exact(orc):
    db, qs = tiny_hn(50, 8, 8, 1 / 32, seed=88)
    db[10] = db[3]
    ti, ts = orc.topk(db, qs, 5)
    bi, bs = orc.bruteforce_top1(db, qs)
    assert (ti[:, 0] == bi).all() and (ts[:, 0] == bs).all()
    for qi, q in enumerate(qs):
        ex = [exact_dot(q, x) for x in db]
        order = sorted(range(len(db)), key=lambda i: (-ex[i], i))
        # exact ties (the duplicate) resolve by index in both orders
        assert list(ti[qi]) == order[:5]
    full_i, _ = orc.topk(db, qs[:1], len(db) + 3)
    assert sorted(full_i[0][: len(db)]) == list(range(len(db)))
    assert (full_i[0][len(db):] == -1).all()


# ----------------------------------------------------- k-means++ anchors

def test_kmeanspp_properties(orc):
    db = hn_inputs.make_db(500, 16, 1 / 8, 8, 12)
    u = hn_inputs.uniform_draws(32, 13)
    a = orc.kmeanspp(db, 32, u)
    assert a[0] == int(math.floor(u[0] * 500))
    assert len(set(a.tolist())) == 32
    assert (orc.kmeanspp(db, 32, u) == a).all()
    # a duplicate of a chosen anchor carries (almost) no weight and a single
    # far-away entry is then picked whatever the draw
    near = np.tile(db[:1], (6, 1))
    far = -db[:1]
    tiny = np.concatenate([near, far])
    for u1 in (0.05, 0.3, 0.999):
        got = orc.kmeanspp(tiny, 2, np.array([0.0, u1]))
        assert got[0] == 0 and got[1] == 6


def test_kmeanspp_inverse_cdf_closed_form(orc):
    # three entries: the first pick is entry 0; D^2 weights of the others are
    # 2 - 2 sim; entry 2 is orthogonal (weight 2), entry 1 opposite (weight 4)
    e = np.zeros((3, 4), dtype=np.float32)
    e[0, 0] = 1.0
    e[1, 0] = -1.0
    e[2, 1] = 1.0
    w = [0, 4 * 2 ** 30, 2 * 2 ** 30]
    total = sum(w)
    for u1, want in [(0.0, 1), (0.66, 1), (0.67, 2), (0.999, 2)]:
        got = orc.kmeanspp(e, 2, np.array([0.1, u1]))
        target = math.floor(u1 * total)
        assert got[1] == (1 if target < w[1] else 2) == want


def test_literal_bound_fails_on_self_pairs_but_widened_holds(orc):
    """With float32 storage ||x_m||^2 can exceed alpha by a few ulps, so the
    literal Eq. 3 test fails for q = x; the norm term of the oracle's slack
    (||q_m|| mu_m - alpha) restores admissibility."""
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(400, k, alpha, 8, 321)
    mu = orc.db_max_norms(db, k)
    over = 0
    for x in db:
        xm2 = exact_dot(x, x, k, 128)
        s64 = orc.sim(x[:k], x[:k])
        full = orc.sim(x, x)
        slack = orc.lib().or_bnb_slack(np.ascontiguousarray(x), 128, k, alpha, *mu)
        assert full <= s64 + alpha + slack
        if xm2 > Fraction(alpha) * (1 + Fraction(1, 2 ** 30)):
            over += 1
            assert full > s64 + alpha
    assert over > 0


# ------------------------------------------------ soft mode (Section 7)

def _soft_case():
    """Five entries (d = 4, k = 2) with dyadic values, so every dot product
    and bound below is exact.  Query q = (1, 0, 1/2, 0), ||q_m|| = 1/2.
      x0: major (3/8, 0),  minor (0, 1/2)  -> s = 3/8,  sim = 3/8
      x1: major (5/8, 0),  minor (0, 1/2)  -> s = 5/8,  sim = 5/8  (the seed b)
      x2: major (1/2, 0),  minor (1/2, 0)  -> s = 1/2,  sim = 3/4  (the NN)
      x3: major (0, 1),    minor (1/2, 0)  -> s = 0,    sim = 1/4
      x4: major (7/16, 0), minor (0, 1/2)  -> s = 7/16, sim = 7/16
    mu_m = 1/2, so ||q_m|| mu_m = alpha = 1/4 and the norm term of the slack
    is zero; what remains of the slack is below 1e-13."""
    db = np.array([[0.375, 0, 0, 0.5], [0.625, 0, 0, 0.5], [0.5, 0, 0.5, 0], [0, 1, 0.5, 0],
                   [0.4375, 0, 0, 0.5]], dtype=np.float32)
    q = np.array([[1, 0, 0.5, 0]], dtype=np.float32)
    return db, q


@pytest.mark.parametrize("beta,want_idx,want_phase2", [
    (None, 2, 2),
    (0.25, 2, 2),
    (0.125, 2, 1),
    (0.125 - 2.0 ** -20, 1, 0),
    (0.0, 1, 0),
])
def test_soft_mode_beta_exact_case(orc, beta, want_idx, want_phase2):
    """Section 7: replacing alpha by beta < alpha in the skip test prunes more
    and may lose the NN.  Worked by hand on the exact dyadic input above, in
    Algorithm 1's index order after the seed x1 (best = 5/8):
      beta = alpha = 1/4: x0's bound 3/8 + 1/4 = 5/8 is not strictly below the
        best, so x0 is evaluated; x2 (bound 3/4) is evaluated and lifts the
        best to 3/4; x3 (1/4) and x4 (11/16, above the seed's 5/8 but below
        the running best 3/4) are skipped: 2 evaluations, result x2;
      beta = 1/8: x0 (1/2) skipped, x2 (exactly 5/8) evaluated: 1, result x2;
      beta just below 1/8, or 0: x2's bound falls below 5/8 and nothing is
        evaluated: the soft mode returns the seed x1."""
    db, q = _soft_case()
    r = orc.bnb_top1(db, q, 2, 0.25, beta=beta, threads=1)
    assert r["seed_idx"][0] == 1 and r["seed_sim"][0] == 0.625
    assert r["idx"][0] == want_idx
    assert r["sim"][0] == (0.75 if want_idx == 2 else 0.625)
    assert r["phase2"][0] == want_phase2


@pytest.mark.parametrize("k,alpha", [(8, 1 / 32), (16, 1 / 8)])
def test_soft_mode_properties_exact(orc, k, alpha):
    """Properties of Algorithm 1 with beta in the skip test, checked with exact
    rational dots on small random HN inputs:
      * the result r is a real entry's sim, at least the seed's and at most the
        exact best;
      * every entry whose major dot plus beta reaches r (with a 2^-40 margin
        for the float64 scores) was compared, so none of them beats r: r is
        the best over {b} and {i : dot_K + beta >= r};
      * if the NN's minor dot is at most beta, the NN is found (the weakened
        bound is still admissible for it)."""
    db, qs = tiny_hn(60, 12, k, alpha, seed=700 + k, clusters=3)
    sims = [[exact_dot(q, x) for x in db] for q in qs]
    majs = [[exact_dot(q, x, 0, k) for x in db] for q in qs]
    for frac in (0.0, 0.25, 0.5, 0.75, 1.0):
        beta = frac * alpha
        r = orc.bnb_top1(db, qs, k, alpha, beta=beta, threads=2)
        for qi in range(len(qs)):
            i, v = int(r["idx"][qi]), r["sim"][qi]
            assert v == orc.sim(qs[qi], db[i])
            assert v >= r["seed_sim"][qi]
            best = max(range(len(db)), key=lambda j: (sims[qi][j], -j))
            assert Fraction(v) <= sims[qi][best] + Fraction(1, 10 ** 12)
            for j in range(len(db)):
                if majs[qi][j] + Fraction(beta) >= Fraction(v) + Fraction(2.0 ** -40):
                    assert sims[qi][j] <= Fraction(v) + Fraction(1, 10 ** 12), (frac, qi, j)
            if sims[qi][best] - majs[qi][best] <= Fraction(beta):
                assert i == best or abs(Fraction(v) - sims[qi][best]) < Fraction(1, 10 ** 12)
