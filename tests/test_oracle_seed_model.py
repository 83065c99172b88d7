"""Pins of the oracle's float64 seed-model and HN-layer pieces: closed forms
of GELU, softmax cross-entropy and the first Adam step, and central finite
differences for every backward pass."""
import math

import numpy as np
import pytest


def _params(rng, scale=0.2):
    shapes = [(256, 128), (256,), (256, 256), (256,), (512, 256), (512,)]
    return [rng.standard_normal(s) * scale for s in shapes]


def test_gelu_closed_form(orc):
    # Phi(1) = 0.5 (1 + erf(1/sqrt 2)); erf(1/sqrt2) = 0.6826894921370859
    phi1 = 0.8413447460685429
    assert orc.gelu(np.array([0.0]))[0] == 0.0
    assert abs(orc.gelu(np.array([1.0]))[0] - phi1) < 1e-15
    assert abs(orc.gelu(np.array([-1.0]))[0] + (1 - phi1)) < 1e-15
    # large |x|: GELU -> x for x >> 0 and -> 0 for x << 0
    assert abs(orc.gelu(np.array([12.0]))[0] - 12.0) < 1e-12
    assert abs(orc.gelu(np.array([-12.0]))[0]) < 1e-12
    # derivative at 0 is 1/2
    assert abs(orc.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-16


def test_gelu_grad_finite_difference(orc):
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (orc.gelu(x + h) - orc.gelu(x - h)) / (2 * h)
    assert np.abs(fd - orc.gelu_grad(x)).max() < 1e-8


def test_softmax_ce_closed_form(orc):
    z = np.zeros((3, 512))
    loss, g = orc.softmax_ce(z, np.array([0, 7, 511]))
    assert abs(loss - math.log(512)) < 1e-13
    # gradient (p - onehot)/B sums to zero per row
    assert np.abs(g.sum(1)).max() < 1e-15
    assert abs(g[1, 7] - (1 / 512 - 1) / 3) < 1e-16
    # shift invariance
    l2, g2 = orc.softmax_ce(z + 3.0, np.array([0, 7, 511]))
    assert abs(l2 - loss) < 1e-13 and np.abs(g2 - g).max() < 1e-16


def test_mlp_backward_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    params = _params(rng)
    x = rng.standard_normal((5, 128))
    y = rng.integers(0, 512, 5)

    def loss_of(ps):
        lg, _ = orc.mlp_forward(ps, x)
        return orc.softmax_ce(lg, y)[0]

    logits, cache = orc.mlp_forward(params, x)
    _, dl = orc.softmax_ce(logits, y)
    grads = orc.mlp_backward(params, cache, dl)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        assert g.shape == p.shape
        flat = p.reshape(-1)
        for t in rng.choice(flat.size, 6, replace=False):
            old = flat[t]
            flat[t] = old + h
            lp = loss_of(params)
            flat[t] = old - h
            lm = loss_of(params)
            flat[t] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g.reshape(-1)[t]) < 1e-7 + 1e-5 * abs(fd), (pi, t)


def test_adam_first_step_is_signed_lr(orc):
    # at t = 1 the bias-corrected m/sqrt(v) equals g/|g|, so each weight moves
    # by lr * sign(g) (up to eps)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(100)
    g = rng.standard_normal(100)
    w1, m, v = orc.adamw_step(w, g, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    assert np.allclose(w - w1, 1e-3 * np.sign(g), atol=1e-10)
    # decoupled weight decay adds lr*wd*w
    w2, _, _ = orc.adamw_step(w, g, np.zeros(100), np.zeros(100), 1, lr=1e-3, wd=0.1)
    assert np.allclose(w1 - w2, 1e-3 * 0.1 * w, atol=1e-15)


def test_top4_ties_to_smaller_index(orc):
    z = np.array([[1.0, 3.0, 3.0, 0.5, 3.0, 2.0, 3.0]])
    assert orc.top4(z)[0].tolist() == [1, 2, 4, 6]
    z2 = np.array([[0.0, 5.0, 1.0, 4.0, 3.0, 2.0]])
    assert orc.top4(z2)[0].tolist() == [1, 3, 4, 5]


@pytest.mark.parametrize("k,alpha", [(16, 1 / 8), (8, 1 / 32), (16, 0.0)])
def test_hn_backward_matches_finite_differences(orc, k, alpha):
    rng = np.random.default_rng(4)
    f = rng.standard_normal((3, 128))
    g = rng.standard_normal((3, 128))
    got = orc.hn_backward(f, g, k, alpha)
    h = 1e-6
    for r in range(3):
        for j in rng.choice(128, 10, replace=False):
            fp = f.copy()
            fp[r, j] += h
            fm = f.copy()
            fm[r, j] -= h
            fd = ((orc.hn_normalize(fp, k, alpha) - orc.hn_normalize(fm, k, alpha))[r] @ g[r]) / (2 * h)
            assert abs(fd - got[r, j]) < 1e-7
    # scale invariance of Eq. 1: the gradient is orthogonal to each block
    assert abs((got[:, :k] * f[:, :k]).sum()) < 1e-12
    assert abs((got[:, k:] * f[:, k:]).sum()) < 1e-12
    if alpha == 0.0:
        assert (got[:, k:] == 0).all()


def _dyadic_net():
    """A sparse network whose every pre-activation is a dyadic number of
    magnitude >= 16 or exactly 0, so every product and sum is exact in
    float64 and GELU is exact too: erf(z / sqrt 2) rounds to +-1 for
    |z| >= 16, so GELU(z) = z for z >= 16 and 0 for z <= -16.
      x[j]      = 1 + j/128
      W1[u, :]  = one entry: column u mod 128 (u < 128) or (5u) mod 128
                  (u >= 128), value 16, or -16 when u mod 16 == 7
      b1[u]     = 16 (u mod 3)   (same sign as the weight)
      W2[v, :]  = 1 at column (3v + 1) mod 256, 1/2 at (7v + 2) mod 256, or
                  -1 / -1/2 when v mod 32 == 5; b2[v] = +-16 with that sign
      W3[o, :]  = 1 at column (5o + 3) mod 256, -1/4 at (11o + 7) mod 256;
                  b3[o] = o / 64
    W2 is not symmetric, so a transposed square layer changes the logits."""
    W1 = np.zeros((256, 128))
    b1 = np.zeros(256)
    for u in range(256):
        col = u % 128 if u < 128 else (5 * u) % 128
        sgn = -1.0 if u % 16 == 7 else 1.0
        W1[u, col] = 16.0 * sgn
        b1[u] = 16.0 * (u % 3) * sgn
    W2 = np.zeros((256, 256))
    b2 = np.zeros(256)
    for v in range(256):
        sgn = -1.0 if v % 32 == 5 else 1.0
        W2[v, (3 * v + 1) % 256] += 1.0 * sgn
        W2[v, (7 * v + 2) % 256] += 0.5 * sgn
        b2[v] = 16.0 * sgn
    W3 = np.zeros((512, 256))
    b3 = np.zeros(512)
    for o in range(512):
        W3[o, (5 * o + 3) % 256] += 1.0
        W3[o, (11 * o + 7) % 256] += -0.25
        b3[o] = o / 64.0
    x = np.array([[1.0 + j / 128.0 for j in range(128)]])
    return [W1, b1, W2, b2, W3, b3], x


def _hand_logits():
    """The same network evaluated entry by entry from its description, with
    exact fractions and GELU taken as its two saturated branches."""
    from fractions import Fraction as F
    x = [F(1) + F(j, 128) for j in range(128)]

    def act(z):
        assert z == 0 or abs(z) >= 16
        return z if z > 0 else F(0)

    h1 = []
    for u in range(256):
        col = u % 128 if u < 128 else (5 * u) % 128
        sgn = -1 if u % 16 == 7 else 1
        h1.append(act(16 * sgn * x[col] + 16 * (u % 3) * sgn))
    h2 = []
    for v in range(256):
        sgn = -1 if v % 32 == 5 else 1
        a, b = (3 * v + 1) % 256, (7 * v + 2) % 256
        z = sgn * (h1[a] + F(1, 2) * h1[b]) + 16 * sgn
        h2.append(act(z))
    out = []
    for o in range(512):
        a, b = (5 * o + 3) % 256, (11 * o + 7) % 256
        out.append(h2[a] - F(1, 4) * h2[b] + F(o, 64))
    return out


def test_mlp_forward_dyadic_network_exact(orc):
    """The forward composition (128 -> 256 -> 256 -> 512, GELU after the two
    hidden layers, biases added before the activation, weights output-major)
    equals a hand evaluation of an exactly representable network.  A
    transposed W2, a missing bias or GELU on the output layer changes logits
    by whole units."""
    params, x = _dyadic_net()
    logits, _ = orc.mlp_forward(params, x)
    want = _hand_logits()
    assert logits.shape == (1, 512)
    for o in range(512):
        assert logits[0, o] == float(want[o]), o
    # the pin separates the two orientations of the square layer
    alt = list(params)
    alt[2] = params[2].T.copy()
    bad, _ = orc.mlp_forward(alt, x)
    assert np.abs(bad - logits).max() >= 1.0
