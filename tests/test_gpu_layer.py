"""GPU parity of the HN layer (Eq. 1) and its vector-Jacobian product against
the CPU float64 oracle, through the C ABI.  The kernels compute in float64 and
round each output once to float32, so the forward matches the oracle to one
float32 rounding (2^-24 relative, plus the float64 summation-order difference
of the norms); the backward's cancellation (g - v (v . g)) makes its error
relative to the block's scale, bounded by 2^-21 of the row block's largest
gradient."""
import numpy as np
import pytest

import hn_inputs
import oracle

pytestmark = pytest.mark.gpu


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


CASES = [(1, 0.25), (8, 1 / 32), (16, 1 / 8), (16, 0.0), (63, 0.5), (127, 1 / 8)]


@pytest.mark.parametrize("k,alpha", CASES)
def test_layer_forward_matches_oracle(hn, k, alpha):
    rng = np.random.Generator(np.random.PCG64(900 + k))
    f = (rng.normal(size=(1001, 128)) * rng.uniform(0.1, 10, size=(1001, 1))).astype(np.float32)
    say("hn layer forward k=%d alpha=%g b=1001" % (k, alpha))
    y, st = hn.hn_layer(dev(f), k, alpha, status=True)
    y = y.cpu().numpy().astype(np.float64)
    ref = oracle.hn_normalize(f, k, alpha)
    assert (st.cpu().numpy() == 0).all()
    assert (np.abs(y - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-38).all(), np.abs(y - ref).max()
    # the output is a valid HN database for the index
    ix = hn.Index(dev(y.astype(np.float32)), k, alpha)
    ix.close()


@pytest.mark.parametrize("k,alpha", CASES)
def test_layer_backward_matches_oracle(hn, k, alpha):
    rng = np.random.Generator(np.random.PCG64(950 + k))
    f = rng.normal(size=(517, 128)).astype(np.float32)
    g = rng.normal(size=(517, 128)).astype(np.float32)
    say("hn layer backward k=%d alpha=%g b=517" % (k, alpha))
    got = hn.hn_layer_backward(dev(f), dev(g), k, alpha).cpu().numpy().astype(np.float64)
    ref = oracle.hn_backward(f, g, k, alpha)
    for lo, hi in ((0, k), (k, 128)):
        scale = np.abs(ref[:, lo:hi]).max(axis=1, keepdims=True)
        assert (np.abs(got[:, lo:hi] - ref[:, lo:hi]) <= 2.0 ** -21 * scale + 1e-38).all()


def test_layer_degenerate_rows(hn):
    f = np.random.Generator(np.random.PCG64(990)).normal(size=(6, 128)).astype(np.float32)
    f[1, :16] = 0.0          # zero major block
    f[2, 16:] = 0.0          # zero minor block (alpha > 0)
    f[3, 40] = np.nan        # non-finite
    f[4, 16:] = 0.0          # zero minor block at alpha = 0 is fine
    say("hn layer degenerate rows")
    y, st = hn.hn_layer(dev(f), 16, 1 / 8, status=True)
    y, st = y.cpu().numpy(), st.cpu().numpy()
    assert list(st[:4]) == [0, 1, 2, 3]
    assert (y[1, :16] == 0).all() and np.isfinite(y[1]).all()
    assert (y[2, 16:] == 0).all() and (y[3] == 0).all()
    y0, st0 = hn.hn_layer(dev(f[4:5]), 16, 0.0, status=True)
    assert int(st0.cpu()[0]) == 0 and (y0.cpu().numpy()[0, 16:] == 0).all()
    gz = hn.hn_layer_backward(dev(f), dev(np.ones_like(f)), 16, 1 / 8).cpu().numpy()
    assert (gz[1, :16] == 0).all() and (gz[2, 16:] == 0).all()
    with pytest.raises(ValueError):  # the binding checks the width
        hn.hn_layer(dev(f[:, :64]), 16, 1 / 8)
