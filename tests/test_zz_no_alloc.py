"""hn_search_top1_noalloc through the C ABI: the allocation-free variant of
hn_search_top1 (its scratch is one static device array per GPU) gives the same
results as hn_search_top1 and the oracle, on consecutive calls of decreasing
size (the array keeps the previous call's contents), allocates no device
memory, and rejects what does not fit or is not supported before enqueuing
any work."""
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


def _outs(q):
    import torch
    return (torch.empty(q, dtype=torch.int64, device="cuda:0"),
            torch.empty(q, dtype=torch.float64, device="cuda:0"))


def _same(a, b):
    import torch
    return bool(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_equals_search_on_consecutive_calls(hn, precision):
    import torch
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(50000, k, alpha, 200, 8800)
    qs = hn_inputs.make_queries(db, k, alpha, 900, 100, 8801)
    ix = hn.Index(dev(db), k, alpha)
    ref = oracle.bnb_top1(db, qs, k, alpha)
    for lo, hi in ((0, 1000), (200, 237), (999, 1000), (0, 513)):
        q = dev(qs[lo:hi])
        want = ix.search(q, precision=precision, aux=True)
        out = _outs(hi - lo)
        torch.cuda.synchronize()
        held = hn.memory_held()
        torch_held = torch.cuda.memory_allocated()
        say("noalloc %s: queries [%d, %d)" % (precision, lo, hi))
        got = ix.search_noalloc(q, precision=precision, out=out, aux=True)
        torch.cuda.synchronize()
        assert hn.memory_held() == held
        assert got[0].data_ptr() == out[0].data_ptr()
        assert _same(got[:2], want[:2])
        for name in ("seed_idx", "seed_sim", "threshold", "survivors", "slack"):
            assert torch.equal(got[2][name], want[2][name]), name
        gi, gs = got[0].cpu().numpy(), got[1].cpu().numpy()
        assert (gi == ref["idx"][lo:hi]).all()
        assert np.array_equal(gs.view(np.int64), ref["sim"][lo:hi].view(np.int64))
        del torch_held
    ix.close()


def test_noalloc_overflow_fallback_and_seed_scan(hn):
    """A survivor list far too small: the overflowing queries are finished by
    the exhaustive float64 pass, as in hn_search_top1; and the float32 seed
    scan gives the same results."""
    k, alpha = 16, 1 / 8
    base = hn_inputs.make_db(64, k, alpha, 2, 77)
    db = np.tile(base, (40, 1))
    qs = hn_inputs.make_queries(base, k, alpha, 24, 8, 78)
    ix = hn.Index(dev(db), k, alpha)
    q = dev(qs)
    ref = oracle.bnb_top1(db, qs, k, alpha)
    for ss in ("bf16", "fp32"):
        say("noalloc overflow, seed scan %s" % ss)
        want = ix.search(q, survivor_cap=500, seed_scan=ss)
        got = ix.search_noalloc(q, survivor_cap=500, seed_scan=ss)
        assert _same(got, want)
        assert (got[0].cpu().numpy() == ref["idx"]).all()
    ix.close()


def test_noalloc_full_size_benchmark_workload(hn):
    """N = 2^20, K = 16, alpha = 1/8 with 10,000 queries fits the static
    scratch and matches hn_search_top1; then a call with 7 queries."""
    k, alpha = 16, 1 / 8
    say("noalloc full size: generating N=2^20")
    db = hn_inputs.make_db(1 << 20, k, alpha, 4096, 8900)
    qs = hn_inputs.make_queries(db, k, alpha, 9000, 1000, 8901)
    ix = hn.Index(dev(db), k, alpha)
    q = dev(qs)
    for n_q in (10000, 7):
        say("noalloc full size: q=%d" % n_q)
        want = ix.search(q[:n_q])
        got = ix.search_noalloc(q[:n_q])
        assert _same(got, want)
    ref = oracle.bnb_top1(db, qs[:5], k, alpha)
    assert (got[0].cpu().numpy()[:5] == ref["idx"]).all()
    ix.close()


def test_noalloc_rejects_before_enqueuing(hn):
    import torch
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(1000, k, alpha, 4, 8950)
    ix = hn.Index(dev(db), k, alpha)
    qs = dev(hn_inputs.make_queries(db, k, alpha, 30, 0, 8951))
    for kw, code in (({"precision": "fp8"}, -5), ({"precision": "int8"}, -5),
                     ({"survivor_cap": 1 << 40}, -1)):
        say("noalloc rejects %s" % kw)
        with pytest.raises(hn.HNError) as e:
            ix.search_noalloc(qs, **kw)
        assert e.value.code == code
    big = torch.zeros((400000, 128), dtype=torch.float32, device="cuda:0")
    out = _outs(400000)
    out[0].fill_(-7)
    say("noalloc rejects q=400000")
    with pytest.raises(hn.HNError) as e:
        ix.search_noalloc(big, out=out)
    assert e.value.code == -1 and "fewer queries" in str(e.value)
    torch.cuda.synchronize()
    assert int(out[0].min()) == -7 and int(out[0].max()) == -7  # nothing written
    got = ix.search_noalloc(qs)
    assert _same(got, ix.search(qs))
    ix.close()
