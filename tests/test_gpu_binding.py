"""The Python binding rejects malformed arguments with ValueError before it
calls the library: the C ABI takes bare pointers and sizes, so a wrong width,
length, dtype, layout or device would otherwise make a kernel read or write
outside an allocation.  Also the library's device-memory budget: an injected
limit makes the build, the search and the multi-database plan fail with
HN_ERR_OOM, releasing everything they took."""
import numpy as np
import pytest

import hn_inputs

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


class _NoCall:
    """Stands in for the loaded library: any attribute access fails the test,
    so a ValueError must come before the first library call."""

    def __getattr__(self, name):
        raise AssertionError("library function %s reached with a bad argument" % name)


def test_bad_arguments_raise_before_any_library_call(hn, monkeypatch):
    import torch
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(700, k, alpha, 4, 31)
    qs = hn_inputs.make_queries(db, k, alpha, 20, 4, 32)
    ix = hn.Index(dev(db), k, alpha)
    q = dev(qs)
    d = q.device
    params = torch.zeros(hn.HN_MLP_PARAMS, dtype=torch.float32, device=d)
    anchors = torch.arange(512, dtype=torch.int64, device=d)
    plan = hn.MultiPlan([ix], [len(qs)])
    bad = {
        "queries of width 64": lambda: ix.search(q[:, :64].contiguous()),
        "queries of width 129": lambda: ix.search(torch.zeros(3, 129, device=d)),
        "float64 queries": lambda: ix.search(q.double()),
        "host queries": lambda: ix.search(torch.from_numpy(qs)),
        "1-d queries": lambda: ix.search(q[0].contiguous()),
        "strided queries": lambda: ix.search(torch.zeros(128, 8, device=d).t()),
        "short out idx": lambda: ix.search(q, out=(torch.empty(3, dtype=torch.int64, device=d),
                                                   torch.empty(len(qs), dtype=torch.float64,
                                                               device=d))),
        "int32 out idx": lambda: ix.search(q, out=(torch.empty(len(qs), dtype=torch.int32,
                                                               device=d),
                                                   torch.empty(len(qs), dtype=torch.float64,
                                                               device=d))),
        "float32 out sim": lambda: ix.search(q, out=(torch.empty(len(qs), dtype=torch.int64,
                                                                 device=d),
                                                     torch.empty(len(qs), dtype=torch.float32,
                                                                 device=d))),
        "strided out": lambda: ix.search(q, out=(torch.empty(2 * len(qs), dtype=torch.int64,
                                                             device=d)[::2],
                                                 torch.empty(len(qs), dtype=torch.float64,
                                                             device=d))),
        "noalloc narrow queries": lambda: ix.search_noalloc(q[:, :100].contiguous()),
        "noalloc short out": lambda: ix.search_noalloc(
            q, out=(torch.empty(1, dtype=torch.int64, device=d),
                    torch.empty(1, dtype=torch.float64, device=d))),
        "topk narrow queries": lambda: ix.search_topk(q[:, :64].contiguous(), 3),
        "topk of 0": lambda: ix.search_topk(q, 0),
        "filter lower too short": lambda: ix.filter_survivors(
            q, torch.zeros(len(qs) - 1, dtype=torch.float64, device=d), cap=10),
        "filter lower float32": lambda: ix.filter_survivors(
            q, torch.zeros(len(qs), dtype=torch.float32, device=d), cap=10),
        "filter negative cap": lambda: ix.filter_survivors(
            q, torch.zeros(len(qs), dtype=torch.float64, device=d), cap=-1),
        "scores narrow queries": lambda: ix.scan_scores(q[:, :64].contiguous()),
        "kmeans host draws": lambda: ix.kmeanspp(4, torch.zeros(4, dtype=torch.float64)),
        "kmeans too few draws": lambda: ix.kmeanspp(8, torch.zeros(4, dtype=torch.float64,
                                                                   device=d)),
        "labels int32 anchors": lambda: ix.seed_labels(anchors.int(), q),
        "labels narrow queries": lambda: ix.seed_labels(anchors, q[:, :64].contiguous()),
        "model short params": lambda: ix.set_seed_model(params[:100], anchors),
        "model 511 anchors": lambda: ix.set_seed_model(params, anchors[:511].contiguous()),
        "plan wrong row count": lambda: plan.search(q[:5].contiguous()),
        "plan narrow queries": lambda: plan.search(q[:, :64].contiguous()),
        "build width 64": lambda: hn.Index(q[:, :64].contiguous(), k, alpha),
        "bruteforce narrow db": lambda: hn.bruteforce_top1(dev(db)[:, :64].contiguous(), q),
        "bruteforce host queries": lambda: hn.bruteforce_top1(dev(db), torch.from_numpy(qs)),
        "layer width 64": lambda: hn.hn_layer(q[:, :64].contiguous(), k, alpha),
        "layer backward g rows": lambda: hn.hn_layer_backward(q, q[:3].contiguous(), k, alpha),
        "mlp x width 64": lambda: hn.mlp_forward(params, q[:, :64].contiguous()),
        "mlp short params": lambda: hn.mlp_forward(params[:10], q),
        "grad labels length": lambda: hn.mlp_grad(params, q, torch.zeros(3, dtype=torch.int32,
                                                                          device=d)),
        "adamw m length": lambda: hn.mlp_adamw(params, params, params[:5], params, 1, 1e-3),
        "train labels length": lambda: hn.seed_train(params, q, torch.zeros(
            1, dtype=torch.int32, device=d), 8, 1, 1e-3),
    }
    from paper_2606_27280_amd import _lib
    monkeypatch.setattr(_lib, "_lib", _NoCall())
    for what, call in bad.items():
        say("bad argument: %s" % what)
        with pytest.raises(ValueError):
            call()
    monkeypatch.undo()
    # the same objects still work with good arguments
    idx, sim = ix.search(q)
    assert idx.shape == (len(qs),)
    plan.close()
    ix.close()


def test_memory_budget_makes_allocations_fail_cleanly(hn):
    """An injected device-memory budget makes every allocating entry point
    return HN_ERR_OOM; the library then holds exactly what it held before the
    call (no leak), and works again once the budget is lifted."""
    import torch
    k, alpha = 16, 1 / 8
    db = hn_inputs.make_db(20000, k, alpha, 40, 41)
    qs = hn_inputs.make_queries(db, k, alpha, 200, 20, 42)
    d_db, d_q = dev(db), dev(qs)
    stream = torch.cuda.current_stream()
    hn.release_scratch()
    try:
        base = hn.memory_held()
        say("budget: build with too little room")
        hn.set_memory_budget(base + 4 * 1024 * 1024)  # the rows alone take 10 MB
        with pytest.raises(hn.HNError) as e:
            hn.Index(d_db, k, alpha)
        assert e.value.code == -3
        assert hn.memory_held() == base
        hn.set_memory_budget(0)
        ix = hn.Index(d_db, k, alpha)
        with_index = hn.memory_held()
        assert with_index > base + 10 * 1024 * 1024
        say("budget: search scratch beyond the budget")
        hn.set_memory_budget(with_index + 1024)
        with pytest.raises(hn.HNError) as e:
            ix.search(d_q)
        assert e.value.code == -3
        assert hn.memory_held() == with_index
        say("budget: multi-database plan beyond the budget")
        with pytest.raises(hn.HNError) as e:
            hn.MultiPlan([ix], [len(qs)])
        assert e.value.code == -3
        assert hn.memory_held() == with_index
        say("budget: seed model beyond the budget")
        params = torch.zeros(hn.HN_MLP_PARAMS, dtype=torch.float32, device="cuda:0")
        anchors = torch.arange(512, dtype=torch.int64, device="cuda:0")
        with pytest.raises(hn.HNError) as e:
            ix.set_seed_model(params, anchors)
        assert e.value.code == -3
        assert hn.memory_held() == with_index
        hn.set_memory_budget(0)
        say("budget lifted: search, plan and model work again")
        idx, sim = ix.search(d_q)
        ref_idx, ref_sim = hn.bruteforce_top1(d_db, d_q)
        assert torch.equal(idx, ref_idx) and torch.equal(sim, ref_sim)
        plan = hn.MultiPlan([ix], [len(qs)])
        pi, ps = plan.search(d_q)
        assert torch.equal(pi, idx)
        plan.close()
        ix.set_seed_model(params, anchors)
        ix.close()
        hn.release_scratch()
        stream.synchronize()
        assert hn.memory_held() == base
    finally:
        hn.set_memory_budget(0)
    with pytest.raises(hn.HNError):
        hn.set_memory_budget(-1)
