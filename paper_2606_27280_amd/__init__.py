"""Exact top-1 inner-product search over HN vectors on MI355X.

Thin binding over libhnsearch (include/hnsearch.h): torch tensors provide
device memory and the current HIP stream; every step of the search runs in the
library's HIP kernels.  Importing this package does not load the library; the
first call does, and it raises if the library has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (HN_BUILD_NO_VALIDATE, HN_MLP_PARAMS, HN_PREC_BF16, HN_PREC_FP8,
                   HN_PREC_FP32, HN_SEED_LEARNED, HN_SEED_PLAIN, HN_SEED_WINDOW, HNError)

__all__ = ["Index", "bruteforce_top1", "profile", "HNError", "PRECISIONS", "SEEDS",
           "HN_PREC_FP32", "HN_PREC_BF16", "HN_PREC_FP8", "HN_SEED_PLAIN", "HN_SEED_LEARNED",
           "HN_SEED_WINDOW", "HN_BUILD_NO_VALIDATE", "HN_MLP_PARAMS", "SEED_SCANS",
           "mlp_forward", "mlp_grad", "mlp_adamw", "seed_train", "MultiPlan", "hn_layer",
           "hn_layer_backward", "set_memory_budget", "memory_held", "release_scratch"]

D = 128  # descriptor length the library is built for

PRECISIONS = {"fp32": HN_PREC_FP32, "bf16": HN_PREC_BF16, "fp8": HN_PREC_FP8,
              "int8": _lib.HN_PREC_INT8}
SEEDS = {"plain": HN_SEED_PLAIN, "learned": HN_SEED_LEARNED, "window": HN_SEED_WINDOW}


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, ndim=None, shape=None, device=None):
    """Check one device tensor argument and return its pointer.  Every array
    the library reads or writes goes through here, so a wrong width, size,
    dtype, layout or device raises ValueError before any library call (the
    C ABI takes bare pointers and sizes and cannot see the allocation)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA/HIP tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s (got %s)" % (name, dtype, t.dtype))
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dimensions (got %d)" % (name, ndim, t.dim()))
    if shape is not None:
        want = tuple(shape)
        got = tuple(t.shape)
        if len(got) != len(want) or any(w is not None and g != w for g, w in zip(got, want)):
            raise ValueError("%s must have shape %s (got %s)" % (
                name, tuple("*" if w is None else w for w in want), got))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, the index on %s" % (name, t.device, device))
    return ctypes.c_void_p(t.data_ptr())


def _rows(t, name, device=None, n=None):
    """float32 [n][128] rows (queries, databases, HN-layer inputs)."""
    return _dev(t, _torch().float32, name, 2, (n, D), device)


def _outputs(out, q, device, idx_shape=None):
    """The caller's (idx int64, sim float64) outputs, or new ones."""
    torch = _torch()
    shape = (q,) if idx_shape is None else idx_shape
    if out is None:
        return (torch.empty(shape, dtype=torch.int64, device=device),
                torch.empty(shape, dtype=torch.float64, device=device))
    if not isinstance(out, (tuple, list)) or len(out) != 2:
        raise ValueError("out must be a pair (idx, sim)")
    idx, sim = out
    _dev(idx, torch.int64, "out idx", len(shape), shape, device)
    _dev(sim, torch.float64, "out sim", len(shape), shape, device)
    return idx, sim


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


SEED_SCANS = {"bf16": _lib.HN_SEED_SCAN_BF16, "fp32": _lib.HN_SEED_SCAN_FP32}


def _opts(precision="fp32", query_tiles=0, chunk_blocks=0, survivor_cap=0, beta=None,
          seed="plain", seed_scan="bf16"):
    o = _lib.SearchOpts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.seed = SEEDS[seed] if isinstance(seed, str) else int(seed)
    o.query_tiles = int(query_tiles)
    o.chunk_blocks = int(chunk_blocks)
    o.survivor_cap = int(survivor_cap)
    o.beta = -1.0 if beta is None else float(beta)
    o.seed_scan = SEED_SCANS[seed_scan] if isinstance(seed_scan, str) else int(seed_scan)
    return o


class Index:
    """hn_build_index / hn_search_top1 / hn_filter_survivors / hn_scan_scores.
    Every array argument must live on the index's device."""

    def __init__(self, db, k: int, alpha: float, flags: int = 0, stream=None):
        L = _lib.lib()
        dp = _rows(db, "db")
        h = ctypes.c_void_p()
        _lib.check(L.hn_build_index(dp, db.shape[0], db.shape[1], int(k), float(alpha),
                                    int(flags), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n = int(db.shape[0])
        self.k = int(k)
        self.alpha = float(alpha)
        self.device = db.device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().hn_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, k, a = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        norms = (ctypes.c_double * 3)()
        _lib.check(_lib.lib().hn_index_info(self._h, ctypes.byref(n), ctypes.byref(k),
                                            ctypes.byref(a), norms))
        return {"n": n.value, "k": k.value, "alpha": a.value, "norms": tuple(norms)}

    def _aux(self, q):
        torch = _torch()
        dev = self.device
        auxd = {"seed_idx": torch.empty(q, dtype=torch.int64, device=dev),
                "seed_sim": torch.empty(q, dtype=torch.float64, device=dev),
                "threshold": torch.empty(q, dtype=torch.float32, device=dev),
                "survivors": torch.empty(q, dtype=torch.int32, device=dev),
                "slack": torch.empty(q, dtype=torch.float64, device=dev)}
        return auxd, _lib.SearchAux(*[_ptr(auxd[f]) for f, _ in _lib.SearchAux._fields_])

    def search(self, queries, precision="fp32", query_tiles=0, chunk_blocks=0,
               survivor_cap=0, beta=None, aux=False, stats=False, stream=None, out=None,
               seed="plain", seed_scan="bf16"):
        """Exact top-1 per query: (idx int64 [q], sim float64 [q]) plus the
        auxiliary outputs (dict) and/or the call's stats when requested.
        seed_scan: precision of the plain seed's argmax scan ("bf16" or
        "fp32"); the result does not depend on it."""
        qp = _rows(queries, "queries", self.device)
        q = queries.shape[0]
        idx, sim = _outputs(out, q, self.device)
        o = _opts(precision, query_tiles, chunk_blocks, survivor_cap, beta, seed, seed_scan)
        auxd, a = self._aux(q) if aux else (None, None)
        st = _lib.SearchStats() if stats else None
        _lib.check(_lib.lib().hn_search_top1(
            self._h, qp, q, _ptr(idx), _ptr(sim), ctypes.byref(o),
            ctypes.byref(a) if a is not None else None,
            ctypes.byref(st) if st is not None else None, _stream(stream)))
        res = [idx, sim]
        if aux:
            res.append(auxd)
        if stats:
            res.append({"survivors": st.survivors, "overflow_queries": st.overflow_queries})
        return tuple(res)

    def search_noalloc(self, queries, precision="fp32", query_tiles=0, chunk_blocks=0,
                       survivor_cap=0, beta=None, aux=False, stream=None, out=None,
                       seed_scan="bf16"):
        """hn_search_top1_noalloc: the same search with the library's static
        per-GPU scratch (no device allocation inside the call; pass `out` to
        allocate nothing at all).  Calls that overlap on one GPU race."""
        qp = _rows(queries, "queries", self.device)
        q = queries.shape[0]
        idx, sim = _outputs(out, q, self.device)
        o = _opts(precision, query_tiles, chunk_blocks, survivor_cap, beta, "plain", seed_scan)
        auxd, a = self._aux(q) if aux else (None, None)
        _lib.check(_lib.lib().hn_search_top1_noalloc(
            self._h, qp, q, _ptr(idx), _ptr(sim), ctypes.byref(o),
            ctypes.byref(a) if a is not None else None, _stream(stream)))
        return (idx, sim, auxd) if aux else (idx, sim)

    def search_topk(self, queries, topk, precision="fp32", query_tiles=0, chunk_blocks=0,
                    survivor_cap=0, beta=None, stream=None, seed_scan="bf16"):
        """Exact top-k per query (hn_search_topk): (idx int64 [q][topk],
        sim float64 [q][topk]) ordered by (sim desc, index asc)."""
        qp = _rows(queries, "queries", self.device)
        q = queries.shape[0]
        if not 1 <= int(topk) <= 128:
            raise ValueError("topk must be in [1, 128]")
        idx, sim = _outputs(None, q, self.device, (q, int(topk)))
        o = _opts(precision, query_tiles, chunk_blocks, survivor_cap, beta, "plain", seed_scan)
        _lib.check(_lib.lib().hn_search_topk(self._h, qp, q, int(topk), _ptr(idx), _ptr(sim),
                                             ctypes.byref(o), _stream(stream)))
        return idx, sim

    def filter_survivors(self, queries, lower, cap, precision="fp32", beta=None, stream=None):
        """Pairs (query, entry) with scan score >= round_down(L - alpha - eps);
        returns (pairs int32 [min(count,cap)][2], count, slack float64 [q])."""
        torch = _torch()
        qp = _rows(queries, "queries", self.device)
        q = queries.shape[0]
        lp = _dev(lower, torch.float64, "lower", 1, (q,), self.device)
        if int(cap) < 0:
            raise ValueError("cap must be >= 0")
        pairs = torch.empty((max(int(cap), 1), 2), dtype=torch.int32, device=self.device)
        slack = torch.empty(q, dtype=torch.float64, device=self.device)
        cnt = ctypes.c_int64()
        o = _opts(precision, beta=beta)
        _lib.check(_lib.lib().hn_filter_survivors(self._h, qp, q, lp, _ptr(pairs), int(cap),
                                                  ctypes.byref(cnt), _ptr(slack),
                                                  ctypes.byref(o), _stream(stream)))
        return pairs[: min(cnt.value, int(cap))], cnt.value, slack

    def scan_scores(self, queries, precision="fp32", stream=None):
        torch = _torch()
        qp = _rows(queries, "queries", self.device)
        q = queries.shape[0]
        out = torch.empty((q, self.n), dtype=torch.float32, device=self.device)
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _lib.check(_lib.lib().hn_scan_scores(self._h, qp, q, p, _ptr(out), _stream(stream)))
        return out

    def kmeanspp(self, n_anchor, u, stream=None):
        """k-means++ D^2 seeding (hn_kmeanspp): int64 [n_anchor] entry ids
        from the uniform draws u (float64 [n_anchor], device)."""
        torch = _torch()
        if int(n_anchor) < 1:
            raise ValueError("n_anchor must be >= 1")
        up = _dev(u, torch.float64, "u", 1, None, self.device)
        if u.shape[0] < n_anchor:
            raise ValueError("u needs n_anchor draws")
        out = torch.empty(int(n_anchor), dtype=torch.int64, device=self.device)
        _lib.check(_lib.lib().hn_kmeanspp(self._h, int(n_anchor), up, _ptr(out),
                                          _stream(stream)))
        return out

    def seed_labels(self, anchors, queries, stream=None):
        """Training labels (hn_seed_labels): int32 [q]."""
        torch = _torch()
        ap = _dev(anchors, torch.int64, "anchors", 1, None, self.device)
        qp = _rows(queries, "queries", self.device)
        out = torch.empty(queries.shape[0], dtype=torch.int32, device=self.device)
        _lib.check(_lib.lib().hn_seed_labels(self._h, ap, anchors.shape[0], qp,
                                             queries.shape[0], _ptr(out), _stream(stream)))
        return out

    def set_seed_model(self, params, anchors, stream=None):
        """Install the seed model (hn_set_seed_model) for seed="learned"."""
        torch = _torch()
        pp = _dev(params, torch.float32, "params", 1, (HN_MLP_PARAMS,), self.device)
        ap = _dev(anchors, torch.int64, "anchors", 1, (_lib.HN_MLP_OUT,), self.device)
        _lib.check(_lib.lib().hn_set_seed_model(self._h, pp, ap, anchors.shape[0],
                                                _stream(stream)))


class MultiPlan:
    """hn_multi_plan_create / hn_multi_search: one search of ragged query
    batches against several indexes (the plain two-pass seed)."""

    def __init__(self, indexes, q_counts, precision="fp32", query_tiles=0, chunk_blocks=0,
                 survivor_cap=0, beta=None):
        n = len(indexes)
        if n != len(q_counts):
            raise ValueError("one query count per index")
        if n == 0:
            raise ValueError("a plan needs at least one index")
        devs = {ix.device for ix in indexes}
        if len(devs) != 1:
            raise ValueError("the indexes of a plan must share one device")
        self.device = indexes[0].device
        self._indexes = list(indexes)  # keep them alive
        hs = (ctypes.c_void_p * n)(*[ix._h.value for ix in indexes])
        qc = (ctypes.c_int64 * n)(*[int(c) for c in q_counts])
        o = _opts(precision, query_tiles, chunk_blocks, survivor_cap, beta)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().hn_multi_plan_create(hs, n, qc, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.q_counts = [int(c) for c in q_counts]
        self.total = sum(self.q_counts)

    def info(self):
        tq, wi, sl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _lib.check(_lib.lib().hn_multi_plan_info(self._h, ctypes.byref(tq), ctypes.byref(wi),
                                                 ctypes.byref(sl)))
        return {"total_queries": tq.value, "work_items": wi.value, "scan_launches": sl.value}

    def search(self, queries, use_graph=True, out=None, stream=None):
        """(idx int64 [total], sim float64 [total]) for the concatenated
        queries (database by database)."""
        qp = _rows(queries, "queries", self.device, self.total)
        idx, sim = _outputs(out, self.total, self.device)
        _lib.check(_lib.lib().hn_multi_search(self._h, qp, _ptr(idx), _ptr(sim),
                                              1 if use_graph else 0, _stream(stream)))
        return idx, sim

    def batch_times(self, stream=None):
        """hn_multi_batch_times: per database, milliseconds from the start of
        the last search to the last write of its results (device clock)."""
        n = len(self.q_counts)
        ms = (ctypes.c_double * n)()
        _lib.check(_lib.lib().hn_multi_batch_times(self._h, ms, _stream(stream)))
        return list(ms)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().hn_multi_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hn_layer(f, k, alpha, status=False, stream=None):
    """Eq. 1 on a batch (hn_layer_forward): float32 [b][128] out, plus the
    int32 row status when asked."""
    torch = _torch()
    fp = _rows(f, "f")
    out = torch.empty_like(f)
    st = torch.empty(f.shape[0], dtype=torch.int32, device=f.device) if status else None
    _lib.check(_lib.lib().hn_layer_forward(fp, f.shape[0], f.shape[1], int(k), float(alpha),
                                           _ptr(out), _ptr(st), _stream(stream)))
    return (out, st) if status else out


def hn_layer_backward(f, g, k, alpha, stream=None):
    """Vector-Jacobian product of Eq. 1 (hn_layer_backward)."""
    torch = _torch()
    fp = _rows(f, "f")
    gp = _rows(g, "g", f.device, f.shape[0])
    out = torch.empty_like(f)
    _lib.check(_lib.lib().hn_layer_backward(fp, gp, f.shape[0], f.shape[1], int(k), float(alpha),
                                            _ptr(out), _stream(stream)))
    return out


def _adamw(lr, beta1, beta2, eps, weight_decay):
    return _lib.AdamWOpts(float(lr), float(beta1), float(beta2), float(eps), float(weight_decay))


def _params(params):
    return _dev(params, _torch().float32, "params", 1, (HN_MLP_PARAMS,))


def mlp_forward(params, x, stream=None):
    """Seed-model logits [b][512] (hn_mlp_forward)."""
    torch = _torch()
    pp = _params(params)
    xp = _rows(x, "x", params.device)
    out = torch.empty((x.shape[0], _lib.HN_MLP_OUT), dtype=torch.float32, device=x.device)
    _lib.check(_lib.lib().hn_mlp_forward(pp, xp, x.shape[0], _ptr(out), _stream(stream)))
    return out


def mlp_grad(params, x, labels, stream=None):
    """(grads float32 [HN_MLP_PARAMS], mean loss float32 [1]) (hn_mlp_grad)."""
    torch = _torch()
    pp = _params(params)
    xp = _rows(x, "x", params.device)
    lp = _dev(labels, torch.int32, "labels", 1, (x.shape[0],), params.device)
    grads = torch.empty(HN_MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _lib.check(_lib.lib().hn_mlp_grad(pp, xp, lp, x.shape[0], _ptr(grads), _ptr(loss),
                                      _stream(stream)))
    return grads, loss


def mlp_adamw(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
              stream=None):
    """One in-place AdamW step (hn_mlp_adamw)."""
    torch = _torch()
    o = _adamw(lr, beta1, beta2, eps, weight_decay)
    n = params.shape[0]
    dev = params.device
    ptrs = (_dev(params, torch.float32, "params", 1),
            _dev(grads, torch.float32, "grads", 1, (n,), dev),
            _dev(m, torch.float32, "m", 1, (n,), dev), _dev(v, torch.float32, "v", 1, (n,), dev))
    _lib.check(_lib.lib().hn_mlp_adamw(*ptrs, n, int(t), ctypes.byref(o), _stream(stream)))


def seed_train(params, x, labels, batch, epochs, lr, beta1=0.9, beta2=0.999, eps=1e-8,
               weight_decay=0.0, stream=None):
    """Train the seed model in place (hn_seed_train); returns the per-step
    mean losses (float32 tensor)."""
    torch = _torch()
    pp = _params(params)
    xp = _rows(x, "x", params.device)
    lp = _dev(labels, torch.int32, "labels", 1, (x.shape[0],), params.device)
    n = x.shape[0]
    if int(batch) < 1 or int(epochs) < 0:
        raise ValueError("batch must be >= 1 and epochs >= 0")
    steps = int(epochs) * ((n + int(batch) - 1) // int(batch))
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device=x.device)
    o = _adamw(lr, beta1, beta2, eps, weight_decay)
    _lib.check(_lib.lib().hn_seed_train(pp, xp, lp, n, int(batch), int(epochs), ctypes.byref(o),
                                        _ptr(losses), _stream(stream)))
    return losses[:steps]


class profile:
    """Context manager over hn_profile_begin / hn_profile_end: per-kernel
    total milliseconds and launch counts for kernels enqueued on `stream`."""

    def __init__(self, stream=None):
        self.stream = stream
        self.result = {}

    def __enter__(self):
        _lib.check(_lib.lib().hn_profile_begin(_stream(self.stream)))
        return self

    def __exit__(self, *exc):
        mx = 64
        names = (ctypes.c_char_p * mx)()
        ms = (ctypes.c_double * mx)()
        cnt = (ctypes.c_int64 * mx)()
        n = ctypes.c_int32()
        _lib.check(_lib.lib().hn_profile_end(_stream(self.stream), names, ms, cnt, mx,
                                             ctypes.byref(n)))
        self.result = {names[i].decode(): {"ms": ms[i], "launches": cnt[i]}
                       for i in range(n.value)}
        return False


def bruteforce_top1(db, queries, stream=None, out=None):
    """Exhaustive exact top-1 (hn_bruteforce_top1): (idx int64, sim float64)."""
    dp = _rows(db, "db")
    qp = _rows(queries, "queries", db.device)
    q = queries.shape[0]
    idx, sim = _outputs(out, q, db.device)
    _lib.check(_lib.lib().hn_bruteforce_top1(dp, db.shape[0], db.shape[1], qp, q, _ptr(idx),
                                             _ptr(sim), _stream(stream)))
    return idx, sim


def set_memory_budget(max_bytes: int) -> None:
    """hn_set_memory_budget: cap the library's device holdings (0 = none)."""
    _lib.check(_lib.lib().hn_set_memory_budget(int(max_bytes)))


def memory_held() -> int:
    """hn_memory_held: bytes the library holds in device allocations."""
    return int(_lib.lib().hn_memory_held())


def release_scratch(stream=None) -> None:
    """hn_release_scratch: free the scratch arenas kept for `stream`."""
    _lib.check(_lib.lib().hn_release_scratch(_stream(stream)))
