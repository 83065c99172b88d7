"""CPU float64 oracle for HN exact top-1 search.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the HIP
library or its Python binding, and nothing here imports them.

The search functions live in ``oracle.c`` (plain C, float64, one thread per
contiguous query range); this module compiles it with gcc, loads it with
ctypes, and adds the float64 numpy pieces that are easier to read in numpy:
the HN layer of Eq. 1 (Section 3.1) with its Jacobian, and the seed-model MLP
forward/backward with its optimiser step.

Seed-model pieces (not in the paper; they follow the learned-seed design used
by this project): a 128-256-256-512 MLP with exact-erf GELU, softmax
cross-entropy over anchors, and AdamW with decoupled weight decay.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fno-fast-math",
                               "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.or_sim.argtypes = [_f32p, _f32p, _int]
        L.or_sim.restype = _dbl
        L.or_norm.argtypes = [_f32p, _int, _int]
        L.or_norm.restype = _dbl
        L.or_db_max_norms.argtypes = [_f32p, _i64, _int, _int, _f64p]
        L.or_db_max_norms.restype = None
        L.or_bruteforce_top1.argtypes = [_f32p, _i64, _int, _f32p, _i64, _int, _i64p, _f64p]
        L.or_bruteforce_top1.restype = None
        L.or_bnb_slack.argtypes = [_f32p, _int, _int, _dbl, _dbl, _dbl, _dbl]
        L.or_bnb_slack.restype = _dbl
        L.or_bnb_top1.argtypes = [_f32p, _i64, _int, _int, _dbl, _dbl, _f64p, _f32p, _i64,
                                  _int, _i64p, _f64p, _i64p, _f64p, _i64p, _f64p]
        L.or_bnb_top1.restype = None
        L.or_survivor_counts.argtypes = [_f32p, _i64, _int, _int, _dbl, _f32p, _i64, _f64p,
                                         _f64p, _int, _i64p, _i64p]
        L.or_survivor_counts.restype = None
        L.or_survivor_list.argtypes = [_f32p, _i64, _int, _int, _dbl, _f32p, _dbl, _i64p, _i64]
        L.or_survivor_list.restype = _i64
        L.or_topk.argtypes = [_f32p, _i64, _int, _f32p, _i64, _int, _int, _i64p, _f64p]
        L.or_topk.restype = None
        L.or_kmeanspp.argtypes = [_f32p, _i64, _int, _int, _f64p, _i64p]
        L.or_kmeanspp.restype = None
        _lib = L
    return _lib


def default_threads() -> int:
    """Host threads to use: the CPUs this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ----------------------------------------------------------------- search

def sim(q, x) -> float:
    """Canonical float64 sim of two float32 vectors (ascending-j sum)."""
    q, x = _f32(q), _f32(x)
    assert q.shape == x.shape and q.ndim == 1
    return lib().or_sim(q, x, q.shape[0])


def db_max_norms(db, k: int):
    """(mu_M, mu_m, mu): largest major, minor and full norms over the rows."""
    db = _f32(db)
    out = np.zeros(3, dtype=np.float64)
    lib().or_db_max_norms(db, db.shape[0], db.shape[1], k, out)
    return tuple(out)


def bruteforce_top1(db, qs, threads: int | None = None):
    """Exhaustive top-1 (index, sim) per query, ties to the smallest index."""
    db, qs = _f32(db), _f32(qs)
    nq = qs.shape[0]
    idx = np.empty(nq, dtype=np.int64)
    sv = np.empty(nq, dtype=np.float64)
    lib().or_bruteforce_top1(db, db.shape[0], db.shape[1], qs, nq,
                             threads or default_threads(), idx, sv)
    return idx, sv


def bnb_top1(db, qs, k: int, alpha: float, beta: float | None = None,
             threads: int | None = None, norms=None):
    """Algorithm 1 (Section 3.3) per query in float64.  Returns a dict with
    idx, sim, seed_idx, seed_sim, phase2 (entries evaluated in full besides
    the seed) and slack."""
    db, qs = _f32(db), _f32(qs)
    nq = qs.shape[0]
    if norms is None:
        norms = db_max_norms(db, k)
    nrm = np.ascontiguousarray(norms, dtype=np.float64)
    out = {n: np.empty(nq, dtype=t) for n, t in
           [("idx", np.int64), ("sim", np.float64), ("seed_idx", np.int64),
            ("seed_sim", np.float64), ("phase2", np.int64), ("slack", np.float64)]}
    lib().or_bnb_top1(db, db.shape[0], db.shape[1], k, alpha,
                      -1.0 if beta is None else float(beta), nrm, qs, nq,
                      threads or default_threads(), out["idx"], out["sim"],
                      out["seed_idx"], out["seed_sim"], out["phase2"], out["slack"])
    return out


def survivor_counts(db, qs, k: int, alpha: float, lo, hi, threads: int | None = None):
    """|{i : dot_K(q, x_i) + alpha >= lo[q]}| and the same at hi[q]."""
    db, qs = _f32(db), _f32(qs)
    nq = qs.shape[0]
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    a = np.empty(nq, dtype=np.int64)
    b = np.empty(nq, dtype=np.int64)
    lib().or_survivor_counts(db, db.shape[0], db.shape[1], k, alpha, qs, nq, lo, hi,
                             threads or default_threads(), a, b)
    return a, b


def survivor_list(db, q, k: int, alpha: float, L: float):
    """Ascending indices of S(q, L) = {i : dot_K(q, x_i) + alpha >= L}."""
    db, q = _f32(db), _f32(q)
    cap = db.shape[0]
    out = np.empty(cap, dtype=np.int64)
    m = lib().or_survivor_list(db, db.shape[0], db.shape[1], k, alpha, q, float(L), out, cap)
    return out[:m].copy()


def topk(db, qs, kk: int, threads: int | None = None):
    """Exhaustive top-kk per query, ordered by (sim desc, index asc)."""
    db, qs = _f32(db), _f32(qs)
    nq = qs.shape[0]
    idx = np.empty((nq, kk), dtype=np.int64)
    sv = np.empty((nq, kk), dtype=np.float64)
    lib().or_topk(db, db.shape[0], db.shape[1], qs, nq, kk,
                  threads or default_threads(), idx, sv)
    return idx, sv


def kmeanspp(db, n_anchor: int, u):
    """k-means++ D^2 seeding with quantised weights (see oracle.c)."""
    db = _f32(db)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape[0] >= n_anchor
    out = np.empty(n_anchor, dtype=np.int64)
    lib().or_kmeanspp(db, db.shape[0], db.shape[1], n_anchor, u, out)
    return out


# ------------------------------------------------------- HN layer (Eq. 1)

def hn_normalize(f, k: int, alpha: float) -> np.ndarray:
    """Eq. 1 in float64: major = sqrt(1-alpha) f[:K]/||f[:K]||, minor =
    sqrt(alpha) f[K:]/||f[K:]||; at alpha = 0 the minor is exactly zero."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    for r in range(f.shape[0]):
        m = f[r, :k]
        out[r, :k] = math.sqrt(1.0 - alpha) * m / math.sqrt(float(m @ m))
        if alpha > 0.0:
            t = f[r, k:]
            out[r, k:] = math.sqrt(alpha) * t / math.sqrt(float(t @ t))
    return out


def hn_backward(f, g, k: int, alpha: float) -> np.ndarray:
    """Vector-Jacobian product of Eq. 1: for a block scaled to norm c,
    y = c f/||f|| has dy/df = (c/||f||)(I - u u^T), u = f/||f||."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros_like(f)
    for r in range(f.shape[0]):
        for lo, hi, c in ((0, k, math.sqrt(1.0 - alpha)), (k, f.shape[1], math.sqrt(alpha))):
            if c == 0.0:
                continue
            v = f[r, lo:hi]
            nv = math.sqrt(float(v @ v))
            u = v / nv
            gb = g[r, lo:hi]
            out[r, lo:hi] = (c / nv) * (gb - u * float(u @ gb))
    return out


# ----------------------------------------------------- seed-model MLP

_SQRT2 = math.sqrt(2.0)
_INV_SQRT2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def gelu(x):
    """Exact GELU: x * Phi(x) = 0.5 x (1 + erf(x / sqrt 2))."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + _erf(x / _SQRT2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + _erf(x / _SQRT2)) + x * _INV_SQRT2PI * np.exp(-0.5 * x * x)


def mlp_forward(params, x):
    """params = (W1 [256,128], b1, W2 [256,256], b2, W3 [512,256], b3), all
    float64.  Returns logits and the cache for the backward pass."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    logits = h2 @ W3.T + b3
    return logits, (x, z1, h1, z2, h2)


def softmax_ce(logits, labels):
    """Mean softmax cross-entropy and its gradient w.r.t. the logits."""
    z = np.asarray(logits, dtype=np.float64)
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    s = e.sum(axis=1, keepdims=True)
    p = e / s
    B = z.shape[0]
    loss = float(np.mean(np.log(s[:, 0]) + m[:, 0] - z[np.arange(B), labels]))
    g = p.copy()
    g[np.arange(B), labels] -= 1.0
    return loss, g / B


def mlp_backward(params, cache, dlogits):
    """Gradients (dW1, db1, dW2, db2, dW3, db3) for the given dL/dlogits."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    x, z1, h1, z2, h2 = cache
    dW3 = dlogits.T @ h2
    db3 = dlogits.sum(axis=0)
    dz2 = (dlogits @ W3) * gelu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def adamw_step(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
               eps: float = 1e-8, wd: float = 0.0):
    """One AdamW update (decoupled weight decay), step count t >= 1.
    Returns the new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v


def top4(logits):
    """Indices of the 4 largest logits per row, ties to the smaller index."""
    z = np.asarray(logits)
    order = np.lexsort((np.broadcast_to(np.arange(z.shape[1]), z.shape), -z), axis=1)
    return order[:, :4]
