"""Seeded synthetic inputs for HN exact top-1 search.

This module only draws inputs: clustered Gaussian databases, perturbed and
fresh queries, and the uniform draws that seeded procedures consume.  It holds
none of the search arithmetic (no scan, bound, rescoring or argmax).  Both the
HIP path (through its tests and the benchmark) and the CPU oracle read what it
produces, and neither side imports the other.

Every vector is produced in float64 and stored in float32.  The final step of
the recipe places each raw vector on the hierarchical-normalisation sphere of
Eq. 1 (Section 3.1): the first K coordinates are scaled to norm sqrt(1-alpha)
and the remaining D-K to norm sqrt(alpha); at alpha = 0 the minor block is set
to exactly zero.  This stands in for the descriptor network's HN layer, whose
output the paper searches; the paper's UBC descriptors and trained weights are
not available, so these seeded clustered vectors replace them.

Recipe (one ``numpy.random.Generator(PCG64(seed))`` stream per database and
one per query set):
  * centres ~ N(0, I_D), D = 128; cluster id uniform per entry;
  * entry = HN(centre[cid] + N(0, 0.3^2 I));
  * perturbed query = HN(x_r + N(0, 0.05^2 I)), r uniform with replacement;
  * fresh query = HN(N(0, I)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

D = 128
DB_SEED_BASE = 0x484E0000
QUERY_SEED_OFFSET = 0x100
_CHUNK = 1 << 18


def _hn_place(v: np.ndarray, k: int, alpha: float) -> np.ndarray:
    """Scale the K-prefix of float64 rows to norm sqrt(1-alpha) and the rest to
    sqrt(alpha) (alpha = 0 gives an exact zero minor).  Returns float32."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    maj = v[:, :k]
    nm = np.sqrt(np.einsum("ij,ij->i", maj, maj))
    out[:, :k] = maj * (math.sqrt(1.0 - alpha) / nm)[:, None]
    if alpha == 0.0:
        out[:, k:] = 0.0
    else:
        mi = v[:, k:]
        nn = np.sqrt(np.einsum("ij,ij->i", mi, mi))
        out[:, k:] = mi * (math.sqrt(alpha) / nn)[:, None]
    return out.astype(np.float32)


def make_db(n: int, k: int, alpha: float, n_clusters: int, seed: int,
            noise: float = 0.3, d: int = D) -> np.ndarray:
    """Clustered HN database, float32 [n][d], C-contiguous."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.standard_normal((n_clusters, d))
    db = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        cid = rng.integers(0, n_clusters, size=e - s)
        raw = centres[cid] + noise * rng.standard_normal((e - s, d))
        db[s:e] = _hn_place(raw, k, alpha)
    return db


def make_queries(db: np.ndarray, k: int, alpha: float, n_perturbed: int,
                 n_fresh: int, seed: int, noise: float = 0.05) -> np.ndarray:
    """Perturbed database entries first, then fresh random HN vectors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = db.shape[1]
    out = np.empty((n_perturbed + n_fresh, d), dtype=np.float32)
    for s in range(0, n_perturbed, _CHUNK):
        e = min(n_perturbed, s + _CHUNK)
        r = rng.integers(0, db.shape[0], size=e - s)
        raw = db[r].astype(np.float64) + noise * rng.standard_normal((e - s, d))
        out[s:e] = _hn_place(raw, k, alpha)
    if n_fresh:
        out[n_perturbed:] = _hn_place(rng.standard_normal((n_fresh, d)), k, alpha)
    return out


def uniform_draws(n: int, seed: int) -> np.ndarray:
    """float64 draws in [0, 1) for procedures that sample (k-means++ picks,
    minibatch order)."""
    return np.random.Generator(np.random.PCG64(seed)).random(n)


def mlp_init(seed: int, sizes=(128, 256, 256, 512)) -> np.ndarray:
    """Initial seed-model parameters, float32, in the flat layout W1, b1, W2,
    b2, W3, b3 (weights [out][in]): every value uniform in
    [-1/sqrt(in), 1/sqrt(in)] of its layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(rng.uniform(-lim, lim, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Workload:
    name: str
    n: int
    k: int
    alpha: float
    n_clusters: int
    n_perturbed: int
    n_fresh: int
    db_seed: int
    q_seed: int
    extra: dict = field(default_factory=dict)

    def db(self) -> np.ndarray:
        return make_db(self.n, self.k, self.alpha, self.n_clusters, self.db_seed)

    def queries(self, db: np.ndarray | None = None) -> np.ndarray:
        if db is None:
            db = self.db()
        return make_queries(db, self.k, self.alpha, self.n_perturbed,
                            self.n_fresh, self.q_seed)

    def train_queries(self, db: np.ndarray) -> np.ndarray:
        """The learned seed's training queries (perturbed entries, a stream of
        their own, disjoint from the held-out queries' seed)."""
        return make_queries(db, self.k, self.alpha, self.extra["n_train"], 0,
                            self.extra["train_seed"])


def workload(idx: int, scale: float = 1.0) -> Workload:
    """The five synthetic workloads (1-based).  ``scale`` < 1 shrinks N, the
    cluster count and Q proportionally (for quick runs); 1.0 is full size."""
    def sz(v, lo=1):
        return max(lo, int(round(v * scale)))
    seed = DB_SEED_BASE + idx
    qseed = seed + QUERY_SEED_OFFSET
    if idx == 1:
        return Workload("hn_n16k_k8_a1-32", sz(16384, 256), 8, 1 / 32, sz(64),
                        sz(256), 0, seed, qseed)
    if idx == 2:
        return Workload("hn_n1m_k16_a1-8", sz(1 << 20, 256), 16, 1 / 8, sz(4096),
                        sz(9000), sz(1000, 0), seed, qseed)
    if idx == 3:
        return Workload("hn_n4m_k8_a1-32", sz(1 << 22, 256), 8, 1 / 32, sz(16384),
                        sz(65536), 0, seed, qseed)
    if idx == 5:
        return Workload("hn_n4m_k16_a1-8_seed", sz(1 << 22, 256), 16, 1 / 8,
                        sz(16384), sz(65536), 0, seed, qseed,
                        extra={"n_anchor": 512, "n_train": sz(200000),
                               "train_seed": seed + 0x200,
                               "anchor_seed": seed + 0x300})
    raise ValueError("workload 4 is a set of databases: use batched_set()")


@dataclass
class BatchedDB:
    n: int
    k: int
    alpha: float
    q: int
    db_seed: int
    q_seed: int

    def db(self) -> np.ndarray:
        return make_db(self.n, self.k, self.alpha, max(1, self.n // 256),
                       self.db_seed)

    def queries(self, db: np.ndarray) -> np.ndarray:
        return make_queries(db, self.k, self.alpha, self.q, 0, self.q_seed)


def batched_set(n_db: int = 64, n_lo: int = 4096, n_hi: int = 1 << 21,
                q_lo: int = 1, q_hi: int = 4096, seed: int = DB_SEED_BASE + 4):
    """Many independent databases: N_d and Q_d log-uniform, K_d in {8, 16} and
    alpha_d in {1/32, 1/8} uniform and independent; clusters N_d / 256."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for t in range(n_db):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        q = int(round(math.exp(rng.uniform(math.log(q_lo), math.log(q_hi)))))
        k = int(rng.choice([8, 16]))
        a = float(rng.choice([1 / 32, 1 / 8]))
        out.append(BatchedDB(n, k, a, q, seed + 0x1000 + t, seed + 0x2000 + t))
    return out
