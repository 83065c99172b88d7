"""Algorithmic byte and operation counts for HN search (no GPU needed).

Section 6 of the paper prices the method by the bytes each phase streams and
by multiply-add counts ("FLOPs" there: N x 128 for a full scan, N x K for the
major scan, and (D - K) per fully evaluated entry).  The same counts price the
GPU kernels: a roofline fraction divides these algorithmic figures, never the
traffic a kernel happens to generate, by the measured kernel time.
"""
from __future__ import annotations

D = 128


def major_bytes(n: int, k: int, elem_bytes: int = 4) -> int:
    """Bytes of the contiguous major array [N][K] (Section 6.1)."""
    return n * k * elem_bytes


def minor_bytes(n: int, k: int, d: int = D, elem_bytes: int = 4) -> int:
    """Bytes of the minor array [N][D-K] (Section 6.2)."""
    return n * (d - k) * elem_bytes


def full_bytes(n: int, d: int = D, elem_bytes: int = 4) -> int:
    """Bytes of the full descriptor bank [N][D] (Section 6.1)."""
    return n * d * elem_bytes


def score_buffer_bytes(n: int, elem_bytes: int = 4) -> int:
    """Phase-1 score buffer, one score per entry (Section 3.3 note, 6.2)."""
    return n * elem_bytes


def macs_full(n: int, d: int = D) -> int:
    """Multiply-adds of one exhaustive query (the paper's 'N x 128')."""
    return n * d


def macs_phase1(n: int, k: int) -> int:
    """Multiply-adds of the major scan for one query ('N x K')."""
    return n * k


def macs_phase2(n_eval: int, k: int, d: int = D) -> int:
    """Multiply-adds of the minor completions for n_eval entries."""
    return n_eval * (d - k)


# ---------------------------------------------------------------- GPU path

def scan_flops(q: int, n: int, k: int) -> int:
    """Algorithmic flops of one major-prefix pass over Q queries: 2 Q N K."""
    return 2 * q * n * k


def scan_stream_bytes(n: int, k: int, elem_bytes: int) -> int:
    """Bytes of one read of the major stream (the pass's HBM minimum)."""
    return n * k * elem_bytes


def bruteforce_flops(q: int, n: int, d: int = D) -> int:
    """Algorithmic flops of an exhaustive FP32 scan: 2 Q N D."""
    return 2 * q * n * d


def rescore_bytes(n_pairs: int, d: int = D) -> int:
    """Row bytes gathered to rescore n_pairs (query, entry) survivors."""
    return n_pairs * d * 4


def rescore_flops(n_pairs: int, d: int = D) -> int:
    return 2 * n_pairs * d
