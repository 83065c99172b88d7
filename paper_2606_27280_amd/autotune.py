"""Autotuner for the scan launch shape (query tiles per wave, entry blocks per
work item) of hn_search_top1.

For a given index, query batch and scan precision it times every candidate
shape with the library's own kernel timing (hn_profile_begin/end: HIP events
around each kernel on the caller's stream), checks that every candidate
returns bit-identical results (the search is deterministic whatever the
shape), and keeps the fastest.  Results are cached in a JSON file keyed by
device name, stream width bucket, precision and the log2 buckets of N and Q.
"""
from __future__ import annotations

import json
import math
import os
import time

QUERY_TILES = (1, 2, 4, 8)
CHUNK_BLOCKS = (0, 16, 32, 64, 128, 256)
MULTI_QUERY_TILES = (1, 2, 4)
MULTI_CHUNK_BLOCKS = (0, 16, 64)


def _bucket(v: int) -> int:
    return int(math.floor(math.log2(max(1, v))))


def default_cache_path() -> str:
    return os.environ.get("HNSEARCH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hnsearch",
                                       "tune.json"))


class Tuner:
    def __init__(self, cache_path: str | None = None):
        self.path = cache_path or default_cache_path()
        self.table = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.table = json.load(f)
            except (OSError, ValueError):
                self.table = {}

    @staticmethod
    def key(device: str, n: int, k: int, precision: str, q: int) -> str:
        return "%s|k%d|%s|n%d|q%d" % (device, k, precision, _bucket(n), _bucket(q))

    def lookup(self, device, n, k, precision, q):
        e = self.table.get(self.key(device, n, k, precision, q))
        return (e["query_tiles"], e["chunk_blocks"]) if e else (0, 0)

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def tune(self, index, queries, precision="fp32", query_tiles=QUERY_TILES,
             chunk_blocks=CHUNK_BLOCKS, reps=3, save=True, log=None):
        """Time every (query_tiles, chunk_blocks) candidate; returns
        (best_shape, table of {shape: ms per search})."""
        import torch

        import paper_2606_27280_amd as hn
        dev_name = torch.cuda.get_device_name(queries.device)
        ref = index.search(queries, precision=precision)
        results = {}
        for qt in query_tiles:
            for cb in chunk_blocks:
                idx, sim = index.search(queries, precision=precision, query_tiles=qt,
                                        chunk_blocks=cb)
                if not (torch.equal(idx, ref[0]) and torch.equal(sim, ref[1])):
                    raise RuntimeError("shape (%d, %d) changed the results" % (qt, cb))
                torch.cuda.synchronize()
                with hn.profile() as p:
                    for _ in range(reps):
                        index.search(queries, precision=precision, query_tiles=qt,
                                     chunk_blocks=cb, out=(idx, sim))
                ms = sum(v["ms"] for v in p.result.values()) / reps
                results[(qt, cb)] = ms
                if log:
                    log("tune %s qt=%d cb=%d: %.4f ms" % (precision, qt, cb, ms))
        best = min(results, key=results.get)
        k = self.key(dev_name, index.n, index.k, precision, queries.shape[0])
        self.table[k] = {"query_tiles": best[0], "chunk_blocks": best[1],
                         "ms": results[best], "when": time.time()}
        if save:
            self.save()
        return best, results

    def tune_multi(self, indexes, q_counts, queries, precision="fp32",
                   query_tiles=MULTI_QUERY_TILES, chunk_blocks=MULTI_CHUNK_BLOCKS, reps=3,
                   save=True, log=None):
        """The same search for a multi-database plan: every candidate shape
        becomes a plan, replayed as a HIP graph and timed with HIP events;
        all must return bit-identical results.  Returns (best, table)."""
        import torch

        import paper_2606_27280_amd as hn
        dev_name = torch.cuda.get_device_name(queries.device)
        ref = None
        results = {}
        for qt in query_tiles:
            for cb in chunk_blocks:
                plan = hn.MultiPlan(indexes, q_counts, precision=precision, query_tiles=qt,
                                    chunk_blocks=cb)
                idx, sim = plan.search(queries, use_graph=True)
                if ref is None:
                    ref = (idx.clone(), sim.clone())
                elif not (torch.equal(idx, ref[0]) and torch.equal(sim, ref[1])):
                    plan.close()
                    raise RuntimeError("shape (%d, %d) changed the results" % (qt, cb))
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    plan.search(queries, use_graph=True, out=(idx, sim))
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / reps
                plan.close()
                results[(qt, cb)] = ms
                if log:
                    log("tune multi %s qt=%d cb=%d: %.4f ms" % (precision, qt, cb, ms))
        best = min(results, key=results.get)
        k = "multi|%s|%s|db%d|q%d" % (dev_name, precision, len(indexes),
                                      _bucket(int(sum(q_counts))))
        self.table[k] = {"query_tiles": best[0], "chunk_blocks": best[1], "ms": results[best],
                         "when": time.time()}
        if save:
            self.save()
        return best, results
