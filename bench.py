"""Benchmark: exact top-1 queries/s of HN branch-and-bound search on one GPU.

Workload (default): N = 1,048,576 clustered HN vectors (4,096 clusters), D =
128, K = 16, alpha = 1/8; Q = 10,000 queries (9,000 perturbed entries, 1,000
fresh random HN vectors), seeded synthetic data standing in for the paper's
descriptors.  One step = one exact search of all Q queries (both scans,
survivor compaction, float64 rescoring, argmax), inputs resident in HBM.

Prints one JSON line with the throughput, the GPU brute-force baseline on the
same queries, the pruned fraction, the dominant kernel's roofline fraction
(kernel time from HIP events recorded on the library's stream during the
timed steps) and the CPU oracle timed on a bounded sample.

Other workloads: --workload 3 (N = 4M, K = 8, alpha = 1/32, Q = 65,536; the
precision form) and --workload 5 (N = 4M, K = 16, alpha = 1/8, Q = 65,536
held-out queries; the seed model is built first, untimed: k-means++ anchors,
labels of 200,000 training queries, training; then the plain two-pass seed,
the learned single pass and the window-only single pass are all timed).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "exact top-1 queries/s @N=1M,K=16,α=1/8 vs GPU brute force; % entries pruned"
PEAK = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "fp32_mfma_tflops": 157.3,
    "bf16_mfma_tflops": 2500.0,
    "fp8_mfma_tflops": 5000.0,
}


ARGS = None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--bf-steps", type=int, default=3)
    ap.add_argument("--no-bruteforce", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip timing the other scan precisions")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--query-tiles", type=int, default=0)
    ap.add_argument("--chunk-blocks", type=int, default=0)
    ap.add_argument("--seed", default=None, choices=["plain", "learned", "window"],
                    help="timed seed form (default: learned for workload 5, else plain)")
    ap.add_argument("--epochs", type=int, default=4, help="seed-model training epochs")
    ap.add_argument("--batch", type=int, default=1024, help="seed-model training batch")
    ap.add_argument("--lr", type=float, default=2e-3)
    return ap.parse_args()


def build_seed_model(hn, ix, w, db, dev, torch):
    """Anchors (k-means++), labels (exact GPU search), training, install.
    Returns a report dict with the time of each step."""
    import hn_inputs
    rep = {}
    t0 = time.perf_counter()
    u = torch.from_numpy(hn_inputs.uniform_draws(w.extra["n_anchor"],
                                                 w.extra["anchor_seed"])).to(dev)
    anchors = ix.kmeanspp(w.extra["n_anchor"], u)
    torch.cuda.synchronize()
    rep["kmeanspp_s"] = round(time.perf_counter() - t0, 3)
    log("anchors: %.2f s" % rep["kmeanspp_s"])
    qt = w.train_queries(db)
    d_qt = torch.from_numpy(qt).to(dev)
    t0 = time.perf_counter()
    labels = ix.seed_labels(anchors, d_qt)
    torch.cuda.synchronize()
    rep["labels_s"] = round(time.perf_counter() - t0, 3)
    log("labels of %d training queries: %.2f s" % (len(qt), rep["labels_s"]))
    params = torch.from_numpy(hn_inputs.mlp_init(w.extra["train_seed"] + 1)).to(dev)
    t0 = time.perf_counter()
    losses = hn.seed_train(params, d_qt, labels, batch=ARGS.batch, epochs=ARGS.epochs,
                           lr=ARGS.lr)
    torch.cuda.synchronize()
    rep["train_s"] = round(time.perf_counter() - t0, 3)
    ls = losses.cpu().numpy()
    steps_per_epoch = max(1, len(ls) // max(1, ARGS.epochs))
    rep.update({"train_queries": len(qt), "epochs": ARGS.epochs, "batch": ARGS.batch,
                "lr": ARGS.lr, "loss_first_epoch": round(float(ls[:steps_per_epoch].mean()), 4),
                "loss_last_epoch": round(float(ls[-steps_per_epoch:].mean()), 4),
                "anchors": w.extra["n_anchor"]})
    log("training: %.2f s, loss %.3f -> %.3f" % (rep["train_s"], rep["loss_first_epoch"],
                                                 rep["loss_last_epoch"]))
    ix.set_seed_model(params, anchors)
    return rep


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def cpu_baseline(db, qs, k, alpha, budget_s):
    """The CPU oracle's branch-and-bound (Algorithm 1, float64) on the same
    database, over consecutive query batches until about budget_s seconds of
    work have been timed (or every query is done)."""
    import oracle
    threads = min(16, oracle.default_threads())
    done, spent, batch = 0, 0.0, max(threads, 16)
    while done < len(qs) and spent < budget_s:
        n = min(batch, len(qs) - done)
        t0 = time.perf_counter()
        oracle.bnb_top1(db, qs[done:done + n], k, alpha, threads=threads)
        spent += time.perf_counter() - t0
        done += n
        batch = min(4 * batch, max(threads, int(n * budget_s / max(spent, 1e-3))))
    return {"value": done / spent, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d queries, full database (N=%d), float64 "
                      "branch-and-bound (Algorithm 1), %.1f s" % (done, len(qs), len(db), spent)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import hn_inputs
    import paper_2606_27280_amd as hn
    from paper_2606_27280_amd import accounting as acc

    global ARGS
    ARGS = args
    w = hn_inputs.workload(args.workload)
    seed = args.seed or ("learned" if args.workload == 5 else "plain")
    log("generating %s (N=%d, K=%d, alpha=%g)" % (w.name, w.n, w.k, w.alpha))
    db = w.db()
    qs = w.queries(db)
    dev = torch.device("cuda:0")
    d_db = torch.from_numpy(db).to(dev)
    d_q = torch.from_numpy(qs).to(dev)
    Q = len(qs)
    log("building index")
    ix = hn.Index(d_db, w.k, w.alpha)
    idx = torch.empty(Q, dtype=torch.int64, device=dev)
    sim = torch.empty(Q, dtype=torch.float64, device=dev)
    seed_report = None
    if args.workload == 5 or seed == "learned":
        seed_report = build_seed_model(hn, ix, w, db, dev, torch)
    kw = dict(precision=args.precision, query_tiles=args.query_tiles,
              chunk_blocks=args.chunk_blocks, seed=seed)

    def step():
        ix.search(d_q, out=(idx, sim), **kw)

    log("warmup %d + timed %d steps (%s, %s seed)" % (args.warmup, args.steps, args.precision,
                                                     seed))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    with hn.profile() as prof:
        sec, wall = timed(step, args.steps, 0, torch)
    qps = Q * args.steps / sec
    log("HN %s: %.3f ms/step, %.0f queries/s (wall %.3f s)" % (
        args.precision, 1e3 * sec / args.steps, qps, wall))

    # the dominant kernel and its roofline (algorithmic flops of one pass)
    kernels = {k: {"avg_ms": v["ms"] / v["launches"], "launches": v["launches"],
                   "total_ms": v["ms"]} for k, v in prof.result.items()}
    dom = max((k for k in kernels if k.startswith("scan_")), key=lambda k: kernels[k]["total_ms"])
    # one step scans all Q queries once per scan kind, in one launch or (the
    # single-pass forms) in query batches: the work per launch is the step's
    # work divided by the launches per step
    per_step = kernels[dom]["launches"] / args.steps
    avg_s = kernels[dom]["avg_ms"] / 1e3
    flops = acc.scan_flops(Q, w.n, w.k) / per_step
    peak = PEAK[{"f32": "fp32_mfma_tflops", "bf16": "bf16_mfma_tflops",
                 "fp8": "fp8_mfma_tflops"}[dom.rsplit("_", 1)[1]]]
    achieved = flops / avg_s / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "algorithmic": "2*Q*N*K / %d launches per step = %.4g flop per launch" % (
                    per_step, flops)}

    # exactness of this run against the GPU exhaustive search, pruned fraction
    _, _, aux = ix.search(d_q, aux=True, **kw)
    surv = aux["survivors"].double()
    pruned_pct = float(100.0 * (1.0 - surv.mean() / w.n))
    out = {}
    if not args.no_bruteforce:
        bidx = torch.empty(Q, dtype=torch.int64, device=dev)
        bsim = torch.empty(Q, dtype=torch.float64, device=dev)

        def bf_step():
            hn.bruteforce_top1(d_db, d_q, out=(bidx, bsim))

        log("brute force: %d steps" % args.bf_steps)
        bf_step()
        torch.cuda.synchronize()
        with hn.profile() as bprof:
            bsec, _ = timed(bf_step, args.bf_steps, 0, torch)
        bqps = Q * args.bf_steps / bsec
        exact = bool(torch.equal(bidx, idx) and torch.equal(bsim, sim))
        bscan = bprof.result.get("scan_window_f32", {"ms": 0.0, "launches": 1})
        bavg = bscan["ms"] / bscan["launches"] / 1e3
        out["bruteforce"] = {
            "queries_per_s": round(bqps, 1), "ms_per_step": round(1e3 * bsec / args.bf_steps, 3),
            "scan_tflops": round(acc.bruteforce_flops(Q, w.n) / bavg / 1e12, 2) if bavg else None,
            "precision": "fp32 scan + fp64 near-tie rescoring"}
        out["speedup_vs_bruteforce"] = round(qps / bqps, 2)
        out["exact_vs_bruteforce"] = exact
        log("brute force: %.0f queries/s; speed-up %.2fx; exact=%s" % (bqps, qps / bqps, exact))

    forms = {}
    if not args.no_forms:
        for prec in ("fp32", "bf16", "fp8"):
            if prec == args.precision:
                forms[prec] = round(qps, 1)
                continue
            s2, _ = timed(lambda: ix.search(d_q, out=(idx, sim), precision=prec, seed=seed),
                          args.steps, 2, torch)
            forms[prec] = round(Q * args.steps / s2, 1)
        log("forms: %s" % forms)
    seed_forms = {}
    if seed_report is not None:
        # every seed form at the timed precision: queries/s, first-pass
        # survivors per query, exactness against the timed form
        for sf in ("plain", "learned", "window"):
            log("seed form %s" % sf)
            kws = dict(kw, seed=sf)
            i2, s2_, a2 = ix.search(d_q, aux=True, **kws)
            same = bool(torch.equal(i2, idx) and torch.equal(s2_, sim))
            t2, _ = timed(lambda: ix.search(d_q, out=(i2, s2_), **kws), args.steps, 1, torch)
            seed_forms[sf] = {"queries_per_s": round(Q * args.steps / t2, 1),
                              "survivors_per_query": round(float(
                                  a2["survivors"].double().mean()), 2),
                              "mean_seed_sim": round(float(torch.nan_to_num(
                                  a2["seed_sim"], neginf=float("nan")).nanmean()), 5)
                              if sf != "window" else None,
                              "same_result": same}
        log("seed forms: %s" % seed_forms)

    res = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": 128, "k": w.k, "alpha": w.alpha,
                   "queries": Q, "query_mix": "%d perturbed + %d fresh" % (w.n_perturbed, w.n_fresh),
                   "clusters": w.n_clusters, "precision": args.precision, "seed": seed,
                   "rescoring": "f64"},
        "pruned_pct": round(pruned_pct, 4),
        "survivors_per_query": round(float(surv.mean()), 2),
        "roofline": roofline,
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 4), "launches": v["launches"]}
                    for k, v in kernels.items()},
        "forms_queries_per_s": forms,
    }
    res.update(out)
    if seed_report is not None:
        res["seed_model"] = seed_report
        res["seed_forms"] = seed_forms
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(db, qs, w.k, w.alpha, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    ix.close()


if __name__ == "__main__":
    main()
