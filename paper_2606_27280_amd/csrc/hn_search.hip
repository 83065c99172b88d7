// Exact top-1 search on one database (Algorithm 1 on the GPU), the survivor
// filter, the score buffer and the exhaustive baseline: host orchestration of
// the pipeline kernels (hn_pipeline.h) and the scans (hn_scan.h).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "hn_pipeline.h"

namespace hn {
namespace {

// Everything one search call needs on the device.
struct Work {
    Plan plan;
    int cfg = 0;
    int precision = HN_PREC_FP32;
    int width = 0;
    Plan seed_plan;  // the argmax (seed) scan
    int seed_cfg = 0;
    int seed_precision = HN_PREC_BF16;  // HN_PREC_BF16 or HN_PREC_FP32
    int seed_width = 0;
    Arena *fixed = nullptr;  // caller-provided scratch (no allocation), or NULL
    int shape = 16;  // tile shape of the argmax scan (16 or 32): decodes its groups
    const void *stream_x = nullptr;
    float *op32 = nullptr;
    uint16_t *op16 = nullptr;
    uint8_t *op8 = nullptr;
    int8_t *opi = nullptr;
    QNorm *qn = nullptr;
    float *part_val = nullptr;
    int32_t *part_idx = nullptr;
    float *thr = nullptr, *thr32 = nullptr;
    int64_t *seed_idx = nullptr;
    double *seed_sim = nullptr, *slack = nullptr;
    unsigned long long *best_key = nullptr, *counter = nullptr, *n_flagged = nullptr;
    int32_t *best_idx = nullptr, *cnt = nullptr, *qflag = nullptr;
    int2 *pairs = nullptr;
    double *psim = nullptr;
    unsigned *work = nullptr;  // kWorkWords scan counters (see kWorkWords)
    int *redo = nullptr;       // [n_items] items to re-run
    int64_t cap = 0;
    // single-pass forms
    double *win = nullptr;
    float *win_scan = nullptr, *init_best = nullptr, *thr_ref = nullptr, *pair_val = nullptr;
    float *win_max = nullptr;
    int32_t *win_arg = nullptr;
    double *lower = nullptr;
    int64_t *lower_idx = nullptr;
    SeedArgs seed_args;  // as the seed kernel ran (the single pass's refinement reuses it)
};

const void *operands_of(const Work &W) {
    return W.precision == HN_PREC_FP32   ? (const void *)W.op32
           : W.precision == HN_PREC_BF16 ? (const void *)W.op16
           : W.precision == HN_PREC_FP8  ? (const void *)W.op8
                                         : (const void *)W.opi;
}

void launch_prep(const hn_index *ix, const float *queries, int64_t q, int64_t q_pad, Work &W,
                 hipStream_t s) {
    PrepArgs P;
    P.q = queries;
    P.nq = q;
    P.q_pad = q_pad;
    P.k = ix->k;
    P.w32 = ix->kp;
    P.w16 = ix->kb;
    P.w8 = ix->k8;
    P.op32 = W.op32;
    P.op16 = W.op16;
    P.op8 = W.op8;
    P.opi = W.opi;
    P.qn = W.qn;
    P.work = W.work;
    ProfScope prof_(s, "prep_queries");
    hipLaunchKernelGGL(prep_queries, dim3(blocks_for(q_pad, 4)), dim3(256), 0, s, P);
}

int validate_opts(const hn_index *ix, const hn_search_opts *o) {
    if (!o) return HN_OK;
    int rc = check_precision(ix, o->precision);
    if (rc) return rc;
    if (o->seed != HN_SEED_PLAIN && o->seed != HN_SEED_LEARNED && o->seed != HN_SEED_WINDOW)
        return fail(HN_ERR_INVALID_ARG, "seed %d is not a seed mode", o->seed);
    if (o->seed == HN_SEED_LEARNED && !ix->seed_w)
        return fail(HN_ERR_INVALID_ARG, "the learned seed needs a model (hn_set_seed_model)");
    if (o->query_tiles != 0 && o->query_tiles != 1 && o->query_tiles != 2 && o->query_tiles != 4 &&
        o->query_tiles != 8)
        return fail(HN_ERR_INVALID_ARG, "query_tiles must be 0, 1, 2, 4 or 8");
    if (o->chunk_blocks < 0) return fail(HN_ERR_INVALID_ARG, "chunk_blocks must be >= 0");
    if (o->survivor_cap < 0) return fail(HN_ERR_INVALID_ARG, "survivor_cap must be >= 0");
    if (!(o->beta < 0.0 || (o->beta >= 0.0 && o->beta <= ix->alpha)))
        return fail(HN_ERR_INVALID_ARG, "beta must be < 0 (exact) or in [0, alpha]");
    if (o->seed_scan != HN_SEED_SCAN_BF16 && o->seed_scan != HN_SEED_SCAN_FP32)
        return fail(HN_ERR_INVALID_ARG, "seed_scan must be HN_SEED_SCAN_BF16 or HN_SEED_SCAN_FP32");
    return HN_OK;
}

// Launch shapes of a search: the filter (or window) scan and the argmax
// (seed) scan.  The seed scan runs on the bf16 copy unless opts.seed_scan
// asks for float32: the seed only has to be a real entry with a near-maximal
// score (its float64 sim is the bound), and bf16 contracts four times faster
// than float32 on the matrix cores.
int plan_stage(const hn_index *ix, int64_t q, const hn_search_opts &o, Work &W, bool window,
               int topk) {
    W.precision = o.precision;
    W.width = stream_width(ix, W.precision);
    W.stream_x = stream_of(ix, W.precision);
    const TileInfo ti = tile_info(W.precision, W.width);
    W.cfg = pick_cfg(q, ti.cols, ti.cost, o.query_tiles);
    if (W.cfg < 0)
        return fail(HN_ERR_INVALID_ARG, "query_tiles=%d is not available for this width",
                    o.query_tiles);
    // With one query block every item holds the same queries and costs the
    // same: two rounds of the persistent grid (fewer, longer items, less
    // per-item start-up against the stream) instead of about 8192 items.
    const int64_t fslots = scan_slots(W.precision, window ? kWindow : kFilter, W.width, W.cfg);
    const int64_t one_qb = (int64_t)kCfgNQ[W.cfg] * kCfgWQ[W.cfg] * ti.cols;
    W.plan = make_plan(ix->n, q, W.cfg, o.chunk_blocks, ti.rows, ti.cols,
                       q <= one_qb && fslots >= kXcds ? 2 * fslots : 8192, fslots);
    W.seed_precision = o.seed_scan == HN_SEED_SCAN_FP32 ? HN_PREC_FP32 : HN_PREC_BF16;
    W.seed_width = stream_width(ix, W.seed_precision);
    const TileInfo tis = tile_info(W.seed_precision, W.seed_width);
    W.seed_cfg = pick_cfg(q, tis.cols, tis.cost, o.query_tiles);
    if (W.seed_cfg < 0)
        return fail(HN_ERR_INVALID_ARG, "query_tiles=%d is not available for this width",
                    o.query_tiles);
    // top-k seeds take the best of up to 2 topk chunks: plan at least that many.
    // One query block: two rounds of the grid as for the filter plan, which
    // also shortens the seed kernel's walk over the per-chunk partials (one
    // per chunk and query).
    const int64_t sslots = scan_slots(W.seed_precision, kArgmax, W.seed_width, W.seed_cfg);
    const int64_t one_sqb = (int64_t)kCfgNQ[W.seed_cfg] * kCfgWQ[W.seed_cfg] * tis.cols;
    W.seed_plan = make_plan(ix->n, q, W.seed_cfg, o.chunk_blocks, tis.rows, tis.cols,
                            q <= one_sqb && sslots >= kXcds ? 2 * sslots : 8192, sslots,
                            topk > 1 ? 2 * (int64_t)topk : 1);
    W.shape = tis.rows;
    return HN_OK;
}

// Scratch bytes of one search besides its pair list, and per pair.
size_t stage_bytes(const hn_index *ix, int64_t q, const Work &W, bool window,
                   size_t *per_pair) {
    const Plan &p = W.plan, &sp = W.seed_plan;
    const int64_t qp = std::max(p.q_pad, sp.q_pad);
    const size_t part = std::max((size_t)p.n_chunks * p.q_pad, (size_t)sp.n_chunks * sp.q_pad);
    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) { bytes += (count * sz + 255) & ~size_t(255); };
    add(qp * ix->kp, 4);
    add(qp * ix->kb, 2);
    add(qp * ix->k8, 1);
    add(qp, sizeof(QNorm));
    add(part, 4);
    add(part, 4);
    add(qp, 4);
    add(q, 4);
    add(q, 8);
    add(q, 8);
    add(q, 8);
    add(q, 8);
    add(q, 4);
    add(q, 4);
    add(q, 4);
    add(4, 8);
    add(kWorkWords, 4);
    add(p.n_items, 4);
    if (window) {
        add(qp, 8);
        add(qp, 4);
        add(qp, 4);
        add(q, 4);
        add(q, 8);
        add(q, 8);
        add(q, 4);
        add(q, 4);
    }
    // pairs (int2), their float64 sims and, with the window, their scores;
    // plus the rounding of each of those arrays to 256 bytes
    *per_pair = sizeof(int2) + 8 + (window ? 4 : 0);
    return bytes + 3 * 256;
}

// Prepare queries, run the plain-seed pass and compute thresholds.  With
// `lower` the seed pass is skipped and L (and its entry, lower_idx, if not
// NULL) is taken from the caller.  `window`: also the single-pass window
// (W.win, W.win_scan, W.init_best) and the pair values.  Scratch comes from
// W.fixed when set (its capacity checked), else from the stream's arena.
int stage_seed(const hn_index *ix, const float *queries, int64_t q, const hn_search_opts &o,
               const double *lower, const int64_t *lower_idx, int64_t cap, Work &W,
               hipStream_t s, bool window = false, int topk = 0) {
    int rc = plan_stage(ix, q, o, W, window, topk);
    if (rc) return rc;
    const Plan &sp = W.seed_plan;
    const int64_t qp = std::max(W.plan.q_pad, sp.q_pad);
    const size_t part =
        std::max((size_t)W.plan.n_chunks * W.plan.q_pad, (size_t)sp.n_chunks * sp.q_pad);
    W.cap = cap;
    size_t per_pair = 0;
    const size_t bytes = stage_bytes(ix, q, W, window, &per_pair) + (size_t)cap * per_pair;
    Arena *ar = W.fixed;
    if (ar) {
        if (bytes > ar->cap)
            return fail(HN_ERR_INVALID_ARG, "search needs %zu bytes of scratch, %zu available",
                        bytes, ar->cap);
        ar->used = 0;
    } else {
        rc = arena_for((void *)s, bytes, &ar);
        if (rc) return rc;
    }
    W.op32 = ar->take<float>(qp * ix->kp);
    W.op16 = ar->take<uint16_t>(qp * ix->kb);
    if (W.precision != HN_PREC_FP32 && W.seed_precision != HN_PREC_FP32) W.op32 = nullptr;
    W.op8 = W.precision == HN_PREC_FP8 ? ar->take<uint8_t>(qp * ix->k8) : nullptr;
    W.opi = W.precision == HN_PREC_INT8 ? ar->take<int8_t>(qp * ix->k8) : nullptr;
    W.qn = ar->take<QNorm>(qp);
    W.part_val = ar->take<float>(part);
    W.part_idx = ar->take<int32_t>(part);
    W.thr = ar->take<float>(qp);
    W.thr32 = ar->take<float>(q);
    W.seed_idx = ar->take<int64_t>(q);
    W.seed_sim = ar->take<double>(q);
    W.slack = ar->take<double>(q);
    W.best_key = ar->take<unsigned long long>(q);
    W.best_idx = ar->take<int32_t>(q);
    W.cnt = ar->take<int32_t>(q);
    W.qflag = ar->take<int32_t>(q);
    W.counter = ar->take<unsigned long long>(4);
    W.n_flagged = W.counter + 1;
    W.work = ar->take<unsigned>(kWorkWords);
    W.redo = ar->take<int>(W.plan.n_items);
    if (window) {
        W.win = ar->take<double>(qp);
        W.win_scan = ar->take<float>(qp);
        W.init_best = ar->take<float>(qp);
        W.thr_ref = ar->take<float>(q);
        W.lower = ar->take<double>(q);
        W.lower_idx = ar->take<int64_t>(q);
        W.win_max = ar->take<float>(q);
        W.win_arg = ar->take<int32_t>(q);
    }
    W.pairs = ar->take<int2>(cap);
    W.psim = ar->take<double>(cap);
    if (window) W.pair_val = ar->take<float>(cap);

    launch_prep(ix, queries, q, qp, W, s);
    HN_HIP(hipGetLastError());
    if (window) {
        if (o.seed == HN_SEED_LEARNED) {
            rc = learned_seed(ix, queries, q, W.lower, W.lower_idx, s);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(fill_lower, dim3(blocks_for(q)), dim3(256), 0, s, W.lower,
                               W.lower_idx, q);
        }
        lower = W.lower;
        lower_idx = W.lower_idx;
    }

    if (!lower) {
        ScanArgs A;
        memset(&A, 0, sizeof A);
        const bool f32 = W.seed_precision == HN_PREC_FP32;
        A.x = f32 ? (const void *)ix->major32 : (const void *)ix->major16;
        A.x_stride = W.seed_width;
        A.qs = f32 ? (const void *)W.op32 : (const void *)W.op16;
        A.q_stride = W.seed_width;
        A.n = ix->n;
        A.n_blocks = sp.n_blocks;
        A.chunk_blocks = sp.chunk_blocks;
        A.n_chunks = sp.n_chunks;
        A.n_qb = sp.n_qb;
        A.n_items = sp.n_items;
        A.q_count = (int32_t)q;
        A.q_pad = (int32_t)sp.q_pad;
        A.part_val = W.part_val;
        A.part_idx = W.part_idx;
        A.redo = W.redo;
        A.redo_count = W.work + 2 * kXcds;
        rc = launch_scan<kArgmax>(W.seed_precision, W.seed_width, W.seed_cfg, sp, A, s);
        if (rc) return rc;
    }

    SeedArgs S;
    memset(&S, 0, sizeof S);
    S.part_val = W.part_val;
    S.part_idx = W.part_idx;
    S.n_chunks = sp.n_chunks;
    S.q_pad = (int32_t)qp;
    S.part_ld = (int32_t)sp.q_pad;
    S.topk = topk;
    S.shape = W.shape;
    S.group_size = (W.shape == 16 ? 4 : 16) * kArgSpan;
    S.queries = queries;
    S.q = q;
    S.rows = ix->rows;
    S.n = ix->n;
    S.k = ix->k;
    S.alpha = ix->alpha;
    S.beta = o.beta < 0.0 ? ix->alpha : o.beta;
    S.mu_major = ix->mu_major;
    S.mu_minor = ix->mu_minor;
    S.mu_full = ix->mu_full;
    scan_slack(ix, W.precision, S);
    S.lower = lower;
    S.lower_idx = lower_idx;
    if (window) {
        S.win = W.win;
        S.win_scan = W.win_scan;
        S.init_best = W.init_best;
        S.bound_mu = W.precision == HN_PREC_FP32   ? ix->mu_major
                     : W.precision == HN_PREC_BF16 ? ix->mu_major16
                     : W.precision == HN_PREC_FP8  ? ix->mu_major8
                                                   : ix->mu_major_i8;
    }
    S.qn = W.qn;
    S.thr = W.thr;
    S.thr32 = W.precision == HN_PREC_FP32 ? nullptr : W.thr32;
    S.seed_idx = W.seed_idx;
    S.seed_sim = W.seed_sim;
    S.slack = W.slack;
    S.best_key = W.best_key;
    S.best_idx = W.best_idx;
    S.cnt = W.cnt;
    S.qflag = W.qflag;
    S.counter = W.counter;
    {
        ProfScope prof_(s, "seed");
        hipLaunchKernelGGL(seed_kernel, dim3(blocks_for(qp, 4)), dim3(256), 0, s, S);
    }
    W.seed_args = S;
    HN_HIP(hipGetLastError());
    return HN_OK;
}

ScanArgs filter_args(const hn_index *ix, const Work &W, int64_t q, int2 *pairs, int64_t cap) {
    const Plan &p = W.plan;
    ScanArgs A;
    memset(&A, 0, sizeof A);
    A.x = W.stream_x;
    A.x_stride = W.width;
    A.qs = operands_of(W);
    A.q_stride = W.width;
    A.n = ix->n;
    A.n_blocks = p.n_blocks;
    A.chunk_blocks = p.chunk_blocks;
    A.n_chunks = p.n_chunks;
    A.n_qb = p.n_qb;
    A.n_items = p.n_items;
    A.q_count = (int32_t)q;
    A.q_pad = (int32_t)p.q_pad;
    A.thr = W.thr;
    A.pairs = pairs;
    A.counter = W.counter;
    A.cap = cap;
    A.qflag = W.qflag;
    A.redo = W.redo;
    A.redo_count = W.work + 2 * kXcds + 1;
    // dynamic item order only where items differ in cost: with one query
    // block every item holds the same queries and the static order is even
    A.item_ctr = p.n_qb > 1 ? W.work + kXcds : nullptr;
    return A;
}

__global__ __launch_bounds__(256) void scale_scores(float *scores, int64_t q, int64_t n,
                                                   const QNorm *qn, float scale_x, int int8) {
    const int64_t total = q * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256)
        scores[t] *= (int8 ? qn[t / n].sci : qn[t / n].sc8) * scale_x;
}


}  // namespace
}  // namespace hn

using namespace hn;

namespace hn {
namespace {

// Survivor-list budget per query of the single-pass forms (the window keeps
// more pairs than the two-pass threshold) and the query batch that fits it.
__global__ void fill_i32(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

int64_t window_per_query(int64_t n) { return std::max<int64_t>(8192, n / 32); }
int64_t window_batch(int64_t n) {
    return std::max<int64_t>(256, ((int64_t)1 << 29) / window_per_query(n));
}

// Queries whose survivor pairs did not all fit the list, collected for a
// second pass instead of the exhaustive fallback: the best candidate each one
// reached (a real entry, so its sim is an admissible lower bound) becomes its
// seed for a plain filter pass.
struct Overflow {
    int32_t *list = nullptr;      // [q] positions in the batch
    double *lower = nullptr;      // [q] best sim reached
    int64_t *lower_idx = nullptr; // [q] its entry (-1: none)
    unsigned long long *count = nullptr;
    int64_t n = 0;                // host copy of *count after the batch
    int64_t pairs = 0;            // the batch's survivor pairs, stored or not
};

__global__ __launch_bounds__(256) void collect_overflow(const int32_t *qflag, const QNorm *qn,
                                                        const unsigned long long *best_key,
                                                        const int32_t *best_idx, int64_t q,
                                                        Overflow O) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= q || !qflag[i] || qn[i].bad) return;
    const unsigned long long pos = atomicAdd(O.count, 1ull);
    const unsigned long long k = best_key[i];
    const bool any = k != 0ull && best_idx[i] != kIdxNone;
    O.list[pos] = (int32_t)i;
    O.lower[pos] = any ? sim_of_key(k) : -INFINITY;
    O.lower_idx[pos] = any ? (int64_t)best_idx[i] : -1;
}

__global__ void gather_queries(const float *__restrict__ q, const int32_t *__restrict__ list,
                               int64_t n, float *__restrict__ out) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n * kDim;
         t += (int64_t)gridDim.x * 256)
        out[t] = q[(int64_t)list[t / kDim] * kDim + t % kDim];
}

__global__ void scatter_results(const int32_t *__restrict__ list, int64_t n,
                                const int64_t *__restrict__ idx, const double *__restrict__ sim,
                                int64_t *__restrict__ out_idx, double *__restrict__ out_sim) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * 256) {
        out_idx[list[j]] = idx[j];
        out_sim[list[j]] = sim[j];
    }
}

// One batch of queries through the whole pipeline.  lower_in: the plain
// pipeline with given seeds (no argmax scan).  ov: collect the overflowing
// queries instead of finishing them with the exhaustive fallback.
int search_batch(const hn_index *ix, const float *queries, int64_t q, int64_t *out_idx,
                 double *out_sim, const hn_search_opts &o, const hn_search_aux *aux,
                 hn_search_stats *stats, hipStream_t s, const double *lower_in = nullptr,
                 const int64_t *lower_idx_in = nullptr, Overflow *ov = nullptr,
                 Arena *fixed = nullptr) {
    const bool single = o.seed != HN_SEED_PLAIN && !lower_in;
    const int64_t cap =
        o.survivor_cap > 0
            ? o.survivor_cap
            : (single ? std::min<int64_t>(std::max<int64_t>(q * window_per_query(ix->n), 1 << 20),
                                          (int64_t)1 << 29)
                      : default_cap(ix->n, q));
    Work W;
    W.fixed = fixed;
    int rc = stage_seed(ix, queries, q, o, lower_in, lower_idx_in, cap, W, s, single);
    if (rc) return rc;
    ScanArgs A = filter_args(ix, W, q, W.pairs, cap);
    // must match the tiles compiled with kFused (every float32, bf16 and int8
    // tile)
    const bool fused = W.precision != HN_PREC_FP8;
    if (single) {
        A.thr = W.win_scan;
        A.init_best = W.init_best;
        A.pair_val = W.pair_val;
        A.part_val = W.part_val;
        rc = launch_scan<kWindow>(W.precision, W.width, W.cfg, W.plan, A, s);
        if (rc) return rc;
        ProfScope prof_(s, "win_threshold");
        hipLaunchKernelGGL(win_threshold, dim3(blocks_for(q, 4)), dim3(256), 0, s, W.part_val,
                           W.plan.n_chunks, (int32_t)W.plan.q_pad, q, W.win, W.thr, W.thr_ref,
                           W.win_max, W.win_arg);
        // rescore the entry of each query's final maximum and raise the
        // re-filter threshold to the plain seed's threshold at its sim
        hipLaunchKernelGGL(win_argmax, dim3(2048), dim3(256), 0, s, W.pairs, W.pair_val,
                           W.counter, cap, W.win_max, W.win_arg);
        hipLaunchKernelGGL(win_refine, dim3(blocks_for(q)), dim3(256), 0, s, W.seed_args,
                           W.win_max, W.win_arg, W.thr_ref);
    } else if (fused) {
        // float32, bf16 and int8: rescoring fused into the filter's flushes
        // (the scan is bound by its matrix-core work or its epilogue and
        // leaves HBM idle, so the row gathers of the survivors ride along,
        // hidden behind the other waves' scanning); fp8 (thousands of
        // re-check rejects per query) keeps the separate re-check.
        A.psim = W.psim;
        A.best_key = W.best_key;
        A.cnt = ((aux && aux->survivors) || stats) ? W.cnt : nullptr;
        A.rs_queries = queries;
        A.rs_rows = ix->rows;
        if (W.precision != HN_PREC_FP32) {
            A.rs_major32 = ix->major32;
            A.rs_thr32 = W.thr32;
            A.rs_kp = ix->kp;
            A.rs_k = ix->k;
        }
        rc = launch_scan<kFilter>(W.precision, W.width, W.cfg, W.plan, A, s);
        if (rc) return rc;
    } else {
        rc = launch_scan<kFilter>(W.precision, W.width, W.cfg, W.plan, A, s);
        if (rc) return rc;
    }

    RescoreArgs R;
    memset(&R, 0, sizeof R);
    R.pairs = W.pairs;
    R.counter = W.counter;
    R.cap = cap;
    R.queries = queries;
    R.rows = ix->rows;
    R.major32 = ix->major32;
    R.kp = ix->kp;
    R.k = ix->k;
    R.thr32 = W.thr32;
    R.psim = W.psim;
    R.best_key = W.best_key;
    R.best_idx = W.best_idx;
    R.cnt = W.cnt;
    R.seed_idx = W.seed_idx;
    R.seed_sim = W.seed_sim;
    R.q = q;
    R.count = (aux && aux->survivors) || stats;
    const unsigned rgrid = 2048;
    if (single) {
        R.pair_val = W.pair_val;
        R.thr32 = W.thr_ref;
        ProfScope prof_(s, "rescore_window");
        hipLaunchKernelGGL(rescore_kernel<2>, dim3(rgrid), dim3(256), 0, s, R);
    } else if (!fused && W.precision == HN_PREC_FP32) {
        ProfScope prof_(s, "rescore");
        hipLaunchKernelGGL(rescore_kernel<0>, dim3(rgrid), dim3(256), 0, s, R);
    } else if (!fused) {
        ProfScope prof_(s, "rescore_recheck");
        hipLaunchKernelGGL(rescore_kernel<1>, dim3(rgrid), dim3(256), 0, s, R);
    }
    {
        ProfScope prof_(s, "tie");
        hipLaunchKernelGGL(tie_kernel, dim3(rgrid), dim3(256), 0, s, R);
    }

    FallbackArgs F;
    memset(&F, 0, sizeof F);
    F.qflag = W.qflag;
    F.qn = W.qn;
    F.queries = queries;
    F.rows = ix->rows;
    F.q = q;
    F.n = ix->n;
    F.k = ix->k;
    F.full = 0;
    F.beta = o.beta < 0.0 ? ix->alpha : o.beta;
    F.alpha = ix->alpha;
    F.mu_major = ix->mu_major;
    F.mu_minor = ix->mu_minor;
    F.mu_full = ix->mu_full;
    F.seed_sim = W.seed_sim;
    F.best_key = W.best_key;
    F.best_idx = W.best_idx;
    F.cnt = W.cnt;
    if (ov) {
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, ov->count, 1);
        hipLaunchKernelGGL(collect_overflow, dim3(blocks_for(q)), dim3(256), 0, s, W.qflag, W.qn,
                           W.best_key, W.best_idx, q, *ov);
    } else {
        ProfScope prof_(s, "fallback");
        hipLaunchKernelGGL(fallback_kernel, dim3((unsigned)std::min<int64_t>(q, 1024)), dim3(256), 0,
                           s, F);
    }

    FinalArgs Z;
    memset(&Z, 0, sizeof Z);
    Z.q = q;
    Z.qn = W.qn;
    Z.best_key = W.best_key;
    Z.best_idx = W.best_idx;
    Z.cnt = W.cnt;
    Z.qflag = W.qflag;
    Z.out_idx = out_idx;
    Z.out_sim = out_sim;
    if (aux) Z.aux = *aux;
    Z.seed_idx = W.seed_idx;
    Z.seed_sim = W.seed_sim;
    Z.thr = W.thr;
    Z.slack = W.slack;
    Z.n_flagged = stats ? W.n_flagged : nullptr;
    if (stats) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, W.n_flagged, 1);
    {
        ProfScope prof_(s, "finalize");
        hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(q)), dim3(256), 0, s, Z);
    }
    HN_HIP(hipGetLastError());
    if (stats) {
        unsigned long long h[2];
        HN_HIP(hipMemcpyAsync(h, W.counter, sizeof h, hipMemcpyDeviceToHost, s));
        HN_HIP(hipStreamSynchronize(s));
        stats->survivors = (int64_t)h[0];
        stats->overflow_queries = (int64_t)h[1];
    }
    if (ov) {
        unsigned long long h = 0, pairs = 0;
        HN_HIP(hipMemcpyAsync(&h, ov->count, sizeof h, hipMemcpyDeviceToHost, s));
        HN_HIP(hipMemcpyAsync(&pairs, W.counter, sizeof pairs, hipMemcpyDeviceToHost, s));
        HN_HIP(hipStreamSynchronize(s));
        ov->n = (int64_t)h;
        ov->pairs = (int64_t)pairs;
    }
    return HN_OK;
}

// A batch, then the queries whose survivors overflowed its pair list again as
// a plain float32 filter pass seeded with the best candidate each reached
// (exact: every entry that can beat that candidate survives the filter, and
// the candidate is the seed), with a list as long as the first pass's pairs
// (plain seed: the re-run's bound is at least as tight).  Synchronises once
// to learn the number of such queries.
int rerun_batch(const hn_index *ix, const float *queries, int64_t q, int64_t *out_idx,
                double *out_sim, const hn_search_opts &o, const hn_search_aux *aux,
                hn_search_stats *stats, hipStream_t s) {
    Arena *ar = nullptr;
    int rc = arena_for((void *)s, (size_t)q * (4 + 8 + 8 + 8 + 8 + kDim * 4) + 8 * 256, &ar, 2);
    if (rc) return rc;
    Overflow ov;
    ov.list = ar->take<int32_t>(q);
    ov.lower = ar->take<double>(q);
    ov.lower_idx = ar->take<int64_t>(q);
    ov.count = ar->take<unsigned long long>(1);
    int64_t *sub_idx = ar->take<int64_t>(q);
    double *sub_sim = ar->take<double>(q);
    float *sub_q = ar->take<float>(q * kDim);
    rc = search_batch(ix, queries, q, out_idx, out_sim, o, aux, stats, s, nullptr, nullptr, &ov);
    if (rc || ov.n == 0) return rc;
    hipLaunchKernelGGL(gather_queries, dim3(blocks_for(ov.n * kDim)), dim3(256), 0, s, queries,
                       ov.list, ov.n, sub_q);
    hn_search_opts o2 = o;
    o2.seed = HN_SEED_PLAIN;
    o2.precision = HN_PREC_FP32;
    // the plain seed's pairs bound the re-run's (its L is at least the
    // seed's); a single pass's window pairs are no guide
    o2.survivor_cap = std::min<int64_t>(
        std::max<int64_t>(o.seed == HN_SEED_PLAIN ? ov.pairs : 0, default_cap(ix->n, ov.n)),
        (int64_t)1 << 28);
    rc = search_batch(ix, sub_q, ov.n, sub_idx, sub_sim, o2, nullptr, nullptr, s, ov.lower,
                      ov.lower_idx, nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(scatter_results, dim3(blocks_for(ov.n)), dim3(256), 0, s, ov.list, ov.n,
                       sub_idx, sub_sim, out_idx, out_sim);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

}  // namespace
}  // namespace hn

extern "C" int hn_search_top1(const hn_index *ix, const float *queries, int64_t q,
                              int64_t *out_idx, double *out_sim, const hn_search_opts *opts,
                              const hn_search_aux *aux, hn_search_stats *stats, void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (q >= ((int64_t)1 << 31) - 4096) return fail(HN_ERR_UNSUPPORTED, "q must be < 2^31");
    if (q > 0 && (!queries || !out_idx || !out_sim))
        return fail(HN_ERR_INVALID_ARG, "null queries or outputs");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    int rc = validate_opts(ix, opts);
    if (rc) return rc;
    if (stats) memset(stats, 0, sizeof *stats);
    if (q == 0) return HN_OK;
    const hn_search_opts o =
        opts ? *opts : hn_search_opts{HN_PREC_FP32, HN_SEED_PLAIN, 0, 0, 0, -1.0};
    hipStream_t s = (hipStream_t)stream;
    // the single-pass forms run in query batches that bound the pair list
    const int64_t qb = o.seed == HN_SEED_PLAIN ? q : window_batch(ix->n);
    for (int64_t q0 = 0; q0 < q; q0 += qb) {
        const int64_t nb = std::min<int64_t>(qb, q - q0);
        hn_search_aux a2;
        if (aux) {
            a2.seed_idx = aux->seed_idx ? aux->seed_idx + q0 : nullptr;
            a2.seed_sim = aux->seed_sim ? aux->seed_sim + q0 : nullptr;
            a2.threshold = aux->threshold ? aux->threshold + q0 : nullptr;
            a2.survivors = aux->survivors ? aux->survivors + q0 : nullptr;
            a2.slack = aux->slack ? aux->slack + q0 : nullptr;
        }
        hn_search_stats st{0, 0};
        // the plain seed on the float32 and bf16 scans never synchronises:
        // queries whose survivors overflow its (generous) list are finished
        // by the exhaustive pass; the other forms keep many more pairs per
        // query and re-run their overflowing queries instead
        if (o.seed == HN_SEED_PLAIN &&
            (o.precision == HN_PREC_FP32 || o.precision == HN_PREC_BF16))
            rc = search_batch(ix, queries + q0 * kDim, nb, out_idx + q0, out_sim + q0, o,
                              aux ? &a2 : nullptr, stats ? &st : nullptr, s);
        else
            rc = rerun_batch(ix, queries + q0 * kDim, nb, out_idx + q0, out_sim + q0, o,
                             aux ? &a2 : nullptr, stats ? &st : nullptr, s);
        if (rc) return rc;
        if (stats) {
            stats->survivors += st.survivors;
            stats->overflow_queries += st.overflow_queries;
        }
    }
    return HN_OK;
}

namespace hn {
namespace {

// Scratch of the allocation-free search: one copy of this array per GPU,
// which each device that runs the library holds until the process ends.  In
// host code its name is not a device address; the address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = (size_t)HN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev`.
int scratch_on(int dev, char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HN_ERR_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(HN_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return HN_OK;
}

// A pair list shorter than this is not worth a search: the overflowing
// queries would all take the exhaustive fallback.
constexpr int64_t kNoAllocMinPairs = (int64_t)1 << 16;

}  // namespace
}  // namespace hn

extern "C" int hn_search_top1_noalloc(const hn_index *ix, const float *queries, int64_t q,
                                      int64_t *out_idx, double *out_sim,
                                      const hn_search_opts *opts, const hn_search_aux *aux,
                                      void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (q >= ((int64_t)1 << 31) - 4096) return fail(HN_ERR_UNSUPPORTED, "q must be < 2^31");
    if (q > 0 && (!queries || !out_idx || !out_sim))
        return fail(HN_ERR_INVALID_ARG, "null queries or outputs");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    int rc = validate_opts(ix, opts);
    if (rc) return rc;
    if (q == 0) return HN_OK;
    hn_search_opts o = opts ? *opts : hn_search_opts{HN_PREC_FP32, HN_SEED_PLAIN, 0, 0, 0, -1.0};
    if (o.seed != HN_SEED_PLAIN)
        return fail(HN_ERR_UNSUPPORTED, "the allocation-free search takes the plain seed");
    if (o.precision != HN_PREC_FP32 && o.precision != HN_PREC_BF16)
        return fail(HN_ERR_UNSUPPORTED,
                    "the allocation-free search scans in fp32 or bf16 (fp8 and int8 re-run "
                    "overflowing queries with buffers of their own)");
    int dev = 0;
    HN_HIP(hipGetDevice(&dev));
    if (dev != ix->device)
        return fail(HN_ERR_INVALID_ARG, "the index lives on device %d, the current one is %d",
                    ix->device, dev);
    char *base = nullptr;
    rc = scratch_on(dev, &base);
    if (rc) return rc;
    // size the call as search_batch will: everything but the pair list is
    // fixed by (n, q) and the launch shapes; the pair list takes the rest
    Work W;
    rc = plan_stage(ix, q, o, W, false, 0);
    if (rc) return rc;
    size_t per_pair = 0;
    const size_t fixed_bytes = stage_bytes(ix, q, W, false, &per_pair);
    if (fixed_bytes + (size_t)kNoAllocMinPairs * per_pair > kNoAllocBytes)
        return fail(HN_ERR_INVALID_ARG,
                    "q = %lld queries against n = %lld entries need %zu bytes of scratch besides "
                    "the survivor list; the allocation-free search has %zu: pass fewer queries "
                    "per call",
                    (long long)q, (long long)ix->n, fixed_bytes + (size_t)kNoAllocMinPairs * per_pair,
                    kNoAllocBytes);
    const int64_t fit = (int64_t)((kNoAllocBytes - fixed_bytes) / per_pair);
    if (o.survivor_cap > fit)
        return fail(HN_ERR_INVALID_ARG,
                    "survivor_cap = %lld pairs does not fit the allocation-free scratch "
                    "(at most %lld for this call)",
                    (long long)o.survivor_cap, (long long)fit);
    if (o.survivor_cap <= 0) o.survivor_cap = std::min<int64_t>(default_cap(ix->n, q), fit);
    Arena fixed;
    fixed.base = base;
    fixed.cap = kNoAllocBytes;
    return search_batch(ix, queries, q, out_idx, out_sim, o, aux, nullptr, (hipStream_t)stream,
                        nullptr, nullptr, nullptr, &fixed);
}

extern "C" int hn_search_topk(const hn_index *ix, const float *queries, int64_t q, int32_t topk,
                              int64_t *out_idx, double *out_sim, const hn_search_opts *opts,
                              void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (topk < 1 || topk > 128) return fail(HN_ERR_INVALID_ARG, "topk must be in [1, 128]");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (q >= ((int64_t)1 << 31) - 4096) return fail(HN_ERR_UNSUPPORTED, "q must be < 2^31");
    if (q > 0 && (!queries || !out_idx || !out_sim))
        return fail(HN_ERR_INVALID_ARG, "null queries or outputs");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    int rc = validate_opts(ix, opts);
    if (rc) return rc;
    if (q == 0) return HN_OK;
    const hn_search_opts o =
        opts ? *opts : hn_search_opts{HN_PREC_FP32, HN_SEED_PLAIN, 0, 0, 0, -1.0};
    if (o.seed != HN_SEED_PLAIN) return fail(HN_ERR_UNSUPPORTED, "top-k uses the plain seed");
    hipStream_t s = (hipStream_t)stream;
    int64_t cap = o.survivor_cap > 0 ? o.survivor_cap : default_cap(ix->n, q);
    Work W;
    unsigned long long total = 0;
    // The survivor set is fixed by the seeds; if it did not fit, run again
    // with room for all of it (the counter keeps counting past the cap).
    for (int attempt = 0; attempt < 2; ++attempt) {
        rc = stage_seed(ix, queries, q, o, nullptr, nullptr, cap, W, s, false, topk);
        if (rc) return rc;
        ScanArgs A = filter_args(ix, W, q, W.pairs, cap);
        // float32, bf16 and int8: the filter's flushes store each pair's
        // canonical sim and count it, as the rescoring kernel would
        const bool fused = W.precision != HN_PREC_FP8;
        if (fused) {
            A.psim = W.psim;
            A.best_key = W.best_key;
            A.cnt = W.cnt;
            A.rs_queries = queries;
            A.rs_rows = ix->rows;
            if (W.precision != HN_PREC_FP32) {
                A.rs_major32 = ix->major32;
                A.rs_thr32 = W.thr32;
                A.rs_kp = ix->kp;
                A.rs_k = ix->k;
            }
        }
        rc = launch_scan<kFilter>(W.precision, W.width, W.cfg, W.plan, A, s);
        if (rc) return rc;
        RescoreArgs R;
        memset(&R, 0, sizeof R);
        R.pairs = W.pairs;
        R.counter = W.counter;
        R.cap = cap;
        R.queries = queries;
        R.rows = ix->rows;
        R.major32 = ix->major32;
        R.kp = ix->kp;
        R.k = ix->k;
        R.thr32 = W.thr32;
        R.psim = W.psim;
        R.best_key = W.best_key;
        R.best_idx = W.best_idx;
        R.cnt = W.cnt;
        R.q = q;
        R.count = 1;
        if (!fused) {
            ProfScope prof_(s, "topk_rescore");
            hipLaunchKernelGGL(rescore_kernel<1>, dim3(2048), dim3(256), 0, s, R);
        }
        HN_HIP(hipMemcpyAsync(&total, W.counter, sizeof total, hipMemcpyDeviceToHost, s));
        HN_HIP(hipStreamSynchronize(s));
        if ((int64_t)total <= cap) break;
        if (attempt == 1) return fail(HN_ERR_DEVICE, "top-k survivor list grew between passes");
        if (total >= ((unsigned long long)1 << 31))
            return fail(HN_ERR_UNSUPPORTED, "top-k needs %llu survivor pairs (limit 2^31)", total);
        cap = (int64_t)total;
    }
    Arena *ar = nullptr;
    rc = arena_for((void *)s, (size_t)(q + 1) * 8 + (size_t)q * 4 + (size_t)cap * 12 + 1024, &ar, 3);
    if (rc) return rc;
    int64_t *off = ar->take<int64_t>(q + 1);
    int32_t *fill = ar->take<int32_t>(q);
    double *bsim = ar->take<double>(cap);
    int32_t *bent = ar->take<int32_t>(cap);
    hipLaunchKernelGGL(fill_i32, dim3(blocks_for(q)), dim3(256), 0, s, fill, q);
    {
        ProfScope prof_(s, "topk_offsets");
        hipLaunchKernelGGL(prefix_counts, dim3(1), dim3(1024), 0, s, W.cnt, q, off);
    }
    {
        ProfScope prof_(s, "topk_scatter");
        hipLaunchKernelGGL(scatter_pairs, dim3(2048), dim3(256), 0, s, W.pairs, W.psim, W.counter,
                           cap, off, fill, bsim, bent);
    }
    {
        ProfScope prof_(s, "topk_select");
        hipLaunchKernelGGL(topk_select, dim3(blocks_for(q, 4)), dim3(256), 0, s, off, bsim, bent,
                           q, topk, W.qn, out_idx, out_sim);
    }
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_filter_survivors(const hn_index *ix, const float *queries, int64_t q,
                                   const double *lower, int32_t *pairs, int64_t cap,
                                   int64_t *count, double *slack, const hn_search_opts *opts,
                                   void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (q < 0 || cap < 0) return fail(HN_ERR_INVALID_ARG, "q and cap must be >= 0");
    if (!count) return fail(HN_ERR_INVALID_ARG, "count is null");
    if (q > 0 && (!queries || !lower || (cap > 0 && !pairs)))
        return fail(HN_ERR_INVALID_ARG, "null queries, lower bounds or pairs");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    int rc = validate_opts(ix, opts);
    if (rc) return rc;
    *count = 0;
    if (q == 0) return HN_OK;
    hn_search_opts o = opts ? *opts : hn_search_opts{HN_PREC_FP32, HN_SEED_PLAIN, 0, 0, 0, -1.0};
    hipStream_t s = (hipStream_t)stream;
    Work W;
    rc = stage_seed(ix, queries, q, o, lower, nullptr, 1, W, s);
    if (rc) return rc;
    ScanArgs A = filter_args(ix, W, q, reinterpret_cast<int2 *>(pairs), cap);
    rc = launch_scan<kFilter>(W.precision, W.width, W.cfg, W.plan, A, s);
    if (rc) return rc;
    if (slack) HN_HIP(hipMemcpyAsync(slack, W.slack, q * sizeof(double), hipMemcpyDeviceToDevice, s));
    unsigned long long h = 0;
    HN_HIP(hipMemcpyAsync(&h, W.counter, sizeof h, hipMemcpyDeviceToHost, s));
    HN_HIP(hipStreamSynchronize(s));
    *count = (int64_t)h;
    return HN_OK;
}

extern "C" int hn_scan_scores(const hn_index *ix, const float *queries, int64_t q,
                              int32_t precision, float *scores, void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (q > 0 && (!queries || !scores)) return fail(HN_ERR_INVALID_ARG, "null queries or scores");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    int rc = check_precision(ix, precision);
    if (rc) return rc;
    if (q == 0) return HN_OK;
    hipStream_t s = (hipStream_t)stream;
    Work W;
    W.precision = precision;
    W.width = stream_width(ix, precision);
    W.cfg = 0;
    const TileInfo ti = tile_info(precision, W.width);
    W.plan = make_plan(ix->n, q, W.cfg, 0, ti.rows, ti.cols);
    const Plan &p = W.plan;
    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) { bytes += (count * sz + 255) & ~size_t(255); };
    add(p.q_pad * ix->kp, 4);
    add(p.q_pad * ix->kb, 2);
    add(p.q_pad * ix->k8, 1);
    add(p.q_pad, sizeof(QNorm));
    add(kWorkWords, 4);
    add(p.n_items, 4);
    Arena *ar = nullptr;
    rc = arena_for(stream, bytes, &ar);
    if (rc) return rc;
    W.op32 = ar->take<float>(p.q_pad * ix->kp);
    W.op16 = ar->take<uint16_t>(p.q_pad * ix->kb);
    W.op8 = precision == HN_PREC_FP8 ? ar->take<uint8_t>(p.q_pad * ix->k8) : nullptr;
    W.opi = precision == HN_PREC_INT8 ? ar->take<int8_t>(p.q_pad * ix->k8) : nullptr;
    W.qn = ar->take<QNorm>(p.q_pad);
    W.work = ar->take<unsigned>(kWorkWords);
    W.redo = ar->take<int>(p.n_items);
    launch_prep(ix, queries, q, p.q_pad, W, s);
    ScanArgs A;
    memset(&A, 0, sizeof A);
    A.x = stream_of(ix, precision);
    A.x_stride = W.width;
    A.qs = operands_of(W);
    A.q_stride = W.width;
    A.n = ix->n;
    A.n_blocks = p.n_blocks;
    A.chunk_blocks = p.chunk_blocks;
    A.n_chunks = p.n_chunks;
    A.n_qb = p.n_qb;
    A.n_items = p.n_items;
    A.q_count = (int32_t)q;
    A.q_pad = (int32_t)p.q_pad;
    A.scores = scores;
    A.redo = W.redo;
    A.redo_count = W.work + 2 * kXcds;
    rc = launch_scan<kStore>(precision, W.width, W.cfg, p, A, s);
    if (rc || (precision != HN_PREC_FP8 && precision != HN_PREC_INT8)) return rc;
    // fp8 / int8 scores come out in units of s_q s_x: rescale (exact, powers of two)
    hipLaunchKernelGGL(scale_scores, dim3(2048), dim3(256), 0, s, scores, q, ix->n, W.qn,
                       precision == HN_PREC_FP8 ? ix->scale8 : ix->scale_i8,
                       precision == HN_PREC_INT8 ? 1 : 0);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_bruteforce_top1(const float *db, int64_t n, int32_t d, const float *queries,
                                  int64_t q, int64_t *out_idx, double *out_sim, void *stream) {
    clear_error();
    if (d != kDim) return fail(HN_ERR_INVALID_ARG, "d must be 128 (got %d)", d);
    if (n < 1) return fail(HN_ERR_INVALID_ARG, "n must be >= 1");
    if (n >= (int64_t)1 << 31) return fail(HN_ERR_UNSUPPORTED, "n must be < 2^31");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (!db || (q > 0 && (!queries || !out_idx || !out_sim)))
        return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    if (!aligned16(db) || !aligned16(queries))
        return fail(HN_ERR_INVALID_ARG, "db and queries must be 16-byte aligned");
    if (q == 0) return HN_OK;
    hipStream_t s = (hipStream_t)stream;
    const TileInfo ti = tile_info(HN_PREC_FP32, kDim);
    const int cfg = pick_cfg(q, ti.cols, ti.cost, 2);
    Plan p = make_plan(n, q, cfg, 0, ti.rows, ti.cols, 8192,
                       scan_slots(HN_PREC_FP32, kWindow, kDim, cfg));
    // A prefix pass over the first n_pre rows gives each query a starting
    // running maximum: a real scan score, so never above the final maximum,
    // and far fewer near-record candidates in the main pass.  It runs as up
    // to 16 chunks (work items in parallel) reduced to one maximum per query.
    const int64_t n_pre = std::min<int64_t>(n, 4096);
    const int32_t pre_blocks = (int32_t)((n_pre + ti.rows - 1) / ti.rows);
    Plan pp = make_plan(n_pre, q, cfg, std::max<int32_t>(1, (pre_blocks + 15) / 16), ti.rows,
                        ti.cols);
    const int64_t cap = std::min<int64_t>(
        std::max<int64_t>(q * std::max<int64_t>(256, 16 * (int64_t)p.n_chunks), 1 << 16),
        (int64_t)1 << 26);

    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) { bytes += (count * sz + 255) & ~size_t(255); };
    add(p.q_pad, sizeof(QNorm));
    add((size_t)p.n_chunks * p.q_pad, 4);
    add((size_t)pp.n_chunks * pp.q_pad, 4);
    add((size_t)pp.n_chunks * pp.q_pad, 4);
    add(p.q_pad, 4);
    add(p.q_pad, 4);
    add(q, 8);
    add(q, 4);
    add(q, 8);
    add(q, 4);
    add(q, 4);
    add(q, 4);
    add(4, 8);
    add(kWorkWords, 4);
    add(p.n_items + pp.n_items, 4);
    add(cap, sizeof(int2));
    add(cap, 4);
    add(cap, 8);
    Arena *ar = nullptr;
    int rc = arena_for(stream, bytes, &ar);
    if (rc) return rc;
    QNorm *qn = ar->take<QNorm>(p.q_pad);
    float *part_val = ar->take<float>((size_t)p.n_chunks * p.q_pad);
    float *pre_val = ar->take<float>((size_t)pp.n_chunks * pp.q_pad);
    int32_t *pre_idx = ar->take<int32_t>((size_t)pp.n_chunks * pp.q_pad);
    float *pre_max = ar->take<float>(p.q_pad);
    float *win_scan = ar->take<float>(p.q_pad);
    double *win = ar->take<double>(q);
    float *thr = ar->take<float>(q);
    unsigned long long *best_key = ar->take<unsigned long long>(q);
    int32_t *best_idx = ar->take<int32_t>(q);
    int32_t *cnt = ar->take<int32_t>(q);
    int32_t *qflag = ar->take<int32_t>(q);
    unsigned long long *counter = ar->take<unsigned long long>(4);
    unsigned long long *mu_key = counter + 1;
    unsigned *work = ar->take<unsigned>(kWorkWords);
    int *redo = ar->take<int>(p.n_items + pp.n_items);
    int2 *pairs = ar->take<int2>(cap);
    float *pair_val = ar->take<float>(cap);
    double *psim = ar->take<double>(cap);

    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, counter, 4);
    {
        ProfScope prof_(s, "bf_db_norm");
        const unsigned g = (unsigned)std::min<int64_t>(kBfNormGrid, (n + 4 * kBfNormRows - 1) /
                                                                         (4 * kBfNormRows));
        hipLaunchKernelGGL(bf_db_norm, dim3(g), dim3(256), 0, s,
                           reinterpret_cast<const float4 *>(db), n, mu_key);
    }
    {
        PrepArgs P;
        memset(&P, 0, sizeof P);
        P.q = queries;
        P.nq = q;
        P.q_pad = p.q_pad;
        P.k = kDim - 1;
        P.qn = qn;
        P.work = work;
        hipLaunchKernelGGL(prep_queries, dim3(blocks_for(p.q_pad, 4)), dim3(256), 0, s, P);
    }
    BfPrepArgs P{qn, mu_key, q, p.q_pad, win_scan, win, best_key, best_idx, cnt, qflag, counter};
    {
        ProfScope prof_(s, "bf_prep");
        hipLaunchKernelGGL(bf_prep, dim3(blocks_for(p.q_pad)), dim3(256), 0, s, P);
    }

    ScanArgs A;
    memset(&A, 0, sizeof A);
    A.x = db;
    A.x_stride = kDim;
    A.qs = queries;
    A.q_stride = kDim;
    A.q_count = (int32_t)q;
    A.q_pad = (int32_t)p.q_pad;
    A.qflag = qflag;
    // prefix pass: largest scan score over the first n_pre rows per query
    A.n = n_pre;
    A.n_blocks = pp.n_blocks;
    A.chunk_blocks = pp.chunk_blocks;
    A.n_chunks = pp.n_chunks;
    A.n_qb = pp.n_qb;
    A.n_items = pp.n_items;
    A.part_val = pre_val;
    A.part_idx = pre_idx;
    A.redo = redo + p.n_items;
    A.redo_count = work + 2 * kXcds;
    rc = launch_scan<kArgmax>(HN_PREC_FP32, kDim, cfg, pp, A, s);
    if (rc) return rc;
    // main pass over all rows
    A.n = n;
    A.n_blocks = p.n_blocks;
    A.chunk_blocks = p.chunk_blocks;
    A.n_chunks = p.n_chunks;
    A.n_qb = p.n_qb;
    A.n_items = p.n_items;
    A.part_val = part_val;
    A.part_idx = nullptr;
    A.thr = win_scan;
    {
        ProfScope prof_(s, "bf_prefix_max");
        hipLaunchKernelGGL(prefix_max, dim3(blocks_for(p.q_pad, 4)), dim3(256), 0, s, pre_val,
                           pp.n_chunks, (int32_t)pp.q_pad, p.q_pad, pre_max);
    }
    A.init_best = pre_max;
    A.pairs = pairs;
    A.pair_val = pair_val;
    A.counter = counter;
    A.cap = cap;
    A.redo = redo;
    A.redo_count = work + 2 * kXcds + 1;
    A.item_ctr = p.n_qb > 1 ? work + kXcds : nullptr;
    rc = launch_scan<kWindow>(HN_PREC_FP32, kDim, cfg, p, A, s);
    if (rc) return rc;
    {
        ProfScope prof_(s, "bf_threshold");
        hipLaunchKernelGGL(bf_threshold, dim3(blocks_for(q, 4)), dim3(256), 0, s, part_val, p.n_chunks,
                           (int32_t)p.q_pad, q, win, thr);
    }

    RescoreArgs R;
    memset(&R, 0, sizeof R);
    R.pairs = pairs;
    R.pair_val = pair_val;
    R.counter = counter;
    R.cap = cap;
    R.queries = queries;
    R.rows = db;
    R.thr32 = thr;
    R.psim = psim;
    R.best_key = best_key;
    R.best_idx = best_idx;
    R.cnt = cnt;
    R.q = q;
    {
        ProfScope prof_(s, "bf_rescore");
        hipLaunchKernelGGL(rescore_kernel<2>, dim3(1024), dim3(256), 0, s, R);
    }
    {
        ProfScope prof_(s, "bf_tie");
        hipLaunchKernelGGL(tie_kernel, dim3(1024), dim3(256), 0, s, R);
    }

    FallbackArgs F;
    memset(&F, 0, sizeof F);
    F.qflag = qflag;
    F.qn = qn;
    F.queries = queries;
    F.rows = db;
    F.q = q;
    F.n = n;
    F.k = kDim;
    F.full = 1;
    F.best_key = best_key;
    F.best_idx = best_idx;
    F.cnt = cnt;
    hipLaunchKernelGGL(fallback_kernel, dim3((unsigned)std::min<int64_t>(q, 1024)), dim3(256), 0,
                       s, F);

    FinalArgs Z;
    memset(&Z, 0, sizeof Z);
    Z.q = q;
    Z.qn = qn;
    Z.best_key = best_key;
    Z.best_idx = best_idx;
    Z.cnt = cnt;
    Z.qflag = qflag;
    Z.out_idx = out_idx;
    Z.out_sim = out_sim;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(q)), dim3(256), 0, s, Z);
    HN_HIP(hipGetLastError());
    return HN_OK;
}
