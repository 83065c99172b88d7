// Many databases in one search: ragged query batches against indexes of
// different size, K and alpha run as one pipeline.  Each scan is one
// persistent launch over the work items of every database of a stream width
// (one launch in all for bf16 and fp8, whose streams are 16 wide for K <= 16),
// and the per-query kernels look their database up.  A plan owns every buffer
// and table, so an execution allocates nothing and never synchronises: it can
// be replayed as a captured HIP graph.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "hn_pipeline.h"

namespace hn {
namespace {

// Shortest argmax-pass work item of a multi-database plan, in entry blocks
// (measured on the 64-database set: 128 blocks took the pass from 0.77 to
// 0.59 ms; the filter pass is faster with the usual shorter chunks).
constexpr int kMultiArgmaxBlocks = 128;

struct MultiGroup {
    int width = 0, cfg = 0;
    int64_t arg_off = 0;   // first argmax-pass item of the group in the item list
    int arg_items = 0;
    int64_t item_off = 0;  // first filter-pass item of the group in the item list
    int n_items = 0;
};

__global__ void copy_in(const float4 *__restrict__ q, const int64_t *__restrict__ o2p,
                        int64_t total_q, float4 *__restrict__ q_buf) {
    const int64_t n = total_q * (kDim / 4);
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * 256) {
        const int64_t row = t / (kDim / 4), c = t % (kDim / 4);
        q_buf[o2p[row] * (kDim / 4) + c] = q[t];
    }
}

// The first kernel of a search: clears the flags and counters and records
// the start on the constant-rate clock (ts[0]); ts[1 + d] collects database
// d's last result write (finalize_kernel).
__global__ void multi_reset(int32_t *qflag, int64_t total_pad, unsigned *redo_counts,
                            int n_groups, unsigned *item_ctrs, int n_ctrs,
                            unsigned long long *counter, unsigned long long *ts, int n_db) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < total_pad) qflag[t] = 0;
    if (t < n_groups) redo_counts[t] = 0u;
    if (t < n_ctrs) item_ctrs[t] = 0u;
    if (t < 2) counter[t] = 0ull;
    if (t == 0) ts[0] = (unsigned long long)wall_clock64();
    if (t < n_db) ts[1 + t] = 0ull;
}

__global__ __launch_bounds__(256) void prep_multi(const PrepArgs *__restrict__ P,
                                                  const DbRef *__restrict__ db,
                                                  const int32_t *__restrict__ gdb,
                                                  int64_t total_pad) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= total_pad) return;
    const int d = __builtin_amdgcn_readfirstlane(gdb[g]);
    prep_wave(P[d], g - db[d].pad_base, threadIdx.x & 63);
}

__global__ __launch_bounds__(256) void seed_multi(const SeedArgs *__restrict__ S,
                                                  const DbRef *__restrict__ db,
                                                  const int32_t *__restrict__ gdb,
                                                  int64_t total_pad) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= total_pad) return;
    const int d = __builtin_amdgcn_readfirstlane(gdb[g]);
    seed_one(S[d], g - db[d].pad_base, threadIdx.x & 63);
}

}  // namespace
}  // namespace hn

using namespace hn;

struct hn_multi_plan {
    int device = 0;
    int n_db = 0;
    int precision = HN_PREC_FP32;
    int64_t total_q = 0, total_pad = 0, cap = 0, total_items = 0;
    char *mem = nullptr;
    float *q_buf = nullptr;
    QNorm *qn = nullptr;
    float *thr = nullptr, *thr32 = nullptr;
    int64_t *seed_idx = nullptr;
    double *seed_sim = nullptr, *slack = nullptr, *psim = nullptr;
    unsigned long long *best_key = nullptr, *counter = nullptr;
    int32_t *best_idx = nullptr, *cnt = nullptr, *qflag = nullptr, *gdb = nullptr;
    int2 *pairs = nullptr, *items = nullptr;
    int64_t *o2p = nullptr;
    ScanArgs *scan_argmax = nullptr, *scan_filter = nullptr;
    SeedArgs *seeds = nullptr;
    PrepArgs *preps = nullptr;
    DbRef *dbref = nullptr;
    int *redo = nullptr;
    unsigned *redo_counts = nullptr;
    unsigned *item_ctrs = nullptr;  // per group: kXcds item counters of each scan pass
    unsigned long long *ts = nullptr;  // [1 + n_db]: start, then per database its last write
    bool fused = false;  // all but fp8: the filter's flushes rescore their pairs
    std::vector<MultiGroup> groups;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_q = nullptr;
    const void *g_idx = nullptr;
    const void *g_sim = nullptr;
};

namespace {

void plan_destroy(hn_multi_plan *P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    dev_free(P->mem);
    delete P;
}

bool multi_width_ok(int precision, int w) {
    if (precision == HN_PREC_FP32) return w == 8 || w == 16 || w == 32;
    return w == 16 || w == 32;
}

// The whole pipeline on `s`: no allocation, no synchronisation.
int enqueue(hn_multi_plan *P, const float *queries, int64_t *out_idx, double *out_sim,
            hipStream_t s) {
    const int ng = (int)P->groups.size();
    const int n_ctrs = 2 * kXcds * ng;
    const int64_t reset_n = std::max<int64_t>(
        std::max<int64_t>(std::max<int64_t>(P->total_pad, 64), n_ctrs), P->n_db);
    hipLaunchKernelGGL(multi_reset, dim3(blocks_for(reset_n)),
                       dim3(256), 0, s, P->qflag, P->total_pad, P->redo_counts, ng, P->item_ctrs,
                       n_ctrs, P->counter, P->ts, P->n_db);
    hipLaunchKernelGGL(copy_in, dim3((unsigned)std::min<int64_t>(blocks_for(P->total_q * 32), 8192)),
                       dim3(256), 0, s, reinterpret_cast<const float4 *>(queries), P->o2p,
                       P->total_q, reinterpret_cast<float4 *>(P->q_buf));
    {
        ProfScope prof_(s, "multi_prep");
        hipLaunchKernelGGL(prep_multi, dim3(blocks_for(P->total_pad, 4)), dim3(256), 0, s, P->preps,
                           P->dbref, P->gdb, P->total_pad);
    }
    for (int g = 0; g < ng; ++g) {
        const MultiGroup &G = P->groups[g];
        if (G.arg_items == 0) continue;
        ProfScope prof_(s, "multi_scan_argmax");
        if (launch_scan_multi(P->precision, kArgmax, G.width, G.cfg, P->scan_argmax,
                              P->items + G.arg_off, G.arg_items, P->redo + G.arg_off,
                              P->redo_counts + g, P->item_ctrs + (2 * g) * kXcds, s))
            return fail(HN_ERR_INVALID_ARG, "no multi-database scan for width %d", G.width);
    }
    {
        ProfScope prof_(s, "multi_seed");
        hipLaunchKernelGGL(seed_multi, dim3(blocks_for(P->total_pad, 4)), dim3(256), 0, s,
                           P->seeds, P->dbref, P->gdb, P->total_pad);
    }
    for (int g = 0; g < ng; ++g) {
        const MultiGroup &G = P->groups[g];
        if (G.n_items == 0) continue;
        ProfScope prof_(s, "multi_scan_filter");
        if (launch_scan_multi(P->precision, kFilter, G.width, G.cfg, P->scan_filter,
                              P->items + G.item_off, G.n_items, P->redo + G.item_off,
                              P->redo_counts + g, P->item_ctrs + (2 * g + 1) * kXcds, s))
            return fail(HN_ERR_INVALID_ARG, "no multi-database scan for width %d", G.width);
    }
    RescoreArgs R;
    memset(&R, 0, sizeof R);
    R.pairs = P->pairs;
    R.counter = P->counter;
    R.cap = P->cap;
    R.queries = P->q_buf;
    R.thr32 = P->thr32;
    R.psim = P->psim;
    R.best_key = P->best_key;
    R.best_idx = P->best_idx;
    R.cnt = P->cnt;
    R.seed_idx = P->seed_idx;
    R.seed_sim = P->seed_sim;
    R.q = P->total_pad;
    R.db = P->dbref;
    R.gdb = P->gdb;
    if (!P->fused) {
        ProfScope prof_(s, "multi_rescore");
        if (P->precision == HN_PREC_FP32)
            hipLaunchKernelGGL(rescore_kernel<0>, dim3(2048), dim3(256), 0, s, R);
        else
            hipLaunchKernelGGL(rescore_kernel<1>, dim3(2048), dim3(256), 0, s, R);
    }
    hipLaunchKernelGGL(tie_kernel, dim3(2048), dim3(256), 0, s, R);
    FallbackArgs F;
    memset(&F, 0, sizeof F);
    F.qflag = P->qflag;
    F.qn = P->qn;
    F.queries = P->q_buf;
    F.q = P->total_pad;
    F.seed_sim = P->seed_sim;
    F.best_key = P->best_key;
    F.best_idx = P->best_idx;
    F.cnt = P->cnt;
    F.db = P->dbref;
    F.gdb = P->gdb;
    hipLaunchKernelGGL(fallback_kernel, dim3((unsigned)std::min<int64_t>(P->total_pad, 1024)),
                       dim3(256), 0, s, F);
    FinalArgs Z;
    memset(&Z, 0, sizeof Z);
    Z.q = P->total_pad;
    Z.qn = P->qn;
    Z.best_key = P->best_key;
    Z.best_idx = P->best_idx;
    Z.cnt = P->cnt;
    Z.qflag = P->qflag;
    Z.out_idx = out_idx;
    Z.out_sim = out_sim;
    Z.db = P->dbref;
    Z.gdb = P->gdb;
    Z.ts_end = P->ts + 1;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(P->total_pad)), dim3(256), 0, s, Z);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

}  // namespace

extern "C" int hn_multi_plan_create(const hn_index *const *ixs, int32_t n_db,
                                    const int64_t *q_counts, const hn_search_opts *opts,
                                    hn_multi_plan **out) {
    clear_error();
    if (!out) return fail(HN_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!ixs || !q_counts) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    if (n_db < 1 || n_db > (1 << 16)) return fail(HN_ERR_INVALID_ARG, "n_db must be in [1, 65536]");
    const hn_search_opts o =
        opts ? *opts : hn_search_opts{HN_PREC_FP32, HN_SEED_PLAIN, 0, 0, 0, -1.0};
    if (o.seed != HN_SEED_PLAIN)
        return fail(HN_ERR_UNSUPPORTED, "the multi-database search uses the plain seed");
    if (o.query_tiles < 0 || o.chunk_blocks < 0 || o.survivor_cap < 0)
        return fail(HN_ERR_INVALID_ARG, "negative launch option");
    int dev = 0;
    HN_HIP(hipGetDevice(&dev));
    int64_t total_q = 0;
    for (int d = 0; d < n_db; ++d) {
        const hn_index *ix = ixs[d];
        if (!ix) return fail(HN_ERR_INVALID_ARG, "index %d is null", d);
        if (ix->device != dev) return fail(HN_ERR_INVALID_ARG, "index %d is on another device", d);
        if (q_counts[d] < 0) return fail(HN_ERR_INVALID_ARG, "q_counts[%d] < 0", d);
        int rc = check_precision(ix, o.precision);
        if (rc) return rc;
        if (!multi_width_ok(o.precision, stream_width(ix, o.precision)))
            return fail(HN_ERR_UNSUPPORTED, "index %d: the multi-database search needs k <= 32", d);
        if (!(o.beta < 0.0 || o.beta <= ix->alpha))
            return fail(HN_ERR_INVALID_ARG, "beta must be < 0 (exact) or in [0, alpha]");
        total_q += q_counts[d];
    }
    if (total_q >= ((int64_t)1 << 31) - (int64_t)n_db * 1024)
        return fail(HN_ERR_UNSUPPORTED, "too many queries in one plan");

    hn_multi_plan *P = new (std::nothrow) hn_multi_plan();
    if (!P) return fail(HN_ERR_OOM, "host allocation failed");
    P->device = dev;
    P->n_db = n_db;
    P->precision = o.precision;
    P->total_q = total_q;

    // groups of equal stream width, each with one launch configuration
    std::vector<int> width(n_db);
    for (int d = 0; d < n_db; ++d) width[d] = stream_width(ixs[d], o.precision);
    std::vector<int> widths(width);
    std::sort(widths.begin(), widths.end());
    widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
    std::vector<int> group_of(n_db);
    for (int w : widths) {
        MultiGroup G;
        G.width = w;
        int64_t qmax = 1;
        for (int d = 0; d < n_db; ++d)
            if (width[d] == w) qmax = std::max(qmax, q_counts[d]);
        const TileInfo ti = tile_info(o.precision, w);
        G.cfg = pick_cfg(qmax, ti.cols, ti.cost, o.query_tiles);
        if (G.cfg < 0) {
            plan_destroy(P);
            return fail(HN_ERR_INVALID_ARG, "query_tiles=%d is not available", o.query_tiles);
        }
        P->groups.push_back(G);
    }
    for (int d = 0; d < n_db; ++d)
        group_of[d] = (int)(std::lower_bound(widths.begin(), widths.end(), width[d]) - widths.begin());

    // per-database plans and the padded query layout.  The argmax pass has
    // no survivors to stage, so its items can be long: at least
    // kMultiArgmaxBlocks entry blocks (or the whole database), which keeps
    // each item's fixed costs (claim, query tiles, partials) small against
    // its scan when most databases hold few queries; the filter pass keeps
    // the usual chunks, whose survivors fit the per-wave staging buffers.
    std::vector<Plan> plan(n_db), aplan(n_db);
    std::vector<int64_t> pad_base(n_db), out_base(n_db), part_off(n_db), op_off(n_db);
    int64_t total_pad = 0, total_part = 0, total_op = 0, cap = 0;
    int64_t o_cum = 0;
    for (int d = 0; d < n_db; ++d) {
        const TileInfo ti = tile_info(o.precision, width[d]);
        if (q_counts[d] > 0) {
            const int cfg = P->groups[group_of[d]].cfg;
            plan[d] = make_plan(ixs[d]->n, q_counts[d], cfg, o.chunk_blocks, ti.rows, ti.cols);
            aplan[d] = o.chunk_blocks > 0
                           ? plan[d]
                           : make_plan(ixs[d]->n, q_counts[d], cfg,
                                       std::max(plan[d].chunk_blocks, kMultiArgmaxBlocks),
                                       ti.rows, ti.cols);
        }
        pad_base[d] = total_pad;
        out_base[d] = o_cum;
        part_off[d] = total_part;
        op_off[d] = total_op;
        total_pad += plan[d].q_pad;
        total_part += (int64_t)aplan[d].n_chunks * aplan[d].q_pad;
        total_op += plan[d].q_pad * width[d];
        o_cum += q_counts[d];
        if (q_counts[d] > 0) cap += default_cap(ixs[d]->n, q_counts[d]);
    }
    cap = o.survivor_cap > 0 ? o.survivor_cap : std::min<int64_t>(cap, (int64_t)1 << 28);
    cap = std::max<int64_t>(cap, 1);
    P->total_pad = total_pad;
    P->cap = cap;
    // item lists, group by group: the argmax pass's, then the filter pass's
    std::vector<int2> items;
    for (size_t g = 0; g < P->groups.size(); ++g) {
        MultiGroup &G = P->groups[g];
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<Plan> &pl = pass == 0 ? aplan : plan;
            const int64_t off = (int64_t)items.size();
            for (int d = 0; d < n_db; ++d) {
                if (group_of[d] != (int)g) continue;
                for (int it = 0; it < pl[d].n_items; ++it) items.push_back(make_int2(d, it));
            }
            const int64_t cnt = (int64_t)items.size() - off;
            if (cnt >= ((int64_t)1 << 31)) {
                plan_destroy(P);
                return fail(HN_ERR_UNSUPPORTED, "too many work items");
            }
            (pass == 0 ? G.arg_off : G.item_off) = off;
            (pass == 0 ? G.arg_items : G.n_items) = (int)cnt;
        }
    }
    P->total_items = (int64_t)items.size();

    // one device block for every buffer
    const size_t esz = o.precision == HN_PREC_FP32 ? 4 : (o.precision == HN_PREC_BF16 ? 2 : 1);
    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) {
        const size_t off = bytes;
        bytes += (count * sz + 255) & ~size_t(255);
        return off;
    };
    const int64_t tp = std::max<int64_t>(total_pad, 1);
    const size_t o_q = add(tp * kDim, 4), o_op = add(std::max<int64_t>(total_op, 1), esz),
                 o_qn = add(tp, sizeof(QNorm)), o_pv = add(std::max<int64_t>(total_part, 1), 4),
                 o_pi = add(std::max<int64_t>(total_part, 1), 4), o_thr = add(tp, 4),
                 o_thr32 = add(tp, 4), o_sidx = add(tp, 8), o_ssim = add(tp, 8),
                 o_slack = add(tp, 8), o_bk = add(tp, 8), o_bi = add(tp, 4), o_cnt = add(tp, 4),
                 o_qf = add(tp, 4), o_gdb = add(tp, 4), o_ctr = add(4, 8),
                 o_pairs = add(cap, sizeof(int2)), o_psim = add(cap, 8),
                 o_items = add(std::max<int64_t>(P->total_items, 1), sizeof(int2)),
                 o_redo = add(std::max<int64_t>(P->total_items, 1), 4),
                 o_rc = add(P->groups.size() + 1, 4),
                 o_ictr = add(2 * kXcds * P->groups.size() + 1, 4),
                 o_o2p = add(std::max<int64_t>(total_q, 1), 8),
                 o_sa = add(n_db, sizeof(ScanArgs)), o_sf = add(n_db, sizeof(ScanArgs)),
                 o_seed = add(n_db, sizeof(SeedArgs)), o_prep = add(n_db, sizeof(PrepArgs)),
                 o_db = add(n_db, sizeof(DbRef)), o_ts = add(n_db + 1, 8);
    if (dev_alloc(&P->mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        plan_destroy(P);
        return fail(HN_ERR_OOM, "plan allocation of %zu bytes failed", bytes);
    }
    char *m = P->mem;
    P->q_buf = reinterpret_cast<float *>(m + o_q);
    char *op = m + o_op;
    P->qn = reinterpret_cast<QNorm *>(m + o_qn);
    float *part_val = reinterpret_cast<float *>(m + o_pv);
    int32_t *part_idx = reinterpret_cast<int32_t *>(m + o_pi);
    P->thr = reinterpret_cast<float *>(m + o_thr);
    P->thr32 = reinterpret_cast<float *>(m + o_thr32);
    P->seed_idx = reinterpret_cast<int64_t *>(m + o_sidx);
    P->seed_sim = reinterpret_cast<double *>(m + o_ssim);
    P->slack = reinterpret_cast<double *>(m + o_slack);
    P->best_key = reinterpret_cast<unsigned long long *>(m + o_bk);
    P->best_idx = reinterpret_cast<int32_t *>(m + o_bi);
    P->cnt = reinterpret_cast<int32_t *>(m + o_cnt);
    P->qflag = reinterpret_cast<int32_t *>(m + o_qf);
    P->gdb = reinterpret_cast<int32_t *>(m + o_gdb);
    P->counter = reinterpret_cast<unsigned long long *>(m + o_ctr);
    P->pairs = reinterpret_cast<int2 *>(m + o_pairs);
    P->psim = reinterpret_cast<double *>(m + o_psim);
    P->items = reinterpret_cast<int2 *>(m + o_items);
    P->redo = reinterpret_cast<int *>(m + o_redo);
    P->redo_counts = reinterpret_cast<unsigned *>(m + o_rc);
    P->item_ctrs = reinterpret_cast<unsigned *>(m + o_ictr);
    P->o2p = reinterpret_cast<int64_t *>(m + o_o2p);
    P->scan_argmax = reinterpret_cast<ScanArgs *>(m + o_sa);
    P->scan_filter = reinterpret_cast<ScanArgs *>(m + o_sf);
    P->seeds = reinterpret_cast<SeedArgs *>(m + o_seed);
    P->preps = reinterpret_cast<PrepArgs *>(m + o_prep);
    P->dbref = reinterpret_cast<DbRef *>(m + o_db);
    P->ts = reinterpret_cast<unsigned long long *>(m + o_ts);
    // must match the tiles compiled with kFused (every float32, bf16 and
    // int8 tile)
    P->fused = o.precision != HN_PREC_FP8;

    // host tables
    std::vector<ScanArgs> sa(n_db), sf(n_db);
    std::vector<SeedArgs> se(n_db);
    std::vector<PrepArgs> pr(n_db);
    std::vector<DbRef> dr(n_db);
    std::vector<int32_t> gdb((size_t)tp, 0);
    std::vector<int64_t> o2p((size_t)std::max<int64_t>(total_q, 1), 0);
    for (int d = 0; d < n_db; ++d) {
        const hn_index *ix = ixs[d];
        const Plan &p = plan[d], &pa = aplan[d];
        const int g = group_of[d];
        const int w = width[d];
        void *opd = op + op_off[d] * esz;
        ScanArgs A;
        memset(&A, 0, sizeof A);
        A.x = stream_of(ix, o.precision);
        A.x_stride = w;
        A.qs = opd;
        A.q_stride = w;
        A.n = ix->n;
        A.n_blocks = pa.n_blocks;
        A.chunk_blocks = pa.chunk_blocks;
        A.n_chunks = pa.n_chunks;
        A.n_qb = pa.n_qb;
        A.n_items = pa.n_items;
        A.q_count = (int32_t)q_counts[d];
        A.q_pad = (int32_t)pa.q_pad;
        A.part_val = part_val + part_off[d];
        A.part_idx = part_idx + part_off[d];
        A.redo = P->redo + P->groups[g].arg_off;
        A.redo_count = P->redo_counts + g;
        A.q_base = (int32_t)pad_base[d];
        sa[d] = A;
        A.n_blocks = p.n_blocks;
        A.chunk_blocks = p.chunk_blocks;
        A.n_chunks = p.n_chunks;
        A.n_qb = p.n_qb;
        A.n_items = p.n_items;
        A.q_pad = (int32_t)p.q_pad;
        A.part_val = nullptr;
        A.part_idx = nullptr;
        A.redo = P->redo + P->groups[g].item_off;
        A.thr = P->thr + pad_base[d];
        A.pairs = P->pairs;
        A.counter = P->counter;
        A.cap = cap;
        A.qflag = P->qflag;
        if (P->fused) {
            // the filter's flushes rescore their pairs (float32 re-check,
            // canonical float64 sim, running key) with this database's rows;
            // pairs carry padded query positions, which index the padded
            // query copy, the re-check thresholds and the keys directly
            A.psim = P->psim;
            A.best_key = P->best_key;
            A.rs_queries = P->q_buf;
            A.rs_rows = ix->rows;
            if (o.precision != HN_PREC_FP32) {  // low precision: float32 re-check first
                A.rs_major32 = ix->major32;
                A.rs_thr32 = P->thr32;
                A.rs_kp = ix->kp;
                A.rs_k = ix->k;
            }
        }
        sf[d] = A;

        SeedArgs S;
        memset(&S, 0, sizeof S);
        S.part_val = part_val + part_off[d];
        S.part_idx = part_idx + part_off[d];
        S.n_chunks = pa.n_chunks;
        S.q_pad = (int32_t)pa.q_pad;
        S.part_ld = (int32_t)pa.q_pad;
        S.shape = 32;
        S.group_size = 16 * kArgSpan;
        S.queries = P->q_buf + pad_base[d] * kDim;
        S.q = q_counts[d];
        S.rows = ix->rows;
        S.n = ix->n;
        S.k = ix->k;
        S.alpha = ix->alpha;
        S.beta = o.beta < 0.0 ? ix->alpha : o.beta;
        S.mu_major = ix->mu_major;
        S.mu_minor = ix->mu_minor;
        S.mu_full = ix->mu_full;
        scan_slack(ix, o.precision, S);
        S.qn = P->qn + pad_base[d];
        S.thr = P->thr + pad_base[d];
        S.thr32 = o.precision == HN_PREC_FP32 ? nullptr : P->thr32 + pad_base[d];
        S.seed_idx = P->seed_idx + pad_base[d];
        S.seed_sim = P->seed_sim + pad_base[d];
        S.slack = P->slack + pad_base[d];
        S.best_key = P->best_key + pad_base[d];
        S.best_idx = P->best_idx + pad_base[d];
        S.cnt = P->cnt + pad_base[d];
        S.qflag = P->qflag + pad_base[d];
        S.counter = P->counter;
        se[d] = S;

        PrepArgs Q;
        memset(&Q, 0, sizeof Q);
        Q.q = P->q_buf + pad_base[d] * kDim;
        Q.nq = q_counts[d];
        Q.q_pad = p.q_pad;
        Q.k = ix->k;
        if (o.precision == HN_PREC_FP32) {
            Q.op32 = static_cast<float *>(opd);
            Q.w32 = w;
        } else if (o.precision == HN_PREC_BF16) {
            Q.op16 = static_cast<uint16_t *>(opd);
            Q.w16 = w;
        } else if (o.precision == HN_PREC_FP8) {
            Q.op8 = static_cast<uint8_t *>(opd);
            Q.w8 = w;
        } else {
            Q.opi = static_cast<int8_t *>(opd);
            Q.w8 = w;
        }
        Q.qn = P->qn + pad_base[d];
        pr[d] = Q;

        DbRef D;
        D.rows = ix->rows;
        D.major32 = ix->major32;
        D.n = ix->n;
        D.kp = ix->kp;
        D.k = ix->k;
        D.alpha = ix->alpha;
        D.beta = o.beta < 0.0 ? ix->alpha : o.beta;
        D.mu_major = ix->mu_major;
        D.mu_minor = ix->mu_minor;
        D.mu_full = ix->mu_full;
        D.pad_base = pad_base[d];
        D.q = q_counts[d];
        D.out_base = out_base[d];
        dr[d] = D;
        for (int64_t i = 0; i < p.q_pad; ++i) gdb[pad_base[d] + i] = d;
        for (int64_t i = 0; i < q_counts[d]; ++i) o2p[out_base[d] + i] = pad_base[d] + i;
    }
    hipError_t e = hipSuccess;
    auto up = [&](void *dst, const void *src, size_t nbytes) {
        if (e == hipSuccess && nbytes) e = hipMemcpy(dst, src, nbytes, hipMemcpyHostToDevice);
    };
    up(P->scan_argmax, sa.data(), sizeof(ScanArgs) * n_db);
    up(P->scan_filter, sf.data(), sizeof(ScanArgs) * n_db);
    up(P->seeds, se.data(), sizeof(SeedArgs) * n_db);
    up(P->preps, pr.data(), sizeof(PrepArgs) * n_db);
    up(P->dbref, dr.data(), sizeof(DbRef) * n_db);
    up(P->gdb, gdb.data(), sizeof(int32_t) * gdb.size());
    up(P->o2p, o2p.data(), sizeof(int64_t) * (size_t)total_q);
    up(P->items, items.data(), sizeof(int2) * items.size());
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        plan_destroy(P);
        return fail(HN_ERR_DEVICE, "plan set-up failed: %s", hipGetErrorString(e));
    }
    *out = P;
    return HN_OK;
}

extern "C" void hn_multi_plan_free(hn_multi_plan *plan) {
    if (!plan) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) {
        (void)hipSetDevice(plan->device);
        plan_destroy(plan);
        (void)hipSetDevice(cur);
        return;
    }
    plan_destroy(plan);
}

extern "C" int hn_multi_plan_info(const hn_multi_plan *plan, int64_t *total_queries,
                                  int64_t *work_items, int32_t *scan_launches) {
    clear_error();
    if (!plan) return fail(HN_ERR_INVALID_ARG, "null plan");
    if (total_queries) *total_queries = plan->total_q;
    if (work_items) *work_items = plan->total_items;
    if (scan_launches) *scan_launches = 2 * (int32_t)plan->groups.size();
    return HN_OK;
}

extern "C" int hn_multi_batch_times(const hn_multi_plan *plan, double *ms, void *stream) {
    clear_error();
    if (!plan || !ms) return fail(HN_ERR_INVALID_ARG, "null argument");
    std::vector<unsigned long long> ts((size_t)plan->n_db + 1);
    hipStream_t s = (hipStream_t)stream;
    HN_HIP(hipMemcpyAsync(ts.data(), plan->ts, sizeof(unsigned long long) * ts.size(),
                          hipMemcpyDeviceToHost, s));
    HN_HIP(hipStreamSynchronize(s));
    int khz = 0;
    HN_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, plan->device));
    if (khz <= 0) return fail(HN_ERR_DEVICE, "no constant-rate clock rate");
    for (int d = 0; d < plan->n_db; ++d)
        ms[d] = ts[1 + d] >= ts[0] && ts[1 + d] != 0ull
                    ? (double)(ts[1 + d] - ts[0]) / (double)khz
                    : 0.0;
    return HN_OK;
}

extern "C" int hn_multi_search(hn_multi_plan *plan, const float *queries, int64_t *out_idx,
                               double *out_sim, int32_t use_graph, void *stream) {
    clear_error();
    if (!plan) return fail(HN_ERR_INVALID_ARG, "null plan");
    if (plan->total_q == 0) return HN_OK;
    if (!queries || !out_idx || !out_sim) return fail(HN_ERR_INVALID_ARG, "null queries or outputs");
    if (!aligned16(queries)) return fail(HN_ERR_INVALID_ARG, "queries must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) return enqueue(plan, queries, out_idx, out_sim, s);
    if (!plan->exec || plan->g_q != queries || plan->g_idx != out_idx || plan->g_sim != out_sim) {
        if (plan->exec) {
            HN_HIP(hipGraphExecDestroy(plan->exec));
            plan->exec = nullptr;
        }
        HN_HIP(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue(plan, queries, out_idx, out_sim, plan->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(plan->cap_stream, &g);
        if (rc) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return rc;
        }
        HN_HIP(e);
        const hipError_t e2 = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HN_HIP(e2);
        plan->g_q = queries;
        plan->g_idx = out_idx;
        plan->g_sim = out_sim;
    }
    HN_HIP(hipGraphLaunch(plan->exec, s));
    return HN_OK;
}
