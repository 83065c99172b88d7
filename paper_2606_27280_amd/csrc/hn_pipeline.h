// Device side of the search pipeline, shared by the single-database search
// (hn_search.hip) and the multi-database search (hn_multi.hip): query
// preparation, seed selection with the bound slack, float64 rescoring, the
// deterministic argmax, the exact overflow fallback, the output writer and
// the exhaustive baseline's helpers.  Internal to the library.
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>

#include "hn_scan.h"

namespace hn {
namespace {

constexpr double kU32 = 1.0 / 8388608.0;               // 2^-23 (covers RNE and truncation)
constexpr double kU64 = 1.0 / 9007199254740992.0;      // 2^-53
constexpr double kUbf16 = 1.0 / 256.0;                 // 2^-8, bf16 round-to-nearest
constexpr int kIdxNone = 0x7fffffff;
// Scan bookkeeping words zeroed by prep_queries: [0,8) item counters of the
// first scan, [8,16) of the second, 16 and 17 their redo counts.
constexpr int kWorkWords = 32;

// ---------------------------------------------------------------- queries

struct QNorm {
    double major, minor, full;  // rounded-up float64 block norms
    double res16;               // ||bf16(q[:k]) - q[:k]||, rounded up
    double res8;                // ||s8 fp8(q[:k] / s8) - q[:k]||, rounded up
    double resi;                // ||si code - q[:k]|| of the int8 operand, rounded up
    float sc8;                  // s8: power-of-two scale of the fp8 operand
    float sci;                  // si: power-of-two scale of the int8 operand
    int bad;                    // non-finite component
};

__device__ __forceinline__ float bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// Query operands for the scans (any pointer may be NULL), widths per stream.
struct PrepArgs {
    const float *q;
    int64_t nq, q_pad;
    int k;
    int w32, w16, w8;
    float *op32;
    uint16_t *op16;
    uint8_t *op8;
    int8_t *opi;  // int8 codes, width w8
    QNorm *qn;
    unsigned *work;
};

__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Query i (of the padded batch), one wave: norms and the float32 / bf16 /
// fp8 / int8 operands.  Each lane takes two of the 128 values (and operand
// columns lane, lane + 64); the float64 sums are reduced across the wave and
// every norm is rounded up by (1 + 2^-40), which covers their rounding in any
// summation order.
__device__ __forceinline__ void prep_wave(const PrepArgs &P, const int64_t i, const int lane) {
    if (i >= P.q_pad) return;
    if (i >= P.nq) {
        for (int c = lane; c < P.w32; c += 64)
            if (P.op32) P.op32[i * P.w32 + c] = 0.0f;
        for (int c = lane; c < P.w16; c += 64)
            if (P.op16) P.op16[i * P.w16 + c] = 0;
        if (lane < P.w8) {
            if (P.op8) P.op8[i * P.w8 + lane] = 0;
            if (P.opi) P.opi[i * P.w8 + lane] = 0;
        }
        return;
    }
    const int k = P.k;
    const float *v = P.q + i * kDim;
    const float2 f2 = reinterpret_cast<const float2 *>(v)[lane];
    double sM = 0, sm = 0, sr = 0;
    float amax = 0.0f;
    int bad = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int j = 2 * lane + u;
        const float f = u ? f2.y : f2.x;
        bad |= !isfinite(f);
        const double d = (double)f;
        if (j < k) {
            sM = fma(d, d, sM);
            const double b = (double)bf16_rne(f);
            sr = fma(b - d, b - d, sr);
            amax = fmaxf(amax, fabsf(f));
        } else {
            sm = fma(d, d, sm);
        }
    }
    sM = wave_sum64(sM);
    sm = wave_sum64(sm);
    sr = wave_sum64(sr);
    for (int o = 32; o > 0; o >>= 1) {
        amax = fmaxf(amax, __shfl_xor(amax, o));
        bad |= __shfl_xor(bad, o);
    }
    const bool finite = !bad;
    const double up = 1.0 + ldexp(1.0, -40);
    QNorm r;
    r.major = sqrt(sM) * up;
    r.minor = sqrt(sm) * up;
    r.full = sqrt(sM + sm) * up;
    r.res16 = sqrt(sr) * up;
    r.res8 = 0.0;
    r.sc8 = 1.0f;
    r.resi = 0.0;
    r.sci = 1.0f;
    r.bad = finite ? 0 : 1;
    for (int c = lane; c < P.w32; c += 64)
        if (P.op32) P.op32[i * P.w32 + c] = (c < k && finite) ? v[c] : 0.0f;
    for (int c = lane; c < P.w16; c += 64)
        if (P.op16)
            P.op16[i * P.w16 + c] =
                (c < k && finite) ? (uint16_t)(__float_as_uint(bf16_rne(v[c])) >> 16) : 0;
    // fp8 / int8 (w8 <= 32): lane c codes column c
    const float f8 = (lane < P.w8 && lane < k && finite) ? v[lane] : 0.0f;
    if (P.op8) {
        const float sc = finite ? fp8_scale_for(amax) : 1.0f;
        const float inv = 1.0f / sc;  // exact: a power of two
        double e2 = 0.0;
        if (lane < P.w8) {
            const uint8_t code = fp8_e4m3(f8 * inv);
            P.op8[i * P.w8 + lane] = code;
            const double e = (double)fp8_e4m3_value(code) * (double)sc - (double)f8;
            e2 = e * e;
        }
        r.res8 = sqrt(wave_sum64(e2)) * up;
        r.sc8 = sc;
    }
    if (P.opi) {
        const float sc = finite ? int8_scale_for(amax) : 1.0f;
        const float inv = 1.0f / sc;  // exact: a power of two
        double e2 = 0.0;
        if (lane < P.w8) {
            const int8_t code = int8_code(f8 * inv);
            P.opi[i * P.w8 + lane] = code;
            const double e = (double)code * (double)sc - (double)f8;
            e2 = e * e;
        }
        r.resi = sqrt(wave_sum64(e2)) * up;
        r.sci = sc;
    }
    if (lane == 0) P.qn[i] = r;
}

// One wave per (padded) query, 4 per work-group; the first group also zeroes
// the scan bookkeeping words.
__global__ __launch_bounds__(256) void prep_queries(PrepArgs P) {
    if (P.work && blockIdx.x == 0 && (int)threadIdx.x < kWorkWords) P.work[threadIdx.x] = 0u;
    prep_wave(P, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// ---------------------------------------------------------------- seed

struct SeedArgs {
    const float *part_val;
    const int32_t *part_idx;
    int32_t n_chunks, q_pad;
    int32_t part_ld;            // row stride of the partials (the argmax scan's q_pad)
    int32_t topk;               // > 1: L is a bound on the topk-th best sim
    int32_t shape, group_size;  // scan tile shape (16 or 32) and entries per lane group
    const float *queries;
    int64_t q;
    const float *rows;
    int64_t n;
    int32_t k;
    double alpha, beta;  // beta = alpha for exact search
    double mu_major, mu_minor, mu_full;
    // scan slack: worst case rel * major * mu, or the residual-norm form
    // res_q * res_mu + major * res_x + acc_rel * (major + res_q) * res_mu,
    // or the smaller of the two; plus abs
    double scan_rel, scan_mu, scan_abs;
    int scan_res;  // 0: worst case; 1: min(worst case, residual); 2: residual
    int scaled;    // 1: fp8, 2: int8 operands (residuals of the scaled copies,
                   // thresholds in scan units s_q s_x); 0: neither
    double res_mu, res_x, res_acc_rel;
    double scale_x;  // scaled copies: power-of-two scale of the entry copy
    const double *lower;  // given L (filter-only, learned or no seed); NULL: plain seed
    const int64_t *lower_idx;  // entry of each given L, or NULL (none)
    // single-pass window (NULL: none): exact width 2 (beta + eps_q) in scan
    // units, the float width the scan subtracts (widened for its rounding),
    // and the scan's starting running maximum T_q + width
    double *win;
    float *win_scan, *init_best;
    double bound_mu;  // max norm of the scanned entry copy (bounds |s~|)
    const QNorm *qn;
    float *thr;           // [q_pad]: scan threshold T_q (+inf for padding)
    float *thr32;         // [q]: float32 re-check threshold, or NULL
    int64_t *seed_idx;
    double *seed_sim;
    double *slack;
    unsigned long long *best_key;
    int32_t *best_idx;
    int32_t *cnt;
    int32_t *qflag;
    unsigned long long *counter;
};

__device__ __forceinline__ float round_down_f32(double v) { return __double2float_rd(v); }

// Entry of slot v of an argmax lane group gid = span * G + g, for the scan's
// tile shape: per block of the span, 16x16 tiles give 4 consecutive entries
// (rows 4 g + v % 4), 32x32 tiles 16 entries (rows 8 (w / 4) + 4 g + w % 4,
// w = v % 16); slot v lies in block span * kArgSpan + v / (entries per block).
__device__ __forceinline__ int64_t group_entry(int shape, int gid, int v) {
    if (shape == 16)
        return ((int64_t)(gid >> 2) * kArgSpan + (v >> 2)) * 16 + 4 * (gid & 3) + (v & 3);
    const int w = v & 15;
    return ((int64_t)(gid >> 1) * kArgSpan + (v >> 4)) * 32 + 8 * (w >> 2) + 4 * (gid & 1) +
           (w & 3);
}

// Canonical sim of the lane's entry of lane group gid (-inf and e = -1 for
// no entry).  Entries whose float32 major dot lies more than 2 ||q_m|| mu_m
// (plus a margin for the float32 rounding) below the group's best major dot
// are skipped: by Eq. 3 applied to both, such an entry's sim is below the
// best-major entry's, so the group's best sim is unchanged while most lanes
// read only the row's K-prefix.
__device__ __forceinline__ double group_sim(const SeedArgs &S, int gid, int lane,
                                            const float *qv, double q_minor, int64_t &e) {
    e = -1;
    float maj = -INFINITY;
    if (gid >= 0 && lane < S.group_size) {
        const int64_t c = group_entry(S.shape, gid, lane);
        if (c < S.n) {
            const float *xv = S.rows + c * kDim;
            const int k4 = S.k & ~3;
            float d = 0.0f;
            for (int j = 0; j < k4; j += 4) {
                const float4 x4 = *reinterpret_cast<const float4 *>(xv + j);
                const float4 q4 = *reinterpret_cast<const float4 *>(qv + j);
                d = fmaf(q4.x, x4.x, d);
                d = fmaf(q4.y, x4.y, d);
                d = fmaf(q4.z, x4.z, d);
                d = fmaf(q4.w, x4.w, d);
            }
            for (int j = k4; j < S.k; ++j) d = fmaf(qv[j], xv[j], d);
            maj = d;
            e = c;
        }
    }
    float mm = maj;
    for (int o = 32; o > 0; o >>= 1) mm = fmaxf(mm, __shfl_xor(mm, o));
    const float tau = (float)(2.0 * q_minor * S.mu_minor) * (1.0f + 0x1p-10f) + 1e-4f;
    if (e >= 0 && maj >= mm - tau) return sim64(qv, S.rows + e * kDim);
    e = -1;
    return -INFINITY;
}

// Exact top-k seed: the topk-th largest of distinct real entries' canonical
// sims is at most the query's topk-th best sim, so it bounds the survivors
// like L does for top-1.  The entries: for each of the m = min(chunks,
// 2 topk) best chunks, in (score desc, chunk asc) order, the best sim of its
// winning lane group (the group holds the chunk's largest scan score, so
// these are the near-best entries of distinct chunks).  -inf if fewer than
// topk such entries exist.  Chunk r's value sits in lane r % 64, slot r / 64.
// Per-chunk partials read per step by each lane of a seed wave.
constexpr int kPartBatch = 8;

__device__ __forceinline__ double topk_lower(const SeedArgs &S, const int64_t i, const int lane,
                                          const float *qv, double q_minor) {
    const int m = min(S.n_chunks, min(2 * S.topk, 256));
    double cs[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) cs[t] = -INFINITY;
    float pv = INFINITY;
    int pc = -1;
    int found = 0;  // chunks with a real entry
    // The partials are read kPartBatch per lane at a time (independent loads
    // in flight together); with at most 64 x kPartBatch chunks they are read
    // once and stay in registers for all the rounds.
    float v[kPartBatch];
    auto load = [&](int c0) {
#pragma unroll
        for (int u = 0; u < kPartBatch; ++u) {
            const int c = c0 + 64 * u;
            v[u] = c < S.n_chunks ? S.part_val[(int64_t)c * S.part_ld + i] : -INFINITY;
        }
    };
    const bool resident = S.n_chunks <= 64 * kPartBatch;
    if (resident) load(lane);
    for (int r = 0; r < m; ++r) {
        // the next chunk after (pv, pc) in (score desc, chunk asc) order
        float bv = -INFINITY;
        int bc = -1;
        for (int c0 = lane; c0 < S.n_chunks; c0 += 64 * kPartBatch) {
            if (!resident) load(c0);
#pragma unroll
            for (int u = 0; u < kPartBatch; ++u) {
                const int c = c0 + 64 * u;
                const bool after = v[u] < pv || (v[u] == pv && c > pc);
                if (c < S.n_chunks && after && (bc < 0 || v[u] > bv)) {
                    bv = v[u];
                    bc = c;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int oc = __shfl_xor(bc, o);
            if (oc >= 0 && (bc < 0 || ov > bv || (ov == bv && oc < bc))) {
                bv = ov;
                bc = oc;
            }
        }
        bc = __builtin_amdgcn_readfirstlane(bc);
        if (bc < 0) break;
        pv = bv;
        pc = bc;
        const int gid = S.part_idx[(int64_t)bc * S.part_ld + i];
        int64_t e;
        double sv = group_sim(S, gid, lane, qv, q_minor, e);
        for (int o = 32; o > 0; o >>= 1) sv = fmax(sv, __shfl_xor(sv, o));
        if (sv == -INFINITY) continue;
        if (lane == found % 64) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u == found / 64) cs[u] = sv;
        }
        ++found;
    }
    if (found < S.topk) return -INFINITY;
    // the topk-th largest value: topk pops of the wave maximum, one copy each
    double L = -INFINITY;
    for (int r = 0; r < S.topk; ++r) {
        double mv = -INFINITY;
        int ms = -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (cs[u] > mv) {
                mv = cs[u];
                ms = u;
            }
        double wv = mv;
        for (int o = 32; o > 0; o >>= 1) wv = fmax(wv, __shfl_xor(wv, o));
        const unsigned long long owners = __ballot(ms >= 0 && mv == wv);
        if ((int)lane == __builtin_ffsll((long long)owners) - 1) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u == ms) cs[u] = -INFINITY;
        }
        L = wv;
    }
    return L;
}

// Query i, one wave: reduce the per-chunk argmax partials, rescore every
// entry of the winning lane group in float64 (one lane each) and keep the
// best (sim desc, index asc) as the seed; then the slack and thresholds.
__device__ __forceinline__ void seed_one(const SeedArgs &S, const int64_t i, const int lane) {
    if (i >= S.q_pad) return;
    if (i >= S.q) {
        if (lane == 0) {
            S.thr[i] = INFINITY;
            if (S.win_scan) {
                S.win_scan[i] = 0.0f;
                S.init_best[i] = -INFINITY;
            }
        }
        return;
    }
    const QNorm qn = S.qn[i];
    if (qn.bad) {
        if (lane == 0) {
            S.best_idx[i] = kIdxNone;
            S.cnt[i] = 0;
            S.qflag[i] = 0;
            S.thr[i] = INFINITY;
            if (S.thr32) S.thr32[i] = INFINITY;
            S.seed_idx[i] = -1;
            S.seed_sim[i] = NAN;
            S.slack[i] = NAN;
            S.best_key[i] = 0;
            if (S.win_scan) {
                S.win[i] = 0.0;
                S.win_scan[i] = 0.0f;
                S.init_best[i] = INFINITY;
            }
        }
        return;
    }
    const float *qv = S.queries + i * kDim;
    double L;
    int64_t b = -1;
    if (S.lower) {
        L = S.lower[i];
        b = S.lower_idx ? S.lower_idx[i] : -1;
    } else if (S.topk > 1) {
        L = topk_lower(S, i, lane, qv, qn.minor);
    } else {
        float bv = -INFINITY;
        int bi = -1;
        // the query's per-chunk partials, kPartBatch independent loads in
        // flight per lane (the merge is a lexicographic maximum: any order)
        for (int c0 = lane; c0 < S.n_chunks; c0 += 64 * kPartBatch) {
            float v[kPartBatch];
            int x[kPartBatch];
#pragma unroll
            for (int u = 0; u < kPartBatch; ++u) {
                const int c = c0 + 64 * u;
                const bool ok = c < S.n_chunks;
                v[u] = ok ? S.part_val[(int64_t)c * S.part_ld + i] : -INFINITY;
                x[u] = ok ? S.part_idx[(int64_t)c * S.part_ld + i] : -1;
            }
#pragma unroll
            for (int u = 0; u < kPartBatch; ++u) lex_merge(bv, bi, v[u], x[u]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            lex_merge(bv, bi, ov, oi);
        }
        int64_t e;
        double sv = group_sim(S, bi, lane, qv, qn.minor, e);
        for (int o = 32; o > 0; o >>= 1) {
            const double os = __shfl_xor(sv, o);
            const int64_t oe = __shfl_xor(e, o);
            if (oe >= 0 && (e < 0 || os > sv || (os == sv && oe < e))) {
                sv = os;
                e = oe;
            }
        }
        L = sv;
        b = e;
    }
    if (lane != 0) return;
    S.best_idx[i] = kIdxNone;
    S.cnt[i] = 0;
    S.qflag[i] = 0;
    // slack: scan rounding + stored-norm excess (Eq. 3) + float64 evaluation
    double es = S.scan_rel * qn.major * S.scan_mu;
    if (S.scan_res) {
        const double rq = S.scaled == 1 ? qn.res8 : (S.scaled == 2 ? qn.resi : qn.res16);
        const double er =
            rq * S.res_mu + qn.major * S.res_x + S.res_acc_rel * (qn.major + rq) * S.res_mu;
        es = S.scan_res == 2 ? er : fmin(es, er);
    }
    es += S.scan_abs;
    double en = fmax(0.0, qn.minor * S.mu_minor - S.alpha);
    double e64 = gamma_n(kDim, kU64) * qn.full * S.mu_full;
    double eps = (es + en + e64) * (1.0 + ldexp(1.0, -30)) + ldexp(1.0, -40);
    // fp8 and int8 scans score q~ . x~ with q = s_q q~ and x = s_x x~ (powers
    // of two): the threshold in scan units is the bound divided by s_q s_x
    const double unit =
        S.scaled ? 1.0 / ((double)(S.scaled == 1 ? qn.sc8 : qn.sci) * S.scale_x) : 1.0;
    S.thr[i] = round_down_f32((L - S.beta - eps) * unit);
    if (S.win_scan) {
        // |s~| <= (||q_M|| + r_q) max ||x^_M|| (1 + 2^-20), in scan units
        const double rq = S.scaled == 1   ? qn.res8
                          : S.scaled == 2 ? qn.resi
                                          : (S.scan_res ? qn.res16 : 0.0);
        const double bound = (qn.major + rq) * S.bound_mu * unit * (1.0 + ldexp(1.0, -20));
        const double w = 2.0 * (S.beta + eps) * unit;
        S.win[i] = w;
        S.win_scan[i] = __double2float_ru(w + ldexp(1.0, -21) * (bound + w));
        S.init_best[i] = round_down_f32((L - S.beta - eps) * unit + w);
    }
    if (S.thr32) {
        double e32 = gamma_n(S.k, kU32) * qn.major * S.mu_major + S.k * ldexp(1.0, -125);
        double eps32 = (e32 + en + e64) * (1.0 + ldexp(1.0, -30)) + ldexp(1.0, -40);
        S.thr32[i] = round_down_f32(L - S.beta - eps32);
    }
    S.seed_idx[i] = b;
    S.seed_sim[i] = L;
    S.slack[i] = eps;
    S.best_key[i] = b >= 0 ? key_of(L) : 0ull;
}

// One wave per query; also zeroes the survivor-list counter.
__global__ __launch_bounds__(256) void seed_kernel(SeedArgs S) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i == 0 && lane == 0) *S.counter = 0;
    seed_one(S, i, lane);
}

// The scan stream and query operands of a precision.
int stream_width(const hn_index *ix, int precision) {
    return precision == HN_PREC_FP32 ? ix->kp : (precision == HN_PREC_BF16 ? ix->kb : ix->k8);
}
const void *stream_of(const hn_index *ix, int precision) {
    return precision == HN_PREC_FP32   ? (const void *)ix->major32
           : precision == HN_PREC_BF16 ? (const void *)ix->major16
           : precision == HN_PREC_FP8  ? (const void *)ix->major8
                                       : (const void *)ix->major_i8;
}
int check_precision(const hn_index *ix, int precision) {
    if (precision != HN_PREC_FP32 && precision != HN_PREC_BF16 && precision != HN_PREC_FP8 &&
        precision != HN_PREC_INT8)
        return fail(HN_ERR_UNSUPPORTED, "precision %d is not available", precision);
    if ((precision == HN_PREC_FP8 || precision == HN_PREC_INT8) && ix->k8 == 0)
        return fail(HN_ERR_UNSUPPORTED, "the %s scan needs k <= 32 (k = %d)",
                    precision == HN_PREC_FP8 ? "fp8" : "int8", ix->k);
    return HN_OK;
}

// Survivor-list capacity of the two-pass search: max(4096, n / 256) pairs
// per query, at least 2^20 and at most 2^28.
int64_t default_cap(int64_t n, int64_t q) {
    int64_t per = std::max<int64_t>(4096, n / 256);
    int64_t c = q * per;
    return std::min<int64_t>(std::max<int64_t>(c, (int64_t)1 << 20), (int64_t)1 << 28);
}

// The scan-rounding part of the slack for a precision (Section 3.3's bound
// made admissible for the low-precision scans).
inline void scan_slack(const hn_index *ix, int precision, SeedArgs &S) {
    if (precision == HN_PREC_FP32) {
        S.scan_rel = gamma_n(ix->k, kU32);
        S.scan_mu = ix->mu_major;
        S.scan_abs = ix->k * ldexp(1.0, -125);
        S.scan_res = 0;
    } else if (precision == HN_PREC_BF16) {
        // worst case: both roundings relative 2^-8, then float32 accumulation
        const double ub = kUbf16;
        S.scan_rel = (2 * ub + ub * ub) + gamma_n(ix->k, kU32) * (1 + ub) * (1 + ub);
        S.scan_mu = ix->mu_major;
        S.scan_abs = ix->k * ldexp(1.0, -125);
        // residual form (Cauchy-Schwarz on the rounding residuals):
        // |sum(q^x^ - qx)| <= ||q^-q|| ||x^|| + ||q|| ||x^-x||, plus accumulation
        S.scan_res = 1;
        S.res_mu = ix->mu_major16;
        S.res_x = ix->res16;
        S.res_acc_rel = gamma_n(ix->k, kU32);
    } else if (precision == HN_PREC_FP8) {
        // fp8: the residual form only (subnormal codes have no relative
        // bound); the products are summed by the bf16 matrix core (the codes
        // are decoded exactly to bf16), float32 accumulation.
        S.scan_rel = 0.0;
        S.scan_mu = 0.0;
        S.scan_abs = ix->k * ldexp(1.0, -125);
        S.scan_res = 2;
        S.scaled = 1;
        S.scale_x = ix->scale8;
        S.res_mu = ix->mu_major8;
        S.res_x = ix->res8;
        S.res_acc_rel = gamma_n(ix->k, kU32);
    } else {
        // int8: the residual form; the matrix core sums integer products
        // exactly in int32 (|sum| <= 32 * 127^2 < 2^24, so the conversion to
        // float32 is exact too): no accumulation term.
        S.scan_rel = 0.0;
        S.scan_mu = 0.0;
        S.scan_abs = 0.0;
        S.scan_res = 2;
        S.scaled = 2;
        S.scale_x = ix->scale_i8;
        S.res_mu = ix->mu_major_i8;
        S.res_x = ix->res_i8;
        S.res_acc_rel = 0.0;
    }
}

// ------------------------------------------------------ rescoring & argmax

// Per-database constants of a multi-database search, looked up by the
// database of each (padded) query position.
struct DbRef {
    const float *rows;      // [n][128]
    const float *major32;   // [n_pad][kp]
    int64_t n;
    int32_t kp, k;
    double alpha, beta, mu_major, mu_minor, mu_full;
    int64_t pad_base;       // first padded query position of the database
    int64_t q;              // its real queries
    int64_t out_base;       // their first position in the caller's outputs
};

struct RescoreArgs {
    const int2 *pairs;
    const float *pair_val;     // window mode: scan score of the pair
    const unsigned long long *counter;
    int64_t cap;
    const float *queries, *rows;
    const float *major32;      // re-check stream (low-precision scans)
    int32_t kp, k;
    const float *thr32;        // re-check / window threshold per query
    double *psim;              // [cap]
    unsigned long long *best_key;
    int32_t *best_idx;
    int32_t *cnt;
    const int64_t *seed_idx;
    const double *seed_sim;
    int64_t q;
    int count;  // count survivors per query (only when requested)
    const DbRef *db;     // multi-database: per-database rows, stream, k
    const int32_t *gdb;  //   and the database of each query position (or NULL)
};

__device__ __forceinline__ int64_t pair_count(const RescoreArgs &R) {
    unsigned long long c = *R.counter;
    return (int64_t)c < R.cap ? (int64_t)c : R.cap;
}

// The window re-filter (pair_val >= thr32[query]): after the single pass's
// threshold refinement nearly every pair falls below it, so the kernel is
// bound by reading the pairs.  Each thread takes kWinBatch pairs per step
// with their loads in flight together, and only the kept pairs get a psim
// (the tie kernel applies the same test before it reads one).
constexpr int kWinBatch = 4;

__device__ __forceinline__ void rescore_window_pairs(const RescoreArgs &R, int64_t m) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p0 = (int64_t)blockIdx.x * 256 + threadIdx.x; p0 < m;
         p0 += kWinBatch * stride) {
        int2 pr[kWinBatch];
        float pv[kWinBatch];
#pragma unroll
        for (int u = 0; u < kWinBatch; ++u) {
            const int64_t p = p0 + u * stride;
            pr[u] = p < m ? R.pairs[p] : make_int2(-1, -1);
            pv[u] = p < m ? R.pair_val[p] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kWinBatch; ++u) {
            const int64_t p = p0 + u * stride;
            const bool valid = pr[u].x >= 0;
            if (valid && R.count) atomicAdd(&R.cnt[pr[u].x], 1);
            if (!(valid && pv[u] >= R.thr32[pr[u].x])) continue;
            const double s =
                sim64(R.queries + (int64_t)pr[u].x * kDim, R.rows + (int64_t)pr[u].y * kDim);
            const unsigned long long kk = key_of(s);
            if (kk > R.best_key[pr[u].x]) atomicMax(&R.best_key[pr[u].x], kk);
            R.psim[p] = s;
        }
    }
}

// MODE 0: plain; 1: float32 re-check against thr32 first; 2: window re-filter.
template <int MODE>
__global__ __launch_bounds__(256) void rescore_kernel(RescoreArgs R) {
    const int64_t m = pair_count(R);
    if constexpr (MODE == 2) {
        rescore_window_pairs(R, m);
        return;
    }
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * 256) {
        const int2 pr = R.pairs[p];
        const float *qv = R.queries + (int64_t)pr.x * kDim;
        const float *rows = R.rows, *major32 = R.major32;
        int kp = R.kp, k = R.k;
        if (R.gdb) {
            const DbRef &D = R.db[R.gdb[pr.x]];
            rows = D.rows;
            major32 = D.major32;
            kp = D.kp;
            k = D.k;
        }
        if (R.count) atomicAdd(&R.cnt[pr.x], 1);
        bool keep = true;
        if (MODE == 1) {
            // the float32 prefix stream is zero padded to kp (a multiple of
            // 4) and the query row holds 128 values: whole float4 groups, the
            // threshold and four groups of both rows in flight together
            // (fp8 re-check 0.494 to 0.477 ms on 5.3 M pairs)
            const float thr = R.thr32[pr.x];
            const float *xm = major32 + (int64_t)pr.y * kp;
            float s = 0.0f;
            for (int j0 = 0; j0 < k; j0 += 16) {
                float4 x4[4], q4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = j0 + 4 * u < k;
                    x4[u] = ok ? *reinterpret_cast<const float4 *>(xm + j0 + 4 * u)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
                    q4[u] = ok ? *reinterpret_cast<const float4 *>(qv + j0 + 4 * u)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (j0 + 4 * u < k) {
                        s = fmaf(q4[u].x, x4[u].x, s);
                        s = fmaf(q4[u].y, x4[u].y, s);
                        s = fmaf(q4[u].z, x4[u].z, s);
                        s = fmaf(q4[u].w, x4[u].w, s);
                    }
                }
            }
            keep = s >= thr;
        } else if (MODE == 2) {
            keep = R.pair_val[p] >= R.thr32[pr.x];
        }
        double s = -INFINITY;
        if (keep) {
            s = sim64(qv, rows + (int64_t)pr.y * kDim);
            // best_key starts at the seed's key and only grows: most
            // survivors are below it and need no atomic
            const unsigned long long kk = key_of(s);
            if (kk > R.best_key[pr.x]) atomicMax(&R.best_key[pr.x], kk);
        }
        R.psim[p] = s;
    }
}

__global__ __launch_bounds__(256) void tie_kernel(RescoreArgs R) {
    const int64_t m = pair_count(R);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m + R.q;
         p += (int64_t)gridDim.x * 256) {
        if (p < m) {
            const int2 pr = R.pairs[p];
            // window pairs below the re-filter threshold have no psim
            if (R.pair_val && !(R.pair_val[p] >= R.thr32[pr.x])) continue;
            const double s = R.psim[p];
            if (s == -INFINITY) continue;
            if (key_of(s) == R.best_key[pr.x]) atomicMin(&R.best_idx[pr.x], pr.y);
        } else if (R.seed_idx) {
            const int64_t qi = p - m;
            const int64_t b = R.seed_idx[qi];
            if (b >= 0 && key_of(R.seed_sim[qi]) == R.best_key[qi])
                atomicMin(&R.best_idx[qi], (int32_t)b);
        }
    }
}

// Exact completion of queries whose survivors did not fit the pair list: one
// work-group per flagged query scans every entry.  full = 1 evaluates every
// entry (exhaustive baseline); otherwise the float64 major score with the
// rigorous float64 slack decides which entries get the full sim.
struct FallbackArgs {
    const int32_t *qflag;
    const QNorm *qn;
    const float *queries, *rows;
    int64_t q, n;
    int32_t k, full;
    double beta, alpha, mu_major, mu_minor, mu_full;
    const double *seed_sim;
    unsigned long long *best_key;
    int32_t *best_idx;
    int32_t *cnt;
    const DbRef *db;     // multi-database (or NULL): per-database constants
    const int32_t *gdb;
};

__global__ __launch_bounds__(256) void fallback_kernel(FallbackArgs F) {
    __shared__ unsigned long long sk[256];
    __shared__ int si[256];
    __shared__ int sc[256];
    for (int64_t qi = blockIdx.x; qi < F.q; qi += gridDim.x) {
        // uniform: the reduction below holds barriers
        if (!__builtin_amdgcn_readfirstlane(F.qflag[qi])) continue;
        const float *qv = F.queries + qi * kDim;
        const QNorm qn = F.qn[qi];
        const float *rows = F.rows;
        int64_t n = F.n;
        int k = F.k;
        double alpha = F.alpha, beta = F.beta, mu_major = F.mu_major, mu_minor = F.mu_minor,
               mu_full = F.mu_full;
        if (F.gdb) {
            const DbRef &D = F.db[__builtin_amdgcn_readfirstlane(F.gdb[qi])];
            rows = D.rows;
            n = D.n;
            k = D.k;
            alpha = D.alpha;
            beta = D.beta;
            mu_major = D.mu_major;
            mu_minor = D.mu_minor;
            mu_full = D.mu_full;
        }
        double lim = -INFINITY;
        if (!F.full) {
            double en = fmax(0.0, qn.minor * mu_minor - alpha);
            double e = gamma_n(k, kU64) * qn.major * mu_major + en +
                       gamma_n(kDim, kU64) * qn.full * mu_full;
            lim = F.seed_sim[qi] - beta - e * (1.0 + ldexp(1.0, -30)) - ldexp(1.0, -40);
        }
        unsigned long long bk = 0;
        int bi = kIdxNone, c = 0;
        for (int64_t e = threadIdx.x; e < n; e += 256) {
            const float *xv = rows + e * kDim;
            if (!F.full) {
                double s = 0.0;
                for (int j = 0; j < k; ++j) s = fma((double)qv[j], (double)xv[j], s);
                if (s < lim) continue;
            }
            ++c;
            unsigned long long kk = key_of(sim64(qv, xv));
            if (kk > bk || (kk == bk && (int)e < bi)) {
                bk = kk;
                bi = (int)e;
            }
        }
        sk[threadIdx.x] = bk;
        si[threadIdx.x] = bi;
        sc[threadIdx.x] = c;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                unsigned long long ok = sk[threadIdx.x + o];
                int oi = si[threadIdx.x + o];
                if (ok > sk[threadIdx.x] || (ok == sk[threadIdx.x] && oi < si[threadIdx.x])) {
                    sk[threadIdx.x] = ok;
                    si[threadIdx.x] = oi;
                }
                sc[threadIdx.x] += sc[threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            F.best_key[qi] = sk[0];
            F.best_idx[qi] = si[0];
            F.cnt[qi] = sc[0];
        }
        __syncthreads();
    }
}

struct FinalArgs {
    int64_t q;
    const QNorm *qn;
    const unsigned long long *best_key;
    const int32_t *best_idx;
    const int32_t *cnt;
    const int32_t *qflag;
    int64_t *out_idx;
    double *out_sim;
    hn_search_aux aux;
    const int64_t *seed_idx;
    const double *seed_sim;
    const float *thr;
    const double *slack;
    unsigned long long *n_flagged;
    const DbRef *db;     // multi-database (or NULL): F.q counts padded
    const int32_t *gdb;  //   positions; outputs go to out_base + local
    unsigned long long *ts_end;  // multi-database: per database, the latest
                                 // constant-rate clock of its result writes
};

__global__ __launch_bounds__(256) void finalize_kernel(FinalArgs F) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= F.q) return;
    int64_t o = i;
    if (F.gdb) {
        const DbRef &D = F.db[F.gdb[i]];
        const int64_t local = i - D.pad_base;
        if (local >= D.q) return;
        o = D.out_base + local;
    }
    const bool bad = F.qn[i].bad != 0;
    F.out_idx[o] = bad ? -1 : (int64_t)F.best_idx[i];
    F.out_sim[o] = bad ? (double)NAN : sim_of_key(F.best_key[i]);
    if (F.aux.survivors) F.aux.survivors[o] = F.cnt[i];
    if (F.aux.seed_idx) F.aux.seed_idx[o] = F.seed_idx ? F.seed_idx[i] : -1;
    if (F.aux.seed_sim) F.aux.seed_sim[o] = F.seed_sim ? F.seed_sim[i] : (double)NAN;
    if (F.aux.threshold) F.aux.threshold[o] = F.thr ? F.thr[i] : (float)NAN;
    if (F.aux.slack) F.aux.slack[o] = F.slack ? F.slack[i] : (double)NAN;
    if (F.n_flagged && F.qflag[i]) atomicAdd(F.n_flagged, 1ull);
    if (F.ts_end) {
        // the lanes of a wave write together: only the last lane of each
        // database's run in the wave records the time
        const DbRef &D = F.db[F.gdb[i]];
        if (i - D.pad_base + 1 == D.q || (threadIdx.x & 63) == 63 || i + 1 == F.q)
            atomicMax(&F.ts_end[F.gdb[i]], (unsigned long long)wall_clock64());
    }
}

// ------------------------------------------------------------ exact top-k

// Exclusive prefix sums of per-query counts, off[q] = total (one work-group,
// 1024 queries at a time; the loop bound is uniform).
__global__ __launch_bounds__(1024) void prefix_counts(const int32_t *__restrict__ cnt, int64_t q,
                                                      int64_t *__restrict__ off) {
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int64_t base = 0; base < q; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < q ? cnt[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t add = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < q) off[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[q] = carry;
}

// Bucket the rescored pairs by query: each pair's float64 sim and entry go
// to its query's contiguous bucket (order inside a bucket is arbitrary).
__global__ __launch_bounds__(256) void scatter_pairs(const int2 *__restrict__ pairs,
                                                     const double *__restrict__ psim,
                                                     const unsigned long long *counter, int64_t cap,
                                                     const int64_t *__restrict__ off,
                                                     int32_t *__restrict__ fill,
                                                     double *__restrict__ bsim,
                                                     int32_t *__restrict__ bent) {
    const unsigned long long c = *counter;
    const int64_t m = (int64_t)c < cap ? (int64_t)c : cap;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * 256) {
        const int2 pr = pairs[p];
        const int64_t j = off[pr.x] + atomicAdd(&fill[pr.x], 1);
        bsim[j] = psim[p];
        bent[j] = pr.y;
    }
}

// One wave per query: the topk best of its bucket in (sim desc, entry asc)
// order, by topk sweeps that each take the best pair after the previous one
// (the order is total, so the result does not depend on the bucket order).
// Missing places (fewer entries than topk) get index -1 and sim -inf; a query
// with a non-finite component gets -1 and NaN.
// Pairs per lane that topk_select holds in registers: a bucket of at most
// 64 x kSelRegs pairs is gathered once; a larger one is re-read per sweep in
// chunks of that size.
constexpr int kSelRegs = 16;

__global__ __launch_bounds__(256) void topk_select(const int64_t *__restrict__ off,
                                                   const double *__restrict__ bsim,
                                                   const int32_t *__restrict__ bent, int64_t q,
                                                   int topk, const QNorm *__restrict__ qn,
                                                   int64_t *__restrict__ out_idx,
                                                   double *__restrict__ out_sim) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q) return;
    const bool bad = qn[i].bad != 0;
    const int64_t lo = off[i], hi = off[i + 1];
    double pv = INFINITY;
    int64_t pe = -1;
    bool done = bad;
    // The bucket (contiguous sims and entries) is read in chunks of 64 x
    // kSelRegs pairs, all loads of a chunk in flight together, then scanned
    // in registers.  A bucket of one chunk stays in registers across the
    // sweeps.
    double sv[kSelRegs];
    int ev[kSelRegs];
    auto gather = [&](int64_t base) {
#pragma unroll
        for (int u = 0; u < kSelRegs; ++u) {
            const int64_t j = base + lane + 64 * u;
            sv[u] = j < hi ? bsim[j] : -INFINITY;
            ev[u] = j < hi ? bent[j] : -1;
        }
    };
    // best pair strictly after (pv, pe) in (sim desc, entry asc) order
    auto scan = [&](double &bv, int64_t &be) {
#pragma unroll
        for (int u = 0; u < kSelRegs; ++u) {
            const double sc = sv[u];
            const int64_t e = ev[u];
            const bool after = sc < pv || (sc == pv && e > pe);
            if (sc != -INFINITY && after && (be < 0 || sc > bv || (sc == bv && e < be))) {
                bv = sc;
                be = e;
            }
        }
    };
    const bool resident = hi - lo <= 64 * kSelRegs;
    if (resident && !done) gather(lo);
    for (int r = 0; r < topk; ++r) {
        double bv = -INFINITY;
        int64_t be = -1;
        if (!done) {
            if (resident) {
                scan(bv, be);
            } else {
                for (int64_t base = lo; base < hi; base += 64 * kSelRegs) {
                    gather(base);
                    scan(bv, be);
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int64_t oe = __shfl_xor(be, o);
                if (oe >= 0 && (be < 0 || ov > bv || (ov == bv && oe < be))) {
                    bv = ov;
                    be = oe;
                }
            }
            done = be < 0;
        }
        if (lane == 0) {
            out_idx[i * topk + r] = bad ? -1 : be;
            out_sim[i * topk + r] = bad ? (double)NAN : (be < 0 ? -INFINITY : bv);
        }
        pv = bv;
        pe = be;
    }
}

// ------------------------------------------------- brute-force helpers

// Largest row norm of the database (an upper bound after the caller's
// 2^-40 widening, which covers the float64 summation in any order).  Half a
// wave per row, four elements per lane with 16-byte loads, kBfNormRows rows
// per wave loaded before any arithmetic: a streaming read at copy speed.  The
// grid is capped and strides over the rows, so few work-groups contend for
// the one atomic maximum.
constexpr int kBfNormRows = 16;
constexpr unsigned kBfNormGrid = 4096;

__global__ __launch_bounds__(256) void bf_db_norm(const float4 *__restrict__ db, int64_t n,
                                                  unsigned long long *mu_key) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
    double m = 0.0;
    for (int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kBfNormRows; r0 < n;
         r0 += (int64_t)gridDim.x * 4 * kBfNormRows) {
        float4 v[kBfNormRows / 2];
#pragma unroll
        for (int t = 0; t < kBfNormRows / 2; ++t) {
            const int64_t r = r0 + 2 * t + h;
            v[t] = r < n ? db[r * 32 + l] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int t = 0; t < kBfNormRows / 2; ++t) {
            double ss = (double)v[t].x * v[t].x;
            ss = fma((double)v[t].y, (double)v[t].y, ss);
            ss = fma((double)v[t].z, (double)v[t].z, ss);
            ss = fma((double)v[t].w, (double)v[t].w, ss);
            for (int o = 16; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
            m = fmax(m, ss);
        }
    }
    m = fmax(m, __shfl_xor(m, 32));
    if (lane == 0) sh[threadIdx.x >> 6] = sqrt(m);
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(mu_key, key_of(fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]))));
}

__global__ void zero_u64(unsigned long long *p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0ull;
}

// Window width for the exhaustive float32 scan: the true argmax has s~ no
// lower than the scan maximum minus 2 (eps_f32 + eps_f64).
struct BfPrepArgs {
    const QNorm *qn;
    const unsigned long long *mu_key;
    int64_t q, q_pad;
    float *win_scan;  // widened for the float32 subtraction in the scan
    double *win;      // exact window for the re-filter
    unsigned long long *best_key;
    int32_t *best_idx, *cnt, *qflag;
    unsigned long long *counter;
};

__global__ __launch_bounds__(256) void bf_prep(BfPrepArgs P) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) *P.counter = 0;
    if (i >= P.q_pad) return;
    if (i >= P.q) {
        P.win_scan[i] = 0.0f;
        return;
    }
    const double mu = sim_of_key(*P.mu_key) * (1.0 + ldexp(1.0, -40));
    const QNorm qn = P.qn[i];
    const double scale = qn.full * mu;
    double w = 2.0 * (gamma_n(kDim, kU32) * scale + kDim * ldexp(1.0, -125) +
                      gamma_n(kDim, kU64) * scale);
    w = w * (1.0 + ldexp(1.0, -20)) + ldexp(1.0, -100);
    P.win[i] = w;
    P.win_scan[i] = __double2float_ru(w + ldexp(1.0, -22) * scale);
    P.best_key[i] = 0ull;
    P.best_idx[i] = kIdxNone;
    P.cnt[i] = 0;
    P.qflag[i] = 0;
}

// Largest chunk partial of query i: one wave per query, lanes striding over
// the chunks (many independent loads in flight), then a wave maximum.
__device__ __forceinline__ float chunk_max(const float *part_val, int32_t n_chunks, int32_t q_pad,
                                           int64_t i, int lane) {
    float m = -INFINITY;
#pragma unroll 8
    for (int c = lane; c < n_chunks; c += 64) m = fmaxf(m, part_val[(int64_t)c * q_pad + i]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}

// Exhaustive-scan threshold: the scan maximum minus the window, per query
// (launch: blocks_for(q, 4) groups of 4 waves).
__global__ __launch_bounds__(256) void bf_threshold(const float *part_val, int32_t n_chunks,
                                                    int32_t q_pad, int64_t q, const double *win,
                                                    float *thr) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q) return;
    const float m = chunk_max(part_val, n_chunks, q_pad, i, threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0) thr[i] = __double2float_rd((double)m - win[i]);
}

// Largest prefix-pass score per (padded) query position: the exhaustive
// scan's starting running maximum.  Same launch shape as bf_threshold.
__global__ __launch_bounds__(256) void prefix_max(const float *part_val, int32_t n_chunks,
                                                  int32_t ld, int64_t q_pad, float *out) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q_pad) return;
    const float m = chunk_max(part_val, n_chunks, ld, i, threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0) out[i] = m;
}

// Single-pass re-filter threshold: max(T_q, m - w_q) with m the final scan
// maximum over all chunks (which includes the starting value T_q + w_q).
// Same launch shape as bf_threshold.
// Also records m (win_max) and clears the entry of the pair that scored it
// (win_arg, INT_MAX: none found yet).
__global__ __launch_bounds__(256) void win_threshold(const float *part_val, int32_t n_chunks,
                                                     int32_t q_pad, int64_t q, const double *win,
                                                     const float *thr, float *out,
                                                     float *win_max, int32_t *win_arg) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q) return;
    const float m = chunk_max(part_val, n_chunks, q_pad, i, threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0) {
        out[i] = fmaxf(thr[i], __double2float_rd((double)m - win[i]));
        win_max[i] = m;
        win_arg[i] = INT_MAX;
    }
}

// The entry of the final scan maximum: the pair whose score equals m (the
// entry that raised the running maximum to m was inside its own window, so
// it was stored).  Several such pairs: the smallest entry.
__global__ __launch_bounds__(256) void win_argmax(const int2 *__restrict__ pairs,
                                                  const float *__restrict__ pair_val,
                                                  const unsigned long long *counter, int64_t cap,
                                                  const float *__restrict__ win_max,
                                                  int32_t *win_arg) {
    const unsigned long long c = *counter;
    const int64_t m = (int64_t)c < cap ? (int64_t)c : cap;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * 256) {
        const float v = pair_val[p];
        const int2 pr = pairs[p];
        if (v == win_max[pr.x]) atomicMin(&win_arg[pr.x], pr.y);
    }
}

// Algorithm 1's seed taken from the single pass itself: the entry of the
// final scan maximum is the best major-dot entry, so its canonical sim L' is
// an admissible lower bound, and the re-filter threshold rises to
// round_down((L' - beta - eps_q) * u), the plain seed's threshold at L' in
// scan units (u = 1 / (s_q s_x) for the scaled fp8 and int8 scans, else 1),
// but never above m, so that entry's own pair is always rescored.  One
// thread per query; queries without a stored maximum keep the window
// threshold.
__global__ __launch_bounds__(256) void win_refine(SeedArgs S, const float *__restrict__ win_max,
                                                  const int32_t *__restrict__ win_arg,
                                                  float *thr_ref) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= S.q) return;
    const int32_t j = win_arg[i];
    const QNorm qn = S.qn[i];
    if (j == INT_MAX || qn.bad) return;
    const double L = sim64(S.queries + i * kDim, S.rows + (int64_t)j * kDim);
    const double unit =
        S.scaled ? 1.0 / ((double)(S.scaled == 1 ? qn.sc8 : qn.sci) * S.scale_x) : 1.0;
    const float t = round_down_f32((L - S.beta - S.slack[i]) * unit);
    thr_ref[i] = fmaxf(thr_ref[i], fminf(t, win_max[i]));
}

__global__ void fill_lower(double *lower, int64_t *idx, int64_t q) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < q; i += (int64_t)gridDim.x * 256) {
        lower[i] = -INFINITY;
        idx[i] = -1;
    }
}

// ---------------------------------------------------------- launch helpers

unsigned blocks_for(int64_t items, int per = 256) {
    return (unsigned)std::max<int64_t>(1, (items + per - 1) / per);
}

// precision 0: float32 stream of width w; 1: bf16 stream of width w.
const char *scan_tag(int mode, int precision) {
    static const char *const tags[4][4] = {
        {"scan_argmax_f32", "scan_argmax_bf16", "scan_argmax_fp8", "scan_argmax_int8"},
        {"scan_filter_f32", "scan_filter_bf16", "scan_filter_fp8", "scan_filter_int8"},
        {"scan_window_f32", "scan_window_bf16", "scan_window_fp8", "scan_window_int8"},
        {"scan_store_f32", "scan_store_bf16", "scan_store_fp8", "scan_store_int8"}};
    return tags[mode][precision == HN_PREC_FP32   ? 0
                      : precision == HN_PREC_BF16 ? 1
                      : precision == HN_PREC_FP8  ? 2
                                                  : 3];
}

// Resident work-groups of the scan kernel launch_scan<mode> would start (0 if
// not compiled): the slot count that make_plan balances the items over.
inline int64_t scan_slots(int precision, int mode, int w, int cfg) {
    if (precision == HN_PREC_FP32)
        return w <= 32 ? slots_scan_f32_narrow(mode, w, cfg) : slots_scan_f32_wide(mode, w, cfg);
    if (precision == HN_PREC_BF16) return slots_scan_bf16(mode, w, cfg);
    if (precision == HN_PREC_FP8) return slots_scan_fp8(mode, w, cfg);
    if (precision == HN_PREC_INT8) return slots_scan_int8(mode, w, cfg);
    return 0;
}

template <int MODE>
int launch_scan(int precision, int w, int cfg, const Plan &p, const ScanArgs &A,
                hipStream_t s) {
    ProfScope prof(s, scan_tag(MODE, precision));
    int rc;
    if (precision == HN_PREC_FP32)
        rc = w <= 32 ? launch_scan_f32_narrow(MODE, w, cfg, p, A, s)
                     : launch_scan_f32_wide(MODE, w, cfg, p, A, s);
    else if (precision == HN_PREC_BF16)
        rc = launch_scan_bf16(MODE, w, cfg, p, A, s);
    else if (precision == HN_PREC_FP8)
        rc = launch_scan_fp8(MODE, w, cfg, p, A, s);
    else if (precision == HN_PREC_INT8)
        rc = launch_scan_int8(MODE, w, cfg, p, A, s);
    else
        return fail(HN_ERR_UNSUPPORTED, "precision %d is not available", precision);
    if (rc) return fail(HN_ERR_INVALID_ARG, "no scan kernel for mode %d width %d config %d", MODE, w, cfg);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

}  // namespace
}  // namespace hn
