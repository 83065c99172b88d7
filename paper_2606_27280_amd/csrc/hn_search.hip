// Exact top-1 search pipeline (Algorithm 1 on the GPU) and the exhaustive
// baseline.  Kernels other than the scan itself live here: query preparation,
// seed selection with the bound slack, float64 rescoring, the deterministic
// argmax, the exact overflow fallback and the output writer.
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
    float sc8;                  // s8: power-of-two scale of the fp8 operand
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
    QNorm *qn;
    unsigned *work;
};

// One thread per (padded) query: norms and the float32 / bf16 / fp8 operands.
__global__ __launch_bounds__(256) void prep_queries(PrepArgs P) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (P.work && i < kWorkWords) P.work[i] = 0u;
    if (i >= P.q_pad) return;
    if (i >= P.nq) {
        if (P.op32)
            for (int c = 0; c < P.w32; ++c) P.op32[i * P.w32 + c] = 0.0f;
        if (P.op16)
            for (int c = 0; c < P.w16; ++c) P.op16[i * P.w16 + c] = 0;
        if (P.op8)
            for (int c = 0; c < P.w8; ++c) P.op8[i * P.w8 + c] = 0;
        return;
    }
    const int k = P.k;
    const float *v = P.q + i * kDim;
    double sM = 0, sm = 0, sr = 0;
    float amax = 0.0f;
    bool finite = true;
    for (int j = 0; j < kDim; ++j) {
        float f = v[j];
        finite = finite && isfinite(f);
        double d = (double)f;
        if (j < k) {
            sM = fma(d, d, sM);
            double b = (double)bf16_rne(f);
            sr = fma(b - d, b - d, sr);
            amax = fmaxf(amax, fabsf(f));
        } else {
            sm = fma(d, d, sm);
        }
    }
    const double up = 1.0 + ldexp(1.0, -40);
    QNorm r;
    r.major = sqrt(sM) * up;
    r.minor = sqrt(sm) * up;
    r.full = sqrt(sM + sm) * up;
    r.res16 = sqrt(sr) * up;
    r.res8 = 0.0;
    r.sc8 = 1.0f;
    r.bad = finite ? 0 : 1;
    if (P.op32)
        for (int c = 0; c < P.w32; ++c) P.op32[i * P.w32 + c] = (c < k && finite) ? v[c] : 0.0f;
    if (P.op16)
        for (int c = 0; c < P.w16; ++c)
            P.op16[i * P.w16 + c] =
                (c < k && finite) ? (uint16_t)(__float_as_uint(bf16_rne(v[c])) >> 16) : 0;
    if (P.op8) {
        const float sc = finite ? fp8_scale_for(amax) : 1.0f;
        const float inv = 1.0f / sc;  // exact: a power of two
        double s8 = 0;
        for (int c = 0; c < P.w8; ++c) {
            const float f = (c < k && finite) ? v[c] : 0.0f;
            const uint8_t code = fp8_e4m3(f * inv);
            P.op8[i * P.w8 + c] = code;
            const double e = (double)fp8_e4m3_value(code) * (double)sc - (double)f;
            s8 = fma(e, e, s8);
        }
        r.res8 = sqrt(s8) * up;
        r.sc8 = sc;
    }
    P.qn[i] = r;
}

// ---------------------------------------------------------------- seed

struct SeedArgs {
    const float *part_val;
    const int32_t *part_idx;
    int32_t n_chunks, q_pad;
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
    int fp8;       // residuals of the fp8 operands; thresholds in scan units
    double res_mu, res_x, res_acc_rel;
    double scale_x;  // fp8: power-of-two scale of the entry copy
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

// Entry of slot v of an argmax lane group gid = block * G + g, for the scan's
// tile shape: 16x16 tiles give 4 consecutive entries, 32x32 tiles 16 entries
// (rows 8 (v / 4) + 4 g + v % 4 of the block).
__device__ __forceinline__ int64_t group_entry(int shape, int gid, int v) {
    if (shape == 16) return (int64_t)(gid >> 2) * 16 + 4 * (gid & 3) + v;
    return (int64_t)(gid >> 1) * 32 + 8 * (v >> 2) + 4 * (gid & 1) + (v & 3);
}

// One wave per query: reduce the per-chunk argmax partials, rescore every
// entry of the winning lane group in float64 (one lane each) and keep the
// best (sim desc, index asc) as the seed; then the slack and thresholds.
__global__ __launch_bounds__(256) void seed_kernel(SeedArgs S) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i == 0 && lane == 0) *S.counter = 0;
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
    } else {
        float bv = -INFINITY;
        int bi = -1;
        for (int c = lane; c < S.n_chunks; c += 64)
            lex_merge(bv, bi, S.part_val[(int64_t)c * S.q_pad + i],
                      S.part_idx[(int64_t)c * S.q_pad + i]);
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            lex_merge(bv, bi, ov, oi);
        }
        double sv = -INFINITY;
        int64_t e = -1;
        if (bi >= 0 && lane < S.group_size) {
            e = group_entry(S.shape, bi, lane);
            if (e < S.n)
                sv = sim64(qv, S.rows + e * kDim);
            else
                e = -1;
        }
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
        const double rq = S.fp8 ? qn.res8 : qn.res16;
        const double er =
            rq * S.res_mu + qn.major * S.res_x + S.res_acc_rel * (qn.major + rq) * S.res_mu;
        es = S.scan_res == 2 ? er : fmin(es, er);
    }
    es += S.scan_abs;
    double en = fmax(0.0, qn.minor * S.mu_minor - S.alpha);
    double e64 = gamma_n(kDim, kU64) * qn.full * S.mu_full;
    double eps = (es + en + e64) * (1.0 + ldexp(1.0, -30)) + ldexp(1.0, -40);
    // fp8 scans score q~ . x~ with q = s_q q~ and x = s_x x~ (powers of two):
    // the threshold in scan units is the same bound divided by s_q s_x, exact
    const double unit = S.fp8 ? 1.0 / ((double)qn.sc8 * S.scale_x) : 1.0;
    S.thr[i] = round_down_f32((L - S.beta - eps) * unit);
    if (S.win_scan) {
        // |s~| <= (||q_M|| + r_q) max ||x^_M|| (1 + 2^-20), in scan units
        const double rq = S.fp8 ? qn.res8 : (S.scan_res ? qn.res16 : 0.0);
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

// ------------------------------------------------------ rescoring & argmax

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
};

__device__ __forceinline__ int64_t pair_count(const RescoreArgs &R) {
    unsigned long long c = *R.counter;
    return (int64_t)c < R.cap ? (int64_t)c : R.cap;
}

// MODE 0: plain; 1: float32 re-check against thr32 first; 2: window re-filter.
template <int MODE>
__global__ __launch_bounds__(256) void rescore_kernel(RescoreArgs R) {
    const int64_t m = pair_count(R);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * 256) {
        const int2 pr = R.pairs[p];
        const float *qv = R.queries + (int64_t)pr.x * kDim;
        if (R.count) atomicAdd(&R.cnt[pr.x], 1);
        bool keep = true;
        if (MODE == 1) {
            const float *xm = R.major32 + (int64_t)pr.y * R.kp;
            float s = 0.0f;
            for (int j = 0; j < R.k; ++j) s = fmaf(qv[j], xm[j], s);
            keep = s >= R.thr32[pr.x];
        } else if (MODE == 2) {
            keep = R.pair_val[p] >= R.thr32[pr.x];
        }
        double s = -INFINITY;
        if (keep) {
            s = sim64(qv, R.rows + (int64_t)pr.y * kDim);
            atomicMax(&R.best_key[pr.x], key_of(s));
        }
        R.psim[p] = s;
    }
}

__global__ __launch_bounds__(256) void tie_kernel(RescoreArgs R) {
    const int64_t m = pair_count(R);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m + R.q;
         p += (int64_t)gridDim.x * 256) {
        if (p < m) {
            const double s = R.psim[p];
            if (s == -INFINITY) continue;
            const int2 pr = R.pairs[p];
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
        double lim = -INFINITY;
        if (!F.full) {
            double en = fmax(0.0, qn.minor * F.mu_minor - F.alpha);
            double e = gamma_n(F.k, kU64) * qn.major * F.mu_major + en +
                       gamma_n(kDim, kU64) * qn.full * F.mu_full;
            lim = F.seed_sim[qi] - F.beta - e * (1.0 + ldexp(1.0, -30)) - ldexp(1.0, -40);
        }
        unsigned long long bk = 0;
        int bi = kIdxNone, c = 0;
        for (int64_t e = threadIdx.x; e < F.n; e += 256) {
            const float *xv = F.rows + e * kDim;
            if (!F.full) {
                double s = 0.0;
                for (int j = 0; j < F.k; ++j) s = fma((double)qv[j], (double)xv[j], s);
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
};

__global__ __launch_bounds__(256) void finalize_kernel(FinalArgs F) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= F.q) return;
    const bool bad = F.qn[i].bad != 0;
    F.out_idx[i] = bad ? -1 : (int64_t)F.best_idx[i];
    F.out_sim[i] = bad ? (double)NAN : sim_of_key(F.best_key[i]);
    if (F.aux.survivors) F.aux.survivors[i] = F.cnt[i];
    if (F.aux.seed_idx) F.aux.seed_idx[i] = F.seed_idx ? F.seed_idx[i] : -1;
    if (F.aux.seed_sim) F.aux.seed_sim[i] = F.seed_sim ? F.seed_sim[i] : (double)NAN;
    if (F.aux.threshold) F.aux.threshold[i] = F.thr ? F.thr[i] : (float)NAN;
    if (F.aux.slack) F.aux.slack[i] = F.slack ? F.slack[i] : (double)NAN;
    if (F.n_flagged && F.qflag[i]) atomicAdd(F.n_flagged, 1ull);
}

// ------------------------------------------------- brute-force helpers

__global__ __launch_bounds__(256) void bf_db_norm(const float *__restrict__ db, int64_t n,
                                                  unsigned long long *mu_key) {
    __shared__ double sh[4];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const float *x = db + i * kDim;
        double s = 0.0;
        for (int j = 0; j < kDim; ++j) s = fma((double)x[j], (double)x[j], s);
        v = sqrt(s);
    }
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
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

__global__ __launch_bounds__(256) void bf_threshold(const float *part_val, int32_t n_chunks,
                                                    int32_t q_pad, int64_t q, const double *win,
                                                    float *thr) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= q) return;
    float m = -INFINITY;
    for (int c = 0; c < n_chunks; ++c) m = fmaxf(m, part_val[(int64_t)c * q_pad + i]);
    thr[i] = __double2float_rd((double)m - win[i]);
}

// Single-pass re-filter threshold: max(T_q, m - w_q) with m the final scan
// maximum over all chunks (which includes the starting value T_q + w_q).
__global__ __launch_bounds__(256) void win_threshold(const float *part_val, int32_t n_chunks,
                                                     int32_t q_pad, int64_t q, const double *win,
                                                     const float *thr, float *out) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= q) return;
    float m = -INFINITY;
    for (int c = 0; c < n_chunks; ++c) m = fmaxf(m, part_val[(int64_t)c * q_pad + i]);
    out[i] = fmaxf(thr[i], __double2float_rd((double)m - win[i]));
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
    static const char *const tags[4][3] = {
        {"scan_argmax_f32", "scan_argmax_bf16", "scan_argmax_fp8"},
        {"scan_filter_f32", "scan_filter_bf16", "scan_filter_fp8"},
        {"scan_window_f32", "scan_window_bf16", "scan_window_fp8"},
        {"scan_store_f32", "scan_store_bf16", "scan_store_fp8"}};
    return tags[mode][precision == HN_PREC_FP32 ? 0 : (precision == HN_PREC_BF16 ? 1 : 2)];
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
    else
        return fail(HN_ERR_UNSUPPORTED, "precision %d is not available", precision);
    if (rc) return fail(HN_ERR_INVALID_ARG, "no scan kernel for mode %d width %d config %d", MODE, w, cfg);
    HN_HIP(hipGetLastError());
    return HN_OK;
}


// Everything one search call needs on the device.
struct Work {
    Plan plan;
    int cfg = 0;
    int precision = HN_PREC_FP32;
    int width = 0;
    int shape = 16;  // tile shape of the scan (16 or 32): decodes argmax groups
    const void *stream_x = nullptr;
    float *op32 = nullptr;
    uint16_t *op16 = nullptr;
    uint8_t *op8 = nullptr;
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
    double *lower = nullptr;
    int64_t *lower_idx = nullptr;
};

// The scan stream and query operands of a precision.
int stream_width(const hn_index *ix, int precision) {
    return precision == HN_PREC_FP32 ? ix->kp : (precision == HN_PREC_BF16 ? ix->kb : ix->k8);
}
const void *stream_of(const hn_index *ix, int precision) {
    return precision == HN_PREC_FP32   ? (const void *)ix->major32
           : precision == HN_PREC_BF16 ? (const void *)ix->major16
                                       : (const void *)ix->major8;
}
const void *operands_of(const Work &W) {
    return W.precision == HN_PREC_FP32   ? (const void *)W.op32
           : W.precision == HN_PREC_BF16 ? (const void *)W.op16
                                         : (const void *)W.op8;
}

int check_precision(const hn_index *ix, int precision) {
    if (precision != HN_PREC_FP32 && precision != HN_PREC_BF16 && precision != HN_PREC_FP8)
        return fail(HN_ERR_UNSUPPORTED, "precision %d is not available", precision);
    if (precision == HN_PREC_FP8 && ix->k8 == 0)
        return fail(HN_ERR_UNSUPPORTED, "the fp8 scan needs k <= 32 (k = %d)", ix->k);
    return HN_OK;
}

void launch_prep(const hn_index *ix, const float *queries, int64_t q, const Plan &p, Work &W,
                 hipStream_t s) {
    PrepArgs P;
    P.q = queries;
    P.nq = q;
    P.q_pad = p.q_pad;
    P.k = ix->k;
    P.w32 = ix->kp;
    P.w16 = ix->kb;
    P.w8 = ix->k8;
    P.op32 = W.op32;
    P.op16 = W.op16;
    P.op8 = W.op8;
    P.qn = W.qn;
    P.work = W.work;
    ProfScope prof_(s, "prep_queries");
    hipLaunchKernelGGL(prep_queries, dim3(blocks_for(p.q_pad)), dim3(256), 0, s, P);
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
    return HN_OK;
}

// Prepare queries, run the plain-seed pass and compute thresholds.  With
// `lower` the seed pass is skipped and L (and its entry, lower_idx, if not
// NULL) is taken from the caller.  `window`: also the single-pass window
// (W.win, W.win_scan, W.init_best) and the pair values.
int stage_seed(const hn_index *ix, const float *queries, int64_t q, const hn_search_opts &o,
               const double *lower, const int64_t *lower_idx, int64_t cap, Work &W,
               hipStream_t s, bool window = false) {
    W.precision = o.precision;
    W.width = stream_width(ix, W.precision);
    W.stream_x = stream_of(ix, W.precision);
    const TileInfo ti = tile_info(W.precision, W.width);
    W.cfg = pick_cfg(q, ti.cols, ti.cost, o.query_tiles);
    if (W.cfg < 0)
        return fail(HN_ERR_INVALID_ARG, "query_tiles=%d is not available for this width",
                    o.query_tiles);
    W.plan = make_plan(ix->n, q, W.cfg, o.chunk_blocks, ti.rows, ti.cols);
    W.shape = ti.rows;
    const Plan &p = W.plan;
    W.cap = cap;

    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) { bytes += (count * sz + 255) & ~size_t(255); };
    add(p.q_pad * ix->kp, 4);
    add(p.q_pad * ix->kb, 2);
    add(p.q_pad * ix->k8, 1);
    add(p.q_pad, sizeof(QNorm));
    add((size_t)p.n_chunks * p.q_pad, 4);
    add((size_t)p.n_chunks * p.q_pad, 4);
    add(p.q_pad, 4);
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
    add(cap, sizeof(int2));
    add(cap, 8);
    if (window) {
        add(p.q_pad, 8);
        add(p.q_pad, 4);
        add(p.q_pad, 4);
        add(q, 4);
        add(cap, 4);
        add(q, 8);
        add(q, 8);
    }
    Arena *ar = nullptr;
    int rc = arena_for((void *)s, bytes, &ar);
    if (rc) return rc;
    W.op32 = ar->take<float>(p.q_pad * ix->kp);
    W.op16 = ar->take<uint16_t>(p.q_pad * ix->kb);
    W.op8 = ix->k8 ? ar->take<uint8_t>(p.q_pad * ix->k8) : nullptr;
    W.qn = ar->take<QNorm>(p.q_pad);
    W.part_val = ar->take<float>((size_t)p.n_chunks * p.q_pad);
    W.part_idx = ar->take<int32_t>((size_t)p.n_chunks * p.q_pad);
    W.thr = ar->take<float>(p.q_pad);
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
    W.redo = ar->take<int>(p.n_items);
    W.pairs = ar->take<int2>(cap);
    W.psim = ar->take<double>(cap);
    if (window) {
        W.win = ar->take<double>(p.q_pad);
        W.win_scan = ar->take<float>(p.q_pad);
        W.init_best = ar->take<float>(p.q_pad);
        W.thr_ref = ar->take<float>(q);
        W.pair_val = ar->take<float>(cap);
        W.lower = ar->take<double>(q);
        W.lower_idx = ar->take<int64_t>(q);
    }

    launch_prep(ix, queries, q, p, W, s);
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
    A.part_val = W.part_val;
    A.part_idx = W.part_idx;
    A.redo = W.redo;
    A.redo_count = W.work + 2 * kXcds;
    if (!lower) {
        rc = launch_scan<kArgmax>(W.precision, W.width, W.cfg, p, A, s);
        if (rc) return rc;
    }

    SeedArgs S;
    memset(&S, 0, sizeof S);
    S.part_val = W.part_val;
    S.part_idx = W.part_idx;
    S.n_chunks = p.n_chunks;
    S.q_pad = (int32_t)p.q_pad;
    S.shape = W.shape;
    S.group_size = W.shape == 16 ? 4 : 16;
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
    if (W.precision == HN_PREC_FP32) {
        S.scan_rel = gamma_n(ix->k, kU32);
        S.scan_mu = ix->mu_major;
        S.scan_abs = ix->k * ldexp(1.0, -125);
        S.scan_res = 0;
    } else if (W.precision == HN_PREC_BF16) {
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
    } else {
        // fp8: the residual form only (subnormal codes have no relative
        // bound); the products are summed by the bf16 matrix core (the codes
        // are decoded exactly to bf16), float32 accumulation.
        S.scan_rel = 0.0;
        S.scan_mu = 0.0;
        S.scan_abs = ix->k * ldexp(1.0, -125);
        S.scan_res = 2;
        S.fp8 = 1;
        S.scale_x = ix->scale8;
        S.res_mu = ix->mu_major8;
        S.res_x = ix->res8;
        S.res_acc_rel = gamma_n(ix->k, kU32);
    }
    S.lower = lower;
    S.lower_idx = lower_idx;
    if (window) {
        S.win = W.win;
        S.win_scan = W.win_scan;
        S.init_best = W.init_best;
        S.bound_mu = W.precision == HN_PREC_FP32   ? ix->mu_major
                     : W.precision == HN_PREC_BF16 ? ix->mu_major16
                                                   : ix->mu_major8;
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
        hipLaunchKernelGGL(seed_kernel, dim3(blocks_for(p.q_pad, 4)), dim3(256), 0, s, S);
    }
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
    return A;
}

__global__ __launch_bounds__(256) void scale_scores(float *scores, int64_t q, int64_t n,
                                                   const QNorm *qn, float scale_x) {
    const int64_t total = q * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256)
        scores[t] *= qn[t / n].sc8 * scale_x;
}

int64_t default_cap(int64_t n, int64_t q) {
    int64_t per = std::max<int64_t>(2048, n / 512);
    int64_t c = q * per;
    return std::min<int64_t>(std::max<int64_t>(c, (int64_t)1 << 20), (int64_t)1 << 28);
}

}  // namespace
}  // namespace hn

using namespace hn;

namespace hn {
namespace {

// Survivor-list budget per query of the single-pass forms (the window keeps
// more pairs than the two-pass threshold) and the query batch that fits it.
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
                 const int64_t *lower_idx_in = nullptr, Overflow *ov = nullptr) {
    const bool single = o.seed != HN_SEED_PLAIN && !lower_in;
    const int64_t cap =
        o.survivor_cap > 0
            ? o.survivor_cap
            : (single ? std::min<int64_t>(std::max<int64_t>(q * window_per_query(ix->n), 1 << 20),
                                          (int64_t)1 << 29)
                      : default_cap(ix->n, q));
    Work W;
    int rc = stage_seed(ix, queries, q, o, lower_in, lower_idx_in, cap, W, s, single);
    if (rc) return rc;
    ScanArgs A = filter_args(ix, W, q, W.pairs, cap);
    if (single) {
        A.thr = W.win_scan;
        A.init_best = W.init_best;
        A.pair_val = W.pair_val;
        A.part_val = W.part_val;
        rc = launch_scan<kWindow>(W.precision, W.width, W.cfg, W.plan, A, s);
        if (rc) return rc;
        ProfScope prof_(s, "win_threshold");
        hipLaunchKernelGGL(win_threshold, dim3(blocks_for(q)), dim3(256), 0, s, W.part_val,
                           W.plan.n_chunks, (int32_t)W.plan.q_pad, q, W.win, W.thr, W.thr_ref);
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
    } else if (W.precision == HN_PREC_FP32) {
        ProfScope prof_(s, "rescore");
        hipLaunchKernelGGL(rescore_kernel<0>, dim3(rgrid), dim3(256), 0, s, R);
    } else {
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
        unsigned long long h = 0;
        HN_HIP(hipMemcpyAsync(&h, ov->count, sizeof h, hipMemcpyDeviceToHost, s));
        HN_HIP(hipStreamSynchronize(s));
        ov->n = (int64_t)h;
    }
    return HN_OK;
}

// A single-pass batch, then its overflowing queries again as a plain filter
// pass seeded with the best candidate each reached (exact: every entry that
// can beat that candidate survives the filter; the candidate is the seed).
int single_pass_batch(const hn_index *ix, const float *queries, int64_t q, int64_t *out_idx,
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
    o2.survivor_cap = 0;
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
        if (o.seed == HN_SEED_PLAIN)
            rc = search_batch(ix, queries + q0 * kDim, nb, out_idx + q0, out_sim + q0, o,
                              aux ? &a2 : nullptr, stats ? &st : nullptr, s);
        else
            rc = single_pass_batch(ix, queries + q0 * kDim, nb, out_idx + q0, out_sim + q0, o,
                                   aux ? &a2 : nullptr, stats ? &st : nullptr, s);
        if (rc) return rc;
        if (stats) {
            stats->survivors += st.survivors;
            stats->overflow_queries += st.overflow_queries;
        }
    }
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
    W.op8 = ix->k8 ? ar->take<uint8_t>(p.q_pad * ix->k8) : nullptr;
    W.qn = ar->take<QNorm>(p.q_pad);
    W.work = ar->take<unsigned>(kWorkWords);
    W.redo = ar->take<int>(p.n_items);
    launch_prep(ix, queries, q, p, W, s);
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
    if (rc || precision != HN_PREC_FP8) return rc;
    // fp8 scores come out in units of s_q s_x: rescale (exact, powers of two)
    hipLaunchKernelGGL(scale_scores, dim3(2048), dim3(256), 0, s, scores, q, ix->n, W.qn,
                       ix->scale8);
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
    if (q == 0) return HN_OK;
    hipStream_t s = (hipStream_t)stream;
    const TileInfo ti = tile_info(HN_PREC_FP32, kDim);
    const int cfg = pick_cfg(q, ti.cols, ti.cost, 2);
    Plan p = make_plan(n, q, cfg, 0, ti.rows, ti.cols);
    // A prefix pass (one chunk of the first n_pre rows) gives each query a
    // starting running maximum: a real scan score, so never above the final
    // maximum, and far fewer near-record candidates in the main pass.
    const int64_t n_pre = std::min<int64_t>(n, 4096);
    Plan pp = make_plan(n_pre, q, cfg, (int32_t)((n_pre + ti.rows - 1) / ti.rows), ti.rows,
                        ti.cols);
    const int64_t cap = std::min<int64_t>(
        std::max<int64_t>(q * std::max<int64_t>(256, 16 * (int64_t)p.n_chunks), 1 << 16),
        (int64_t)1 << 26);

    size_t bytes = 0;
    auto add = [&](size_t count, size_t sz) { bytes += (count * sz + 255) & ~size_t(255); };
    add(p.q_pad, sizeof(QNorm));
    add((size_t)p.n_chunks * p.q_pad, 4);
    add(p.q_pad, 4);
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
    float *pre_val = ar->take<float>(p.q_pad);
    int32_t *pre_idx = ar->take<int32_t>(p.q_pad);
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
        hipLaunchKernelGGL(bf_db_norm, dim3(blocks_for(n)), dim3(256), 0, s, db, n, mu_key);
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
        hipLaunchKernelGGL(prep_queries, dim3(blocks_for(p.q_pad)), dim3(256), 0, s, P);
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
    A.init_best = pre_val;
    A.pairs = pairs;
    A.pair_val = pair_val;
    A.counter = counter;
    A.cap = cap;
    A.redo = redo;
    A.redo_count = work + 2 * kXcds + 1;
    rc = launch_scan<kWindow>(HN_PREC_FP32, kDim, cfg, p, A, s);
    if (rc) return rc;
    {
        ProfScope prof_(s, "bf_threshold");
        hipLaunchKernelGGL(bf_threshold, dim3(blocks_for(q)), dim3(256), 0, s, part_val, p.n_chunks,
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
