// Index build: block-norm validation (Eq. 1), rigorous norm maxima for the
// bound slack (Eq. 3), and the device copies the search streams.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <unordered_map>

#include "hn_internal.h"

namespace hn {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
void clear_error() { g_err[0] = 0; }

// ------------------------------------------------------- device memory

namespace {
std::mutex g_mem_mu;
std::unordered_map<void *, size_t> g_mem_size;
int64_t g_mem_held = 0;
int64_t g_mem_budget = 0;  // 0: no budget
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes) {
    *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        if (g_mem_budget > 0 && g_mem_held + (int64_t)bytes > g_mem_budget)
            return hipErrorOutOfMemory;
        g_mem_held += (int64_t)bytes;  // reserved before the call
    }
    const hipError_t e = hipMalloc(p, bytes);
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (e != hipSuccess) {
        g_mem_held -= (int64_t)bytes;
        *p = nullptr;
        return e;
    }
    g_mem_size[*p] = bytes;
    return hipSuccess;
}

void dev_free(void *p) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_mem_size.find(p);
        if (it != g_mem_size.end()) {
            g_mem_held -= (int64_t)it->second;
            g_mem_size.erase(it);
        }
    }
    (void)hipFree(p);
}

// ---------------------------------------------------------------- arenas

namespace {
struct ArenaKey {
    int device;
    void *stream;
    int slot;
    bool operator==(const ArenaKey &o) const {
        return device == o.device && stream == o.stream && slot == o.slot;
    }
};
struct ArenaKeyHash {
    size_t operator()(const ArenaKey &k) const {
        return (std::hash<void *>()(k.stream) * 31u + (size_t)k.device) * 7u + (size_t)k.slot;
    }
};
std::mutex g_arena_mu;
std::unordered_map<ArenaKey, Arena *, ArenaKeyHash> g_arenas;
}  // namespace

int arena_for(void *stream, size_t bytes, Arena **out, int slot) {
    int dev = 0;
    HN_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_arena_mu);
    Arena *&a = g_arenas[ArenaKey{dev, stream, slot}];
    if (!a) a = new (std::nothrow) Arena();
    if (!a) return fail(HN_ERR_OOM, "host allocation failed");
    if (a->cap < bytes) {
        if (a->base) {
            // the old buffer may still be in use by work queued on the stream
            HN_HIP(hipStreamSynchronize((hipStream_t)stream));
            dev_free(a->base);
            a->base = nullptr;
            a->cap = 0;
        }
        size_t want = bytes + bytes / 4 + (1u << 20);
        if (dev_alloc(&a->base, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HN_ERR_OOM, "scratch allocation of %zu bytes failed", want);
        }
        a->cap = want;
    }
    a->used = 0;
    *out = a;
    return HN_OK;
}

int release_arenas(void *stream) {
    int dev = 0;
    HN_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_arena_mu);
    bool synced = false;
    for (auto it = g_arenas.begin(); it != g_arenas.end();) {
        if (it->first.device == dev && it->first.stream == stream) {
            if (!synced) {
                HN_HIP(hipStreamSynchronize((hipStream_t)stream));
                synced = true;
            }
            dev_free(it->second->base);
            delete it->second;
            it = g_arenas.erase(it);
        } else {
            ++it;
        }
    }
    return HN_OK;
}

// --------------------------------------------------------------- kernels

namespace {

struct BuildStats {
    unsigned long long key_major, key_minor, key_full;  // max block norms
    unsigned long long key_major16, key_res16;          // bf16 copy
    unsigned long long key_amax;                        // max |x[:k]| (float bits)
    unsigned long long key_major8, key_res8;            // fp8 copy
    unsigned long long key_majori, key_resi;            // int8 copy
    unsigned long long bad_rows, nonfinite_rows;
    long long first_bad;
};

__global__ void build_stats_init(BuildStats *s) {
    if (threadIdx.x == 0) {
        s->key_major = s->key_minor = s->key_full = 0;
        s->key_major16 = s->key_res16 = 0;
        s->key_amax = s->key_major8 = s->key_res8 = 0;
        s->key_majori = s->key_resi = 0;
        s->bad_rows = s->nonfinite_rows = 0;
        s->first_bad = 0x7fffffffffffffffll;
    }
}

__device__ __forceinline__ float bf16_round(float f) {
    // round-to-nearest-even onto the 8-bit bfloat16 significand
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int w = 1; w < NT / 64; ++w) r = fmax(r, sh[w]);
    __syncthreads();
    return r;
}

// Half a wave per row (four elements per lane, 16-byte loads): float64 block
// norms, the Eq. 1 check and the maxima over the rows; a grid-stride loop so
// each work-group issues one set of atomics.
__global__ __launch_bounds__(256) void build_norms(const float4 *__restrict__ db, int64_t n,
                                                   int k, double alpha, BuildStats *st) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
    const double tol = ldexp(1.0, -13);
    const double cM = sqrt(1.0 - alpha), cm = sqrt(alpha);
    double nM = 0, nm = 0, nf = 0, nM16 = 0, r16 = 0, amax = 0;
    for (int64_t r = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 2 + h; r < n;
         r += (int64_t)gridDim.x * 8) {
        const float4 x4 = db[r * 32 + l];
        const float xv[4] = {x4.x, x4.y, x4.z, x4.w};
        double sM = 0, sm = 0, s16 = 0, sr = 0, am = 0;
        int bad = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float v = xv[u];
            bad |= !isfinite(v);
            const double dv = (double)v;
            if (4 * l + u < k) {
                am = fmax(am, fabs(dv));
                sM = fma(dv, dv, sM);
                const double b = (double)bf16_round(v);
                s16 = fma(b, b, s16);
                sr = fma(b - dv, b - dv, sr);
            } else {
                sm = fma(dv, dv, sm);
            }
        }
        for (int o = 16; o > 0; o >>= 1) {
            sM += __shfl_xor(sM, o);
            sm += __shfl_xor(sm, o);
            s16 += __shfl_xor(s16, o);
            sr += __shfl_xor(sr, o);
            am = fmax(am, __shfl_xor(am, o));
            bad |= __shfl_xor(bad, o);
        }
        const bool finite = !bad;
        const double rM = sqrt(sM), rm = sqrt(sm);
        const bool ok = finite && fabs(rM - cM) <= tol * cM &&
                        (alpha > 0.0 ? fabs(rm - cm) <= tol * cm : rm <= ldexp(1.0, -20));
        if (l == 0) {
            if (!ok) {
                atomicAdd(&st->bad_rows, 1ull);
                atomicMin(&st->first_bad, (long long)r);
            }
            if (!finite) atomicAdd(&st->nonfinite_rows, 1ull);
        }
        if (!finite) continue;
        nM = fmax(nM, rM);
        nm = fmax(nm, rm);
        nf = fmax(nf, sqrt(sM + sm));
        nM16 = fmax(nM16, sqrt(s16));
        r16 = fmax(r16, sqrt(sr));
        amax = fmax(amax, am);
    }
    double a = block_max<256>(nM, sh);
    double b = block_max<256>(nm, sh);
    double c = block_max<256>(nf, sh);
    double d = block_max<256>(nM16, sh);
    double e = block_max<256>(r16, sh);
    double f = block_max<256>(amax, sh);
    if (threadIdx.x == 0) {
        atomicMax(&st->key_amax, key_of(f));
        atomicMax(&st->key_major, key_of(a));
        atomicMax(&st->key_minor, key_of(b));
        atomicMax(&st->key_full, key_of(c));
        atomicMax(&st->key_major16, key_of(d));
        atomicMax(&st->key_res16, key_of(e));
    }
}

// major32[i][c] = x[i][c] for c < k (zero elsewhere and for padded rows).
__global__ __launch_bounds__(256) void build_major32(const float *__restrict__ db, int64_t n,
                                                     int64_t n_pad, int k, int kp,
                                                     float *__restrict__ out) {
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_pad * kp) return;
    int64_t i = t / kp;
    int c = (int)(t % kp);
    out[t] = (i < n && c < k) ? db[i * kDim + c] : 0.0f;
}

__global__ __launch_bounds__(256) void build_major16(const float *__restrict__ db, int64_t n,
                                                     int64_t n_pad, int k, int kb,
                                                     uint16_t *__restrict__ out) {
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_pad * kb) return;
    int64_t i = t / kb;
    int c = (int)(t % kb);
    float v = (i < n && c < k) ? db[i * kDim + c] : 0.0f;
    out[t] = (uint16_t)(__float_as_uint(bf16_round(v)) >> 16);
}

// fp8 and int8 copies: thread per row; each scale comes from the measured
// max |x[:k]| (every thread derives the same power of two), and the row's
// residual ||scale * code - x|| and scaled-copy norm feed the bound slack.
__global__ __launch_bounds__(256) void build_major8(const float *__restrict__ db, int64_t n,
                                                    int64_t n_pad, int k, int k8,
                                                    BuildStats *st, uint8_t *__restrict__ out,
                                                    int8_t *__restrict__ out_i8) {
    __shared__ double sh[4];
    const float amax = (float)sim_of_key(st->key_amax);
    const float scale = fp8_scale_for(amax), scale_i = int8_scale_for(amax);
    const float inv = 1.0f / scale, inv_i = 1.0f / scale_i;  // exact: powers of two
    double rn = 0, rr = 0, rni = 0, rri = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_pad;
         i += (int64_t)gridDim.x * 256) {
        double sn = 0, sr = 0, sni = 0, sri = 0;
        for (int c = 0; c < k8; ++c) {
            const float v = (i < n && c < k) ? db[i * kDim + c] : 0.0f;
            const uint8_t code = fp8_e4m3(v * inv);
            out[i * k8 + c] = code;
            const double back = (double)fp8_e4m3_value(code) * (double)scale;
            sn = fma(back, back, sn);
            sr = fma(back - (double)v, back - (double)v, sr);
            const int8_t ci = int8_code(v * inv_i);
            out_i8[i * k8 + c] = ci;
            const double bi = (double)ci * (double)scale_i;
            sni = fma(bi, bi, sni);
            sri = fma(bi - (double)v, bi - (double)v, sri);
        }
        if (i < n) {
            rn = fmax(rn, sqrt(sn));
            rr = fmax(rr, sqrt(sr));
            rni = fmax(rni, sqrt(sni));
            rri = fmax(rri, sqrt(sri));
        }
    }
    const double a = block_max<256>(rn, sh);
    const double b = block_max<256>(rr, sh);
    const double c = block_max<256>(rni, sh);
    const double d = block_max<256>(rri, sh);
    if (threadIdx.x == 0) {
        atomicMax(&st->key_major8, key_of(a));
        atomicMax(&st->key_res8, key_of(b));
        atomicMax(&st->key_majori, key_of(c));
        atomicMax(&st->key_resi, key_of(d));
    }
}

inline unsigned grid_for(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

double key_to_double_host(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

// The float64 norm of a float32 row block has relative error well below
// 2^-40; scaling by (1 + 2^-40) gives a rigorous upper bound.
double round_up_norm(double v) { return v * (1.0 + ldexp(1.0, -40)); }

void free_index(hn_index *ix) {
    if (!ix) return;
    dev_free(ix->rows);
    dev_free(ix->major32);
    dev_free(ix->major16);
    dev_free(ix->major8);
    dev_free(ix->major_i8);
    dev_free(ix->seed_w);
    dev_free(ix->seed_b);
    dev_free(ix->seed_anchor);
    delete ix;
}

}  // namespace
}  // namespace hn

using namespace hn;

extern "C" const char *hn_last_error(void) { return hn::g_err; }

extern "C" int hn_set_memory_budget(int64_t max_bytes) {
    clear_error();
    if (max_bytes < 0) return fail(HN_ERR_INVALID_ARG, "max_bytes must be >= 0");
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_budget = max_bytes;
    return HN_OK;
}

extern "C" int64_t hn_memory_held(void) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    return g_mem_held;
}

extern "C" int hn_release_scratch(void *stream) {
    clear_error();
    return release_arenas(stream);
}

extern "C" void hn_free_index(hn_index *ix) {
    if (!ix) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != ix->device) {
        (void)hipSetDevice(ix->device);
        free_index(ix);
        (void)hipSetDevice(cur);
        return;
    }
    free_index(ix);
}

extern "C" int hn_index_info(const hn_index *ix, int64_t *n, int32_t *k, double *alpha,
                             double *norms) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (n) *n = ix->n;
    if (k) *k = ix->k;
    if (alpha) *alpha = ix->alpha;
    if (norms) {
        norms[0] = ix->mu_major;
        norms[1] = ix->mu_minor;
        norms[2] = ix->mu_full;
    }
    return HN_OK;
}

extern "C" int hn_build_index(const float *db, int64_t n, int32_t d, int32_t k, double alpha,
                              uint32_t flags, void *stream, hn_index **out) {
    clear_error();
    if (!out) return fail(HN_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!db) return fail(HN_ERR_INVALID_ARG, "db is null");
    if (!aligned16(db)) return fail(HN_ERR_INVALID_ARG, "db must be 16-byte aligned");
    if (d != kDim) return fail(HN_ERR_INVALID_ARG, "d must be 128 (got %d)", d);
    if (k < 1 || k > kDim - 1) return fail(HN_ERR_INVALID_ARG, "k must be in [1,127] (got %d)", k);
    if (!(alpha >= 0.0 && alpha < 1.0)) return fail(HN_ERR_INVALID_ARG, "alpha must be in [0,1)");
    if (n < 1) return fail(HN_ERR_INVALID_ARG, "n must be >= 1");
    if (n >= (int64_t)1 << 31) return fail(HN_ERR_UNSUPPORTED, "n must be < 2^31");
    if (flags & ~(uint32_t)HN_BUILD_NO_VALIDATE)
        return fail(HN_ERR_INVALID_ARG, "unknown build flags 0x%x", flags);
    hipStream_t s = (hipStream_t)stream;

    hn_index *ix = new (std::nothrow) hn_index();
    if (!ix) return fail(HN_ERR_OOM, "host allocation failed");
    HN_HIP(hipGetDevice(&ix->device));
    ix->n = n;
    ix->n_pad = (n + 63) / 64 * 64;
    ix->k = k;
    ix->alpha = alpha;
    ix->kp = f32_width(k);
    ix->kb = bf16_width(k);
    ix->k8 = k <= 16 ? 16 : (k <= 32 ? 32 : 0);

    BuildStats *st = nullptr;
    auto cleanup = [&](int code) {
        dev_free(st);
        free_index(ix);
        return code;
    };
    if (dev_alloc(&st, sizeof(BuildStats)) != hipSuccess ||
        dev_alloc(&ix->rows, (size_t)n * kDim * sizeof(float)) != hipSuccess ||
        dev_alloc(&ix->major32, (size_t)ix->n_pad * ix->kp * sizeof(float)) != hipSuccess ||
        dev_alloc(&ix->major16, (size_t)ix->n_pad * ix->kb * sizeof(uint16_t)) != hipSuccess ||
        (ix->k8 && dev_alloc(&ix->major8, (size_t)ix->n_pad * ix->k8) != hipSuccess) ||
        (ix->k8 && dev_alloc(&ix->major_i8, (size_t)ix->n_pad * ix->k8) != hipSuccess)) {
        (void)hipGetLastError();
        fail(HN_ERR_OOM, "device allocation failed for n=%lld", (long long)n);
        return cleanup(HN_ERR_OOM);
    }
    hipLaunchKernelGGL(build_stats_init, dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL(build_norms, dim3(std::min(grid_for(n, 8), 4096u)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(db), n, k, alpha, st);
    hipLaunchKernelGGL(build_major32, dim3(grid_for(ix->n_pad * ix->kp, 256)), dim3(256), 0, s,
                       db, n, ix->n_pad, k, ix->kp, ix->major32);
    hipLaunchKernelGGL(build_major16, dim3(grid_for(ix->n_pad * ix->kb, 256)), dim3(256), 0, s,
                       db, n, ix->n_pad, k, ix->kb, ix->major16);
    if (ix->k8)
        hipLaunchKernelGGL(build_major8, dim3(std::min(grid_for(ix->n_pad, 256), 4096u)), dim3(256), 0, s, db, n,
                           ix->n_pad, k, ix->k8, st, ix->major8, ix->major_i8);
    hipError_t e = hipMemcpyAsync(ix->rows, db, (size_t)n * kDim * sizeof(float),
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipGetLastError();
    BuildStats h;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fail(HN_ERR_DEVICE, "index build: %s", hipGetErrorString(e));
        return cleanup(HN_ERR_DEVICE);
    }
    if (h.nonfinite_rows || (h.bad_rows && !(flags & HN_BUILD_NO_VALIDATE))) {
        fail(HN_ERR_NOT_NORMALIZED,
             "%llu rows violate the HN block norms (first bad row %lld)", h.bad_rows,
             h.first_bad);
        return cleanup(HN_ERR_NOT_NORMALIZED);
    }
    // With HN_BUILD_NO_VALIDATE a finite off-norm row is accepted: the bound
    // slack uses the measured maxima below, so the search stays exact.
    ix->mu_major = round_up_norm(key_to_double_host(h.key_major));
    ix->mu_minor = round_up_norm(key_to_double_host(h.key_minor));
    ix->mu_full = round_up_norm(key_to_double_host(h.key_full));
    ix->mu_major16 = round_up_norm(key_to_double_host(h.key_major16));
    ix->res16 = round_up_norm(key_to_double_host(h.key_res16));
    {
        // the same power of two the device derived from the same float
        int ex;
        const float amax = (float)key_to_double_host(h.key_amax);
        (void)frexpf(amax, &ex);
        ix->scale8 = amax > 0.0f ? ldexpf(1.0f, ex - 8) : 1.0f;
        ix->scale_i8 = amax > 0.0f ? ldexpf(1.0f, ex - 7) : 1.0f;
    }
    ix->mu_major8 = round_up_norm(key_to_double_host(h.key_major8));
    ix->res8 = round_up_norm(key_to_double_host(h.key_res8));
    ix->mu_major_i8 = round_up_norm(key_to_double_host(h.key_majori));
    ix->res_i8 = round_up_norm(key_to_double_host(h.key_resi));
    dev_free(st);
    *out = ix;
    return HN_OK;
}
