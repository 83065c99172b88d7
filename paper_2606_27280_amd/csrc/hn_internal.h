// Internal declarations shared by the HIP sources of libhnsearch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hnsearch.h"

namespace hn {

constexpr int kDim = 128;     // descriptor length D
constexpr int kWave = 64;     // CDNA wavefront
constexpr int kWaves = 4;     // waves per scan work-group
constexpr int kBlock = 16;    // entries per MFMA tile row block
constexpr int kXcds = 8;      // MI355X accelerator complex dies

// Set the calling thread's error message and return `code`.
int fail(int code, const char *fmt, ...);
// Rows of 128 float32 values are read with 16-byte loads: their base pointer
// must be 16-byte aligned.
inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
void clear_error();

#define HN_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::hn::fail(HN_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

// Round K up to the float32 MFMA stream width (16x16x4 steps per lane group).
inline int f32_width(int k) {
    int w = 4;
    while (w < k) w *= 2;
    return w;
}
// Round K up to the bf16 stream width (one 16x16x16 or 16x16x32 step per 16/32).
inline int bf16_width(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : (k <= 64 ? 64 : 128)); }

// Device allocations of the library, counted against the memory budget
// (hn_set_memory_budget).  dev_malloc fails with hipErrorOutOfMemory when
// the budget would be exceeded; dev_free(nullptr) does nothing.
hipError_t dev_malloc(void **p, size_t bytes);
void dev_free(void *p);
template <class T>
inline hipError_t dev_alloc(T **p, size_t bytes) {
    return dev_malloc(reinterpret_cast<void **>(p), bytes);
}

// Per-stream scratch arena: grows on demand, reused by later calls on the
// same stream (stream order makes reuse safe).
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};
// Reserve `bytes` of scratch for `stream` (device of the caller).  Returns
// HN_OK and an arena whose `used` is 0.  Slots are independent arenas of the
// same stream: the search uses slot 0, the seed-model code slot 1 (so a seed
// step can run a search and keep its own buffers).
int arena_for(void *stream, size_t bytes, Arena **out, int slot = 0);

// Brackets the kernels launched in its scope with HIP events when a profile
// session is open on the stream (hn_profile_begin); otherwise does nothing.
class ProfScope {
   public:
    ProfScope(hipStream_t s, const char *tag);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

   private:
    hipStream_t stream_;
    const char *tag_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool active_ = false;
};

// Ordered 64-bit key of a double: integer order equals numeric order (for
// non-NaN values, with -0 folded to +0).
__device__ __forceinline__ unsigned long long key_of(double d) {
    d = d + 0.0;
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double sim_of_key(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Canonical float64 sim: ascending j, each float32 product exact in float64.
// kUnroll float4 groups of both rows load together (8: one 128-byte line).
template <int kUnroll = 4>
__device__ __forceinline__ double sim64(const float *__restrict__ q, const float *__restrict__ x) {
    double acc = 0.0;
#pragma unroll kUnroll
    for (int j = 0; j < kDim; j += 4) {
        float4 a = *reinterpret_cast<const float4 *>(q + j);
        float4 b = *reinterpret_cast<const float4 *>(x + j);
        acc = __fma_rn((double)a.x, (double)b.x, acc);
        acc = __fma_rn((double)a.y, (double)b.y, acc);
        acc = __fma_rn((double)a.z, (double)b.z, acc);
        acc = __fma_rn((double)a.w, (double)b.w, acc);
    }
    return acc;
}

// Round-to-nearest-even onto OCP FP8 E4M3FN (bias 7, 3 mantissa bits, no
// infinities; magnitudes at or above 448 saturate to 448, callers scale so
// that this never happens).  Subnormal steps are 2^-9.
__device__ __forceinline__ uint8_t fp8_e4m3(float v) {
    const uint32_t sign = (__float_as_uint(v) >> 31) << 7;
    const float a = fabsf(v);
    if (!(a > 0.0f)) return (uint8_t)sign;             // zero (and NaN, never passed)
    if (a >= 448.0f) return (uint8_t)(sign | 0x7e);
    if (a < 0.015625f) {                               // below 2^-6: subnormal range
        const float m = rintf(a * 512.0f);             // multiples of 2^-9, RNE
        return (uint8_t)(sign | (uint32_t)m);          // m == 8 is 2^-6 = code 0x08
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xff) - 127;  // a = 2^e * mant
    const float mant = __uint_as_float((__float_as_uint(a) & 0x007fffffu) | 0x3f800000u);
    int q = (int)rintf((mant - 1.0f) * 8.0f);          // 3 mantissa bits, RNE
    if (q == 8) {
        q = 0;
        ++e;
    }
    if (e > 8 || (e == 8 && q == 7)) return (uint8_t)(sign | 0x7e);
    return (uint8_t)(sign | (uint32_t)((e + 7) << 3) | (uint32_t)q);
}
__device__ __forceinline__ float fp8_e4m3_value(uint8_t c) {
    const int e = (c >> 3) & 15, m = c & 7;
    const float v = e == 0 ? ldexpf((float)m, -9) : ldexpf(1.0f + m * 0.125f, e - 7);
    return (c & 0x80) ? -v : v;
}
// Power-of-two scale 2^(ceil(log2 amax) - 8): amax / scale <= 256 < 448.
__host__ __device__ __forceinline__ float fp8_scale_for(float amax) {
    if (!(amax > 0.0f)) return 1.0f;
    int e;
    (void)frexpf(amax, &e);  // amax = f * 2^e, 0.5 <= f < 1, so amax <= 2^e
    return ldexpf(1.0f, e - 8);
}

// Power-of-two scale for int8 codes: 2^(e - 7) with amax = f 2^e,
// 0.5 <= f < 1, so |x| / scale < 128; codes are rounded to nearest even and
// clamped to [-127, 127] (the measured residuals cover the clamp).
__host__ __device__ __forceinline__ float int8_scale_for(float amax) {
    if (!(amax > 0.0f)) return 1.0f;
    int e;
    (void)frexpf(amax, &e);
    return ldexpf(1.0f, e - 7);
}
__device__ __forceinline__ int8_t int8_code(float scaled) {
    return (int8_t)fminf(127.0f, fmaxf(-127.0f, rintf(scaled)));
}

// Higham's gamma_n(u).
__host__ __device__ __forceinline__ double gamma_n(int n, double u) {
    return (double)n * u / (1.0 - (double)n * u);
}

// The search's learned-seed stage: per query, L (lower) and its entry
// (lower_idx) from the index's seed model.
int learned_seed(const hn_index *ix, const float *queries, int64_t q, double *lower,
                 int64_t *lower_idx, hipStream_t s);

}  // namespace hn

// The index (opaque to callers).
struct hn_index {
    int device = 0;
    int64_t n = 0, n_pad = 0;  // n_pad: multiple of 64
    int32_t d = 128, k = 0;
    int32_t kp = 0;            // float32 stream width
    int32_t kb = 0;            // bf16 stream width (0 = not built)
    double alpha = 0;
    double mu_major = 0, mu_minor = 0, mu_full = 0;  // rigorous upper bounds
    float *rows = nullptr;       // [n][128] float32 copy, rescoring
    float *major32 = nullptr;    // [n_pad][kp] float32, zero padded
    uint16_t *major16 = nullptr; // [n_pad][kb] bf16 (RNE), zero padded
    double mu_major16 = 0;       // max ||bf16(x[:k])||, rounded up
    double res16 = 0;            // max ||bf16(x[:k]) - x[:k]||, rounded up
    int32_t k8 = 0;              // fp8 stream width (0 = not built: k > 32)
    uint8_t *major8 = nullptr;   // [n_pad][k8] E4M3FN codes of x[:k] / scale8
    float scale8 = 1.0f;         // power-of-two scale of the fp8 copy
    double mu_major8 = 0;        // max ||scale8 * fp8(x[:k])||, rounded up
    double res8 = 0;             // max ||scale8 * fp8(x[:k]) - x[:k]||, rounded up
    int8_t *major_i8 = nullptr;  // [n_pad][k8] int8 codes of x[:k] / scale_i8 (k <= 32)
    float scale_i8 = 1.0f;       // power-of-two scale of the int8 copy
    double mu_major_i8 = 0;      // max ||scale_i8 * code||, rounded up
    double res_i8 = 0;           // max ||scale_i8 * code - x[:k]||, rounded up
    // learned seed model (hn_set_seed_model): bf16 weights W1 | W2 | W3,
    // float32 biases b1 | b2 | b3, anchor entry ids
    uint16_t *seed_w = nullptr;
    float *seed_b = nullptr;
    int32_t *seed_anchor = nullptr;
    int32_t n_anchor = 0;
};
