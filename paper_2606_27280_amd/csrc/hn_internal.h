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
// HN_OK and an arena whose `used` is 0.
int arena_for(void *stream, size_t bytes, Arena **out);

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
__device__ __forceinline__ double sim64(const float *__restrict__ q, const float *__restrict__ x) {
    double acc = 0.0;
#pragma unroll 4
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

// Higham's gamma_n(u).
__host__ __device__ __forceinline__ double gamma_n(int n, double u) {
    return (double)n * u / (1.0 - (double)n * u);
}

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
};
