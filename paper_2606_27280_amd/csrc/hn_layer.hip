// The HN layer (Eq. 1) and its vector-Jacobian product: the step that puts
// embeddings on the split sphere before they enter an index.  A wave takes
// kRows consecutive 128-d rows, two elements per lane: all of its row loads
// are issued before any arithmetic, so each wave keeps kRows x 512 B in
// flight.  Block norms in float64, every output rounded once to float32.
// HBM-bound: 1 KiB moved per row forward, 1.5 KiB backward.
#include <math.h>

#include "hn_internal.h"

namespace hn {
namespace {

constexpr int kRows = 8;  // rows per wave

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Row status: 0 ok; 1 zero major block; 2 zero minor block with alpha > 0;
// 3 a non-finite component.  Blocks that cannot be normalised come out zero.
__device__ __forceinline__ void fwd_row(const float2 v, const int64_t r, const int lane, int k,
                                        double c_major, double c_minor,
                                        float2 *__restrict__ out, int32_t *__restrict__ status) {
    const int j0 = 2 * lane, j1 = j0 + 1;
    const double a0 = v.x, a1 = v.y;
    const double sM = wave_sum((j0 < k ? a0 * a0 : 0.0) + (j1 < k ? a1 * a1 : 0.0));
    const double sm = wave_sum((j0 < k ? 0.0 : a0 * a0) + (j1 < k ? 0.0 : a1 * a1));
    const double nM = sqrt(sM), nm = sqrt(sm);
    const bool finite = isfinite(sM) && isfinite(sm);
    const bool okM = finite && nM > 0.0;
    const bool okm = finite && (c_minor == 0.0 || nm > 0.0);
    auto y = [&](double a, int j) -> float {
        if (j < k) return okM ? (float)(c_major * a / nM) : 0.0f;
        return (okm && c_minor != 0.0) ? (float)(c_minor * a / nm) : 0.0f;
    };
    out[r * 64 + lane] = make_float2(y(a0, j0), y(a1, j1));
    if (status && lane == 0) status[r] = !finite ? 3 : (!okM ? 1 : (!okm ? 2 : 0));
}

__global__ __launch_bounds__(256) void layer_fwd(const float2 *__restrict__ f, int64_t b, int k,
                                                 double c_major, double c_minor,
                                                 float2 *__restrict__ out,
                                                 int32_t *__restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kRows;
    if (r0 >= b) return;
    float2 v[kRows];
#pragma unroll
    for (int t = 0; t < kRows; ++t)
        v[t] = r0 + t < b ? f[(r0 + t) * 64 + lane] : make_float2(0.0f, 0.0f);
#pragma unroll
    for (int t = 0; t < kRows; ++t)
        if (r0 + t < b) fwd_row(v[t], r0 + t, lane, k, c_major, c_minor, out, status);
}

// dL/df for y = c u / ||u|| per block: (c / ||u||) (g - v (v . g)), v = u / ||u||.
__device__ __forceinline__ void bwd_row(const float2 v, const float2 w, const int64_t r,
                                        const int lane, int k, double c_major, double c_minor,
                                        float2 *__restrict__ grad) {
    const int j0 = 2 * lane, j1 = j0 + 1;
    const double a0 = v.x, a1 = v.y, g0 = w.x, g1 = w.y;
    const bool M0 = j0 < k, M1 = j1 < k;
    const double nM = sqrt(wave_sum((M0 ? a0 * a0 : 0.0) + (M1 ? a1 * a1 : 0.0)));
    const double nm = sqrt(wave_sum((M0 ? 0.0 : a0 * a0) + (M1 ? 0.0 : a1 * a1)));
    // v . g per block, v = u / ||u||
    const double dM = wave_sum((M0 ? (a0 / nM) * g0 : 0.0) + (M1 ? (a1 / nM) * g1 : 0.0));
    const double dm = wave_sum((M0 ? 0.0 : (a0 / nm) * g0) + (M1 ? 0.0 : (a1 / nm) * g1));
    auto d = [&](double a, double gg, bool major) -> float {
        const double c = major ? c_major : c_minor, n = major ? nM : nm, dot = major ? dM : dm;
        if (c == 0.0 || !(n > 0.0) || !isfinite(n)) return 0.0f;
        return (float)((c / n) * (gg - (a / n) * dot));
    };
    grad[r * 64 + lane] = make_float2(d(a0, g0, M0), d(a1, g1, M1));
}

__global__ __launch_bounds__(256) void layer_bwd(const float2 *__restrict__ f,
                                                 const float2 *__restrict__ g, int64_t b, int k,
                                                 double c_major, double c_minor,
                                                 float2 *__restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kRows;
    if (r0 >= b) return;
    float2 v[kRows], w[kRows];
#pragma unroll
    for (int t = 0; t < kRows; ++t) {
        const bool in = r0 + t < b;
        v[t] = in ? f[(r0 + t) * 64 + lane] : make_float2(0.0f, 0.0f);
        w[t] = in ? g[(r0 + t) * 64 + lane] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int t = 0; t < kRows; ++t)
        if (r0 + t < b) bwd_row(v[t], w[t], r0 + t, lane, k, c_major, c_minor, grad);
}

unsigned blocks_of_rows(int64_t b) { return (unsigned)((b + 4 * kRows - 1) / (4 * kRows)); }

int check_layer(int64_t b, int32_t d, int32_t k, double alpha) {
    if (d != kDim) return fail(HN_ERR_INVALID_ARG, "d must be 128 (got %d)", d);
    if (k < 1 || k > kDim - 1) return fail(HN_ERR_INVALID_ARG, "k must be in [1,127] (got %d)", k);
    if (!(alpha >= 0.0 && alpha < 1.0)) return fail(HN_ERR_INVALID_ARG, "alpha must be in [0,1)");
    if (b < 0) return fail(HN_ERR_INVALID_ARG, "b must be >= 0");
    if (b > ((int64_t)1 << 33)) return fail(HN_ERR_UNSUPPORTED, "b must be <= 2^33");
    return HN_OK;
}

}  // namespace
}  // namespace hn

using namespace hn;

extern "C" int hn_layer_forward(const float *f, int64_t b, int32_t d, int32_t k, double alpha,
                                float *out, int32_t *status, void *stream) {
    clear_error();
    int rc = check_layer(b, d, k, alpha);
    if (rc) return rc;
    if (b == 0) return HN_OK;
    if (!f || !out) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    ProfScope prof_(s, "hn_layer_fwd");
    hipLaunchKernelGGL(layer_fwd, dim3(blocks_of_rows(b)), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(f), b, k, sqrt(1.0 - alpha), sqrt(alpha),
                       reinterpret_cast<float2 *>(out), status);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_layer_backward(const float *f, const float *g, int64_t b, int32_t d, int32_t k,
                                 double alpha, float *grad, void *stream) {
    clear_error();
    int rc = check_layer(b, d, k, alpha);
    if (rc) return rc;
    if (b == 0) return HN_OK;
    if (!f || !g || !grad) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    ProfScope prof_(s, "hn_layer_bwd");
    hipLaunchKernelGGL(layer_bwd, dim3(blocks_of_rows(b)), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(f), reinterpret_cast<const float2 *>(g), b,
                       k, sqrt(1.0 - alpha), sqrt(alpha), reinterpret_cast<float2 *>(grad));
    HN_HIP(hipGetLastError());
    return HN_OK;
}
