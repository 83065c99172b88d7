// The HN layer (Eq. 1) and its vector-Jacobian product: the step that puts
// embeddings on the split sphere before they enter an index.  Half a wave
// (32 lanes, four elements each, 16-byte accesses) takes one 128-d row, so a
// load instruction moves two whole rows; a wave issues the loads of its
// rows of its batch before any arithmetic.  Block norms in float64 (the squares of
// float32 values are exact in float64), each block's scale c / ||u|| formed
// once, every output rounded once to float32.  HBM-bound: 1 KiB moved per
// row forward, 1.5 KiB backward.
#include <math.h>

#include "hn_internal.h"

namespace hn {
namespace {

#ifndef HN_LAYER_ROWS_FWD
#define HN_LAYER_ROWS_FWD 8
#endif
#ifndef HN_LAYER_ROWS_BWD
#define HN_LAYER_ROWS_BWD 2
#endif
// rows per wave (two per load instruction): the backward holds twice the
// inputs and more float64 temporaries per row
constexpr int kRowsFwd = HN_LAYER_ROWS_FWD, kRowsBwd = HN_LAYER_ROWS_BWD;

// Sum over the 32 lanes of a half wave.
__device__ __forceinline__ double half_sum(double v) {
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Row status: 0 ok; 1 zero major block; 2 zero minor block with alpha > 0;
// 3 a non-finite component.  Blocks that cannot be normalised come out zero.
__device__ __forceinline__ void fwd_row(const float4 v, const int64_t r, const int l, int k,
                                        double c_major, double c_minor,
                                        float4 *__restrict__ out, int32_t *__restrict__ status) {
    const int j = 4 * l;  // first element of the lane
    const double a[4] = {v.x, v.y, v.z, v.w};
    double pM = 0.0, pm = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (j + u < k)
            pM += a[u] * a[u];
        else
            pm += a[u] * a[u];
    }
    const double sM = half_sum(pM), sm = half_sum(pm);
    const bool finite = isfinite(sM) && isfinite(sm);
    const bool okM = finite && sM > 0.0;
    const bool okm = finite && (c_minor == 0.0 || sm > 0.0);
    const bool usem = okm && c_minor != 0.0;
    const double fM = c_major * rsqrt(sM), fm = c_minor * rsqrt(sm);
    float y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool major = j + u < k;
        y[u] = (major ? okM : usem) ? (float)(a[u] * (major ? fM : fm)) : 0.0f;
    }
    out[r * 32 + l] = make_float4(y[0], y[1], y[2], y[3]);
    if (status && l == 0) status[r] = !finite ? 3 : (!okM ? 1 : (!okm ? 2 : 0));
}

__global__ __launch_bounds__(256) void layer_fwd(const float4 *__restrict__ f, int64_t b, int k,
                                                 double c_major, double c_minor,
                                                 float4 *__restrict__ out,
                                                 int32_t *__restrict__ status) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kRowsFwd;
    if (r0 >= b) return;
    float4 v[kRowsFwd / 2];
#pragma unroll
    for (int t = 0; t < kRowsFwd / 2; ++t) {
        const int64_t r = r0 + 2 * t + h;
        v[t] = r < b ? f[r * 32 + l] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int t = 0; t < kRowsFwd / 2; ++t) {
        const int64_t r = r0 + 2 * t + h;
        // the two halves diverge only at the batch end; the shuffles stay
        // inside a half wave
        if (r < b) fwd_row(v[t], r, l, k, c_major, c_minor, out, status);
    }
}

// dL/df for y = c u / ||u|| per block: (c / ||u||) (g - v (v . g)), v = u / ||u||.
__device__ __forceinline__ void bwd_row(const float4 v, const float4 w, const int64_t r,
                                        const int l, int k, double c_major, double c_minor,
                                        float4 *__restrict__ grad) {
    const int j = 4 * l;
    const double a[4] = {v.x, v.y, v.z, v.w};
    const double g[4] = {w.x, w.y, w.z, w.w};
    double pM = 0.0, pm = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (j + u < k)
            pM += a[u] * a[u];
        else
            pm += a[u] * a[u];
    }
    const double nM = sqrt(half_sum(pM)), nm = sqrt(half_sum(pm));
    const double iM = 1.0 / nM, im = 1.0 / nm;
    double vv[4];  // v = u / ||u||
    double qM = 0.0, qm = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool major = j + u < k;
        vv[u] = a[u] * (major ? iM : im);
        if (major)
            qM += vv[u] * g[u];
        else
            qm += vv[u] * g[u];
    }
    const double dM = half_sum(qM), dm = half_sum(qm);
    // a one-element block maps to the constant +-c: its gradient is exactly 0
    const bool okM = k > 1 && c_major != 0.0 && nM > 0.0 && isfinite(nM);
    const bool okm = kDim - k > 1 && c_minor != 0.0 && nm > 0.0 && isfinite(nm);
    const double sM = okM ? c_major * iM : 0.0, sm = okm ? c_minor * im : 0.0;
    float d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool major = j + u < k;
        const double sc = major ? sM : sm, dot = major ? dM : dm;
        d[u] = sc == 0.0 ? 0.0f : (float)(sc * (g[u] - vv[u] * dot));
    }
    grad[r * 32 + l] = make_float4(d[0], d[1], d[2], d[3]);
}

__global__ __launch_bounds__(256) void layer_bwd(const float4 *__restrict__ f,
                                                 const float4 *__restrict__ g, int64_t b, int k,
                                                 double c_major, double c_minor,
                                                 float4 *__restrict__ grad) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kRowsBwd;
    if (r0 >= b) return;
    float4 v[kRowsBwd / 2], w[kRowsBwd / 2];
#pragma unroll
    for (int t = 0; t < kRowsBwd / 2; ++t) {
        const int64_t r = r0 + 2 * t + h;
        const bool in = r < b;
        v[t] = in ? f[r * 32 + l] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        w[t] = in ? g[r * 32 + l] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int t = 0; t < kRowsBwd / 2; ++t) {
        const int64_t r = r0 + 2 * t + h;
        if (r < b) bwd_row(v[t], w[t], r, l, k, c_major, c_minor, grad);
    }
}

unsigned blocks_of_rows(int64_t b, int rows) { return (unsigned)((b + 4 * rows - 1) / (4 * rows)); }

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
    if (!aligned16(f) || !aligned16(out))
        return fail(HN_ERR_INVALID_ARG, "f and out must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    ProfScope prof_(s, "hn_layer_fwd");
    hipLaunchKernelGGL(layer_fwd, dim3(blocks_of_rows(b, kRowsFwd)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(f), b, k, sqrt(1.0 - alpha), sqrt(alpha),
                       reinterpret_cast<float4 *>(out), status);
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
    if (!aligned16(f) || !aligned16(g) || !aligned16(grad))
        return fail(HN_ERR_INVALID_ARG, "f, g and grad must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    ProfScope prof_(s, "hn_layer_bwd");
    hipLaunchKernelGGL(layer_bwd, dim3(blocks_of_rows(b, kRowsBwd)), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(f), reinterpret_cast<const float4 *>(g), b,
                       k, sqrt(1.0 - alpha), sqrt(alpha), reinterpret_cast<float4 *>(grad));
    HN_HIP(hipGetLastError());
    return HN_OK;
}
