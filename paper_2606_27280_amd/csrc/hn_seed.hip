// The learned seed: a small MLP maps a query to scores over a fixed set of
// anchor entries; the best canonical sim among the anchors of its 4 largest
// scores is an admissible initial lower bound L_q (any real entry's sim is).
// This file holds the model's kernels (forward, backward, AdamW, on float32
// MFMA), the seeded k-means++ anchor selection (D^2 seeding), the training
// labels (the anchor nearest to each query's exact neighbour) and the seed
// stage the search runs.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hn_internal.h"

namespace hn {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kIn = HN_MLP_IN, kH = HN_MLP_H, kOut = HN_MLP_OUT;
// Flat float32 parameter vector: W1 [kH][kIn] | b1 | W2 [kH][kH] | b2 |
// W3 [kOut][kH] | b3 (weights row-major, output-major).
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kH * kIn;
constexpr int64_t kOffW2 = kOffB1 + kH;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kH * kH;
constexpr int64_t kOffW3 = kOffB2 + kH;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kOut * kH;
constexpr int64_t kParams = kOffB3 + kOut;
static_assert(kParams == HN_MLP_PARAMS, "parameter layout");
// The index keeps the weights as bf16 (W1 | W2 | W3) and the biases as float32.
constexpr int64_t kW1 = 0, kW2 = (int64_t)kH * kIn, kW3 = kW2 + (int64_t)kH * kH;
constexpr int64_t kWeights = kW3 + (int64_t)kOut * kH;
constexpr int kB1 = 0, kB2 = kH, kB3 = 2 * kH, kBiases = 2 * kH + kOut;

unsigned blocks_of(int64_t items, int per = 256) {
    return (unsigned)std::max<int64_t>(1, (items + per - 1) / per);
}

// ---------------------------------------------------------------- GEMM

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m a_m + k a_k] and
// B(k, n) = B[k b_k + n b_n], then an epilogue.  One work-group of 4 waves
// makes a 64x64 tile of C, each wave a 32x32 block on 32x32x2 float32 MFMA;
// 32-deep slices of A and B are staged in LDS (loaded along whichever
// dimension is contiguous).
enum Epi { kEpiStore = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluGrad = 3 };
// B element kinds: float32; float32 rounded to bf16 on load (the forward's
// weights during training); bf16 bits.
enum BKind { kBF32 = 0, kBRound = 1, kBBf16 = 2 };

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t a_m, a_k;
    const void *B;
    int64_t b_k, b_n;
    float *C;
    int64_t c_m;
    const float *bias;  // [N]
    float *Z;           // bias+GELU: receives the pre-activation (may be NULL);
                        // GELU gradient: holds it.  Same layout as C.
};

__device__ __forceinline__ float bf16_round_f(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// Exact GELU x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 and its derivative
// Phi(x) + x phi(x).
constexpr float kRsqrt2 = 0.70710678118654752f;
constexpr float kRsqrt2Pi = 0.39894228040143268f;
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * kRsqrt2)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * kRsqrt2)) + x * kRsqrt2Pi * expf(-0.5f * x * x);
}

template <int EPI, int BK>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs G) {
    __shared__ float As[64][33];
    __shared__ float Bs[32][65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;  // rows on x: up to 2^31 blocks
    const bool a_cols = G.a_m == 1, b_rows = G.b_n == 1;
    v16f acc = {};
    for (int k0 = 0; k0 < G.K; k0 += 32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = tid + 256 * i;
            const int mm = a_cols ? (e & 63) : (e >> 5), ka = a_cols ? (e >> 6) : (e & 31);
            const int gm = m0 + mm, gka = k0 + ka;
            As[mm][ka] = (gm < G.M && gka < G.K) ? G.A[gm * G.a_m + gka * G.a_k] : 0.0f;
            const int nn = b_rows ? (e & 63) : (e >> 5), kb = b_rows ? (e >> 6) : (e & 31);
            const int gn = n0 + nn, gkb = k0 + kb;
            float bv = 0.0f;
            if (gn < G.N && gkb < G.K) {
                const int64_t off = gkb * G.b_k + gn * G.b_n;
                if (BK == kBBf16) {
                    bv = __uint_as_float((uint32_t)(static_cast<const uint16_t *>(G.B)[off]) << 16);
                } else {
                    bv = static_cast<const float *>(G.B)[off];
                    if (BK == kBRound) bv = bf16_round_f(bv);
                }
            }
            Bs[kb][nn] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 2) {
            const float a = As[wm * 32 + (lane & 31)][kk + (lane >> 5)];
            const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn * 32 + (lane & 31);
        if (row < G.M && col < G.N) {
            const int64_t o = row * G.c_m + col;
            float r = acc[v];
            if (EPI == kEpiBias || EPI == kEpiBiasGelu) r += G.bias[col];
            if (EPI == kEpiBiasGelu) {
                if (G.Z) G.Z[o] = r;
                r = gelu_f(r);
            }
            if (EPI == kEpiGeluGrad) r *= gelu_grad_f(G.Z[o]);
            G.C[o] = r;
        }
    }
}

template <int EPI>
void gemm(const GemmArgs &G, int bkind, hipStream_t s) {
    const dim3 grid((unsigned)((G.M + 63) / 64), (unsigned)((G.N + 63) / 64));
    switch (bkind) {
        case kBF32: hipLaunchKernelGGL((gemm_kernel<EPI, kBF32>), grid, dim3(256), 0, s, G); break;
        case kBRound: hipLaunchKernelGGL((gemm_kernel<EPI, kBRound>), grid, dim3(256), 0, s, G); break;
        default: hipLaunchKernelGGL((gemm_kernel<EPI, kBBf16>), grid, dim3(256), 0, s, G); break;
    }
}

GemmArgs gargs(int M, int N, int K, const float *A, int64_t a_m, int64_t a_k, const void *B,
               int64_t b_k, int64_t b_n, float *C, int64_t c_m, const float *bias = nullptr,
               float *Z = nullptr) {
    GemmArgs G;
    G.M = M;
    G.N = N;
    G.K = K;
    G.A = A;
    G.a_m = a_m;
    G.a_k = a_k;
    G.B = B;
    G.b_k = b_k;
    G.b_n = b_n;
    G.C = C;
    G.c_m = c_m;
    G.bias = bias;
    G.Z = Z;
    return G;
}

// ---------------------------------------------------------------- MLP

// Weights of one forward: float32 (rounded to bf16 on load) or bf16 bits.
struct MlpWeights {
    const void *w1, *w2, *w3;
    const float *b1, *b2, *b3;
    int bkind;
};

MlpWeights weights_of_params(const float *p) {
    return MlpWeights{p + kOffW1, p + kOffW2, p + kOffW3, p + kOffB1, p + kOffB2, p + kOffB3,
                      kBRound};
}

struct MlpBufs {
    float *z1, *h1, *z2, *h2, *logits;  // [b][kH] x 4 (z may be NULL), [b][kOut]
};

void mlp_forward(const MlpWeights &W, const float *x, int64_t b, const MlpBufs &M, hipStream_t s) {
    const int B = (int)b;
    gemm<kEpiBiasGelu>(gargs(B, kH, kIn, x, kIn, 1, W.w1, 1, kIn, M.h1, kH, W.b1, M.z1), W.bkind, s);
    gemm<kEpiBiasGelu>(gargs(B, kH, kH, M.h1, kH, 1, W.w2, 1, kH, M.h2, kH, W.b2, M.z2), W.bkind, s);
    gemm<kEpiBias>(gargs(B, kOut, kH, M.h2, kH, 1, W.w3, 1, kH, M.logits, kOut, W.b3), W.bkind, s);
}

// One wave per row: dL/dlogits = (softmax - onehot) / b and the row's loss
// log(sum exp) - z_label.  A label outside [0, kOut) gives a NaN loss.
__global__ __launch_bounds__(256) void ce_kernel(const float *__restrict__ logits,
                                                 const int32_t *__restrict__ labels, int64_t b,
                                                 float *__restrict__ dlogits,
                                                 float *__restrict__ row_loss) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= b) return;
    const float *z = logits + r * kOut;
    constexpr int kPer = kOut / 64;
    float v[kPer];
    float mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        v[i] = z[lane + 64 * i];
        mx = fmaxf(mx, v[i]);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        v[i] = expf(v[i] - mx);
        sum += v[i];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    const int lab = labels[r];
    const bool ok = lab >= 0 && lab < kOut;
    const float inv_b = 1.0f / (float)b;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int j = lane + 64 * i;
        dlogits[r * kOut + j] = (v[i] / sum - (j == lab ? 1.0f : 0.0f)) * inv_b;
    }
    if (lane == 0) row_loss[r] = ok ? logf(sum) + mx - z[lab] : NAN;
}

// out[c] = sum over rows of g[r][c] (bias gradients), sequential per column.
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ g, int64_t rows,
                                                     int cols, float *__restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.0f;
    for (int64_t r = 0; r < rows; ++r) acc += g[r * cols + c];
    out[c] = acc;
}

// Mean of v[0..n) by one work-group in a fixed order.
__global__ __launch_bounds__(256) void mean_kernel(const float *__restrict__ v, int64_t n,
                                                   float *__restrict__ out) {
    __shared__ float sh[256];
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] / (float)n;
}

struct GradBufs {
    MlpBufs f;
    float *dlogits, *dz2, *dz1, *row_loss;
};

size_t grad_floats(int64_t b) { return (size_t)b * (6 * kH + 2 * kOut + 1) + 64 * 11; }

GradBufs grad_bufs(Arena *ar, int64_t b) {
    GradBufs G;
    G.f.z1 = ar->take<float>(b * kH);
    G.f.h1 = ar->take<float>(b * kH);
    G.f.z2 = ar->take<float>(b * kH);
    G.f.h2 = ar->take<float>(b * kH);
    G.f.logits = ar->take<float>(b * kOut);
    G.dlogits = ar->take<float>(b * kOut);
    G.dz2 = ar->take<float>(b * kH);
    G.dz1 = ar->take<float>(b * kH);
    G.row_loss = ar->take<float>(b);
    return G;
}

// Forward with bf16-rounded weights, softmax cross-entropy, backward; the
// gradient has the parameter layout; loss (device, one float) is the mean.
void mlp_grad(const float *params, const float *x, const int32_t *labels, int64_t b,
              float *grads, float *loss, const GradBufs &T, hipStream_t s) {
    const MlpWeights W = weights_of_params(params);
    mlp_forward(W, x, b, T.f, s);
    const int B = (int)b;
    hipLaunchKernelGGL(ce_kernel, dim3(blocks_of(b, 4)), dim3(256), 0, s, T.f.logits, labels, b,
                       T.dlogits, T.row_loss);
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, T.row_loss, b, loss);
    // layer 3: dW3 = dlogits^T h2, db3, dz2 = (dlogits W3) * gelu'(z2)
    gemm<kEpiStore>(gargs(kOut, kH, B, T.dlogits, 1, kOut, T.f.h2, kH, 1, grads + kOffW3, kH),
                    kBF32, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_of(kOut)), dim3(256), 0, s, T.dlogits, b, kOut,
                       grads + kOffB3);
    gemm<kEpiGeluGrad>(gargs(B, kH, kOut, T.dlogits, kOut, 1, W.w3, kH, 1, T.dz2, kH, nullptr,
                             T.f.z2),
                       W.bkind, s);
    // layer 2
    gemm<kEpiStore>(gargs(kH, kH, B, T.dz2, 1, kH, T.f.h1, kH, 1, grads + kOffW2, kH), kBF32, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_of(kH)), dim3(256), 0, s, T.dz2, b, kH,
                       grads + kOffB2);
    gemm<kEpiGeluGrad>(gargs(B, kH, kH, T.dz2, kH, 1, W.w2, kH, 1, T.dz1, kH, nullptr, T.f.z1),
                       W.bkind, s);
    // layer 1
    gemm<kEpiStore>(gargs(kH, kIn, B, T.dz1, 1, kH, x, kIn, 1, grads + kOffW1, kIn), kBF32, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_of(kH)), dim3(256), 0, s, T.dz1, b, kH,
                       grads + kOffB1);
}

// One AdamW step (decoupled weight decay); c1, c2 are the bias corrections
// 1 / (1 - beta^t).
__global__ __launch_bounds__(256) void adamw_kernel(float *__restrict__ w,
                                                    const float *__restrict__ g,
                                                    float *__restrict__ m, float *__restrict__ v,
                                                    int64_t n, float lr, float b1, float b2,
                                                    float eps, float wd, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] = w[i] - lr * (mi * c1 / (sqrtf(vi * c2) + eps) + wd * w[i]);
    }
}

int check_adamw(const hn_adamw_opts *o) {
    if (!o) return fail(HN_ERR_INVALID_ARG, "null optimizer options");
    if (!(o->lr > 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) ||
        !(o->eps > 0) || !(o->weight_decay >= 0))
        return fail(HN_ERR_INVALID_ARG, "optimizer options out of range");
    return HN_OK;
}

void adamw(float *params, const float *grads, float *m, float *v, int64_t n, int t,
           const hn_adamw_opts &o, hipStream_t s) {
    const double c1 = 1.0 / (1.0 - pow(o.beta1, t)), c2 = 1.0 / (1.0 - pow(o.beta2, t));
    hipLaunchKernelGGL(adamw_kernel, dim3((unsigned)std::min<int64_t>(blocks_of(n), 4096)),
                       dim3(256), 0, s, params, grads, m, v, n, (float)o.lr, (float)o.beta1,
                       (float)o.beta2, (float)o.eps, (float)o.weight_decay, (float)c1, (float)c2);
}

__global__ void zero_f32(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        p[i] = 0.0f;
}

// ---------------------------------------------------------------- k-means++

__global__ void km_first(const double *u, int64_t n, int64_t *anchors) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t f = (int64_t)floor(u[0] * (double)n);
        anchors[0] = f >= n ? n - 1 : (f < 0 ? 0 : f);
    }
}

__device__ __forceinline__ unsigned long long km_weight(double d) {
    return (unsigned long long)floor(ldexp(d > 0.0 ? d : 0.0, 30));
}

// D(x_i) = min(D(x_i), 2 - 2 sim(a, x_i)) for the newest anchor a; block
// sums of the quantised weights floor(max(0, D) 2^30).
__global__ __launch_bounds__(256) void km_update(const float *__restrict__ rows, int64_t n,
                                                 const int64_t *__restrict__ anchors, int t,
                                                 int first, double *__restrict__ dist,
                                                 unsigned long long *__restrict__ block_sums) {
    __shared__ unsigned long long sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long w = 0;
    if (i < n) {
        const float *a = rows + anchors[t - 1] * kDim;
        const double v = 2.0 - 2.0 * sim64(a, rows + i * kDim);
        double d = first ? v : dist[i];
        if (v < d) d = v;
        dist[i] = d;
        w = km_weight(d);
    }
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Inverse-CDF pick of anchor t: the first entry whose inclusive weight sum
// exceeds floor(u_t * total); n - 1 if none does.  One work-group; exact
// integer sums, so the pick does not depend on the summation order.
__global__ __launch_bounds__(1024) void km_select(const double *__restrict__ dist, int64_t n,
                                                  const unsigned long long *__restrict__ block_sums,
                                                  int n_blocks, const double *__restrict__ u,
                                                  int t, int64_t *__restrict__ anchors) {
    __shared__ unsigned long long part[1024];
    __shared__ unsigned long long wv[256];
    __shared__ unsigned long long sh_before;
    __shared__ int sh_blk;
    const int tid = threadIdx.x;
    const int per = (n_blocks + 1023) / 1024;
    const int lo = min(tid * per, n_blocks), hi = min(lo + per, n_blocks);
    unsigned long long own = 0;
    for (int b = lo; b < hi; ++b) own += block_sums[b];
    part[tid] = own;
    if (tid == 0) sh_blk = -1;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long add = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    const unsigned long long total = part[1023];
    const unsigned long long target = (unsigned long long)floor(u[t] * (double)total);
    const unsigned long long before = part[tid] - own;
    if (before <= target && part[tid] > target) {
        unsigned long long run = before;
        for (int b = lo; b < hi; ++b) {
            if (run + block_sums[b] > target) {
                sh_blk = b;
                sh_before = run;
                break;
            }
            run += block_sums[b];
        }
    }
    __syncthreads();
    const int blk = __builtin_amdgcn_readfirstlane(sh_blk);
    if (blk < 0) {
        if (tid == 0) anchors[t] = n - 1;
        return;
    }
    unsigned long long mine = 0;
    if (tid < 256) {
        const int64_t i = (int64_t)blk * 256 + tid;
        mine = i < n ? km_weight(dist[i]) : 0ull;
        wv[tid] = mine;
    }
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        unsigned long long add = 0;
        if (tid < 256 && tid >= off) add = wv[tid - off];
        __syncthreads();
        if (tid < 256) wv[tid] += add;
        __syncthreads();
    }
    if (tid < 256) {
        const unsigned long long incl = sh_before + wv[tid];
        if (incl - mine <= target && incl > target) anchors[t] = (int64_t)blk * 256 + tid;
    }
}

// ---------------------------------------------------------------- labels

// One wave per query: the anchor a maximising sim(x_nn, x_anchor[a]) (ties to
// the smaller a); -1 when the query has no neighbour.
__global__ __launch_bounds__(256) void label_kernel(const float *__restrict__ rows,
                                                    const int64_t *__restrict__ nn, int64_t q,
                                                    const int64_t *__restrict__ anchors,
                                                    int n_anchor, int32_t *__restrict__ labels) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q) return;
    const int64_t e = nn[i];
    if (e < 0) {
        if (lane == 0) labels[i] = -1;
        return;
    }
    const float *x = rows + e * kDim;
    double bv = -INFINITY;
    int ba = -1;
    for (int a = lane; a < n_anchor; a += 64) {
        const double s = sim64(x, rows + anchors[a] * kDim);
        if (ba < 0 || s > bv) {
            bv = s;
            ba = a;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o);
        const int oa = __shfl_xor(ba, o);
        if (oa >= 0 && (ba < 0 || ov > bv || (ov == bv && oa < ba))) {
            bv = ov;
            ba = oa;
        }
    }
    if (lane == 0) labels[i] = ba;
}

// ---------------------------------------------------------------- seed stage

// One wave per query: the 4 largest logits (ties to the smaller anchor id),
// the canonical sim of each of those anchors, and the best of them (sim desc,
// entry index asc) as L_q and its entry.
__global__ __launch_bounds__(256) void learned_seed_kernel(
    const float *__restrict__ logits, const float *__restrict__ queries, int64_t q,
    const float *__restrict__ rows, const int32_t *__restrict__ anchor, double *__restrict__ lower,
    int64_t *__restrict__ lower_idx) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= q) return;
    constexpr int kPer = kOut / 64;
    float v[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) v[j] = logits[i * kOut + lane + 64 * j];
    int pick = -1;  // lane t < 4 keeps the t-th pick
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float bv = -INFINITY;
        int ba = kOut;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int a = lane + 64 * j;
            if (v[j] > bv || (v[j] == bv && a < ba)) {
                bv = v[j];
                ba = a;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int oa = __shfl_xor(ba, o);
            if (ov > bv || (ov == bv && oa < ba)) {
                bv = ov;
                ba = oa;
            }
        }
        if (ba >= kOut) ba = t;  // all logits NaN: any anchor is admissible
        if (lane == t) pick = ba;
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (lane + 64 * j == ba) v[j] = -INFINITY;
    }
    double sv = -INFINITY;
    int64_t e = -1;
    if (lane < 4) {
        e = anchor[pick];
        sv = sim64(queries + i * kDim, rows + e * kDim);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double os = __shfl_xor(sv, o);
        const int64_t oe = __shfl_xor(e, o);
        if (oe >= 0 && (e < 0 || os > sv || (os == sv && oe < e))) {
            sv = os;
            e = oe;
        }
    }
    if (lane == 0) {
        lower[i] = sv;
        lower_idx[i] = e;
    }
}

__global__ void round_weights(const float *__restrict__ p, uint16_t *__restrict__ w,
                              float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // weights: W1 | W2 | W3 from their parameter offsets
    if (i < kWeights) {
        int64_t src;
        if (i < kW2) src = kOffW1 + i;
        else if (i < kW3) src = kOffW2 + (i - kW2);
        else src = kOffW3 + (i - kW3);
        w[i] = (uint16_t)(__float_as_uint(bf16_round_f(p[src])) >> 16);
    }
    if (i < kBiases) {
        int64_t src;
        if (i < kB2) src = kOffB1 + i;
        else if (i < kB3) src = kOffB2 + (i - kB2);
        else src = kOffB3 + (i - kB3);
        b[i] = p[src];
    }
}

int check_anchors_host(const int64_t *anchors, int32_t n_anchor, int64_t n, hipStream_t s) {
    std::vector<int64_t> h((size_t)n_anchor);
    HN_HIP(hipMemcpyAsync(h.data(), anchors, sizeof(int64_t) * n_anchor, hipMemcpyDeviceToHost, s));
    HN_HIP(hipStreamSynchronize(s));
    for (int32_t a = 0; a < n_anchor; ++a)
        if (h[a] < 0 || h[a] >= n)
            return fail(HN_ERR_INVALID_ARG, "anchor %d = %lld is not an entry (n = %lld)", a,
                        (long long)h[a], (long long)n);
    return HN_OK;
}

}  // namespace

// The search's learned-seed stage (declared in hn_internal.h).
int learned_seed(const hn_index *ix, const float *queries, int64_t q, double *lower,
                 int64_t *lower_idx, hipStream_t s) {
    if (!ix->seed_w) return fail(HN_ERR_INVALID_ARG, "no seed model: call hn_set_seed_model");
    // the forward in slices bounded in memory
    const int64_t slice = std::min<int64_t>(q, 65536);
    Arena *ar = nullptr;
    int rc = arena_for((void *)s, (size_t)slice * (2 * kH + kOut) * 4 + 4096, &ar, 1);
    if (rc) return rc;
    MlpBufs M;
    M.z1 = M.z2 = nullptr;
    M.h1 = ar->take<float>(slice * kH);
    M.h2 = ar->take<float>(slice * kH);
    M.logits = ar->take<float>(slice * kOut);
    const MlpWeights W{ix->seed_w + kW1, ix->seed_w + kW2, ix->seed_w + kW3,
                       ix->seed_b + kB1, ix->seed_b + kB2, ix->seed_b + kB3, kBBf16};
    for (int64_t q0 = 0; q0 < q; q0 += slice) {
        const int64_t b = std::min<int64_t>(slice, q - q0);
        {
            ProfScope prof_(s, "seed_mlp");
            mlp_forward(W, queries + q0 * kDim, b, M, s);
        }
        {
            ProfScope prof_(s, "seed_learned");
            hipLaunchKernelGGL(learned_seed_kernel, dim3(blocks_of(b, 4)), dim3(256), 0, s,
                               M.logits, queries + q0 * kDim, b, ix->rows, ix->seed_anchor,
                               lower + q0, lower_idx + q0);
        }
    }
    HN_HIP(hipGetLastError());
    return HN_OK;
}

}  // namespace hn

using namespace hn;

extern "C" int hn_mlp_forward(const float *params, const float *x, int64_t b, float *logits,
                              void *stream) {
    clear_error();
    if (b < 0) return fail(HN_ERR_INVALID_ARG, "b must be >= 0");
    if (b > (1 << 24)) return fail(HN_ERR_UNSUPPORTED, "b must be <= 2^24");
    if (b == 0) return HN_OK;
    if (!params || !x || !logits) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    Arena *ar = nullptr;
    int rc = arena_for(stream, (size_t)b * 2 * kH * 4 + 4096, &ar, 1);
    if (rc) return rc;
    MlpBufs M;
    M.z1 = M.z2 = nullptr;
    M.h1 = ar->take<float>(b * kH);
    M.h2 = ar->take<float>(b * kH);
    M.logits = logits;
    mlp_forward(weights_of_params(params), x, b, M, s);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_mlp_grad(const float *params, const float *x, const int32_t *labels, int64_t b,
                           float *grads, float *loss, void *stream) {
    clear_error();
    if (b < 1) return fail(HN_ERR_INVALID_ARG, "b must be >= 1");
    if (b > (1 << 20)) return fail(HN_ERR_UNSUPPORTED, "b must be <= 2^20");
    if (!params || !x || !labels || !grads || !loss)
        return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    Arena *ar = nullptr;
    int rc = arena_for(stream, grad_floats(b) * 4 + 4096, &ar, 1);
    if (rc) return rc;
    mlp_grad(params, x, labels, b, grads, loss, grad_bufs(ar, b), s);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_mlp_adamw(float *params, const float *grads, float *m, float *v, int64_t n,
                            int32_t t, const hn_adamw_opts *opts, void *stream) {
    clear_error();
    if (n < 0 || t < 1) return fail(HN_ERR_INVALID_ARG, "need n >= 0 and t >= 1");
    int rc = check_adamw(opts);
    if (rc) return rc;
    if (n == 0) return HN_OK;
    if (!params || !grads || !m || !v) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    adamw(params, grads, m, v, n, t, *opts, (hipStream_t)stream);
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_seed_train(float *params, const float *x, const int32_t *labels, int64_t n,
                             int32_t batch, int32_t epochs, const hn_adamw_opts *opts,
                             float *losses, void *stream) {
    clear_error();
    if (n < 1 || batch < 1 || epochs < 0)
        return fail(HN_ERR_INVALID_ARG, "need n >= 1, batch >= 1, epochs >= 0");
    if (batch > (1 << 20)) return fail(HN_ERR_UNSUPPORTED, "batch must be <= 2^20");
    int rc = check_adamw(opts);
    if (rc) return rc;
    if (!params || !x || !labels) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t b = std::min<int64_t>(batch, n);
    Arena *ar = nullptr;
    rc = arena_for(stream, (grad_floats(b) + 3 * (size_t)kParams + 64) * 4 + 8192, &ar, 1);
    if (rc) return rc;
    const GradBufs T = grad_bufs(ar, b);
    float *grads = ar->take<float>(kParams);
    float *m = ar->take<float>(kParams);
    float *v = ar->take<float>(kParams);
    float *scratch_loss = ar->take<float>(1);
    hipLaunchKernelGGL(zero_f32, dim3(256), dim3(256), 0, s, m, kParams);
    hipLaunchKernelGGL(zero_f32, dim3(256), dim3(256), 0, s, v, kParams);
    const int64_t per_epoch = (n + b - 1) / b;
    int t = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t st = 0; st < per_epoch; ++st) {
            const int64_t start = st * b, bs = std::min<int64_t>(b, n - start);
            float *loss = losses ? losses + (int64_t)ep * per_epoch + st : scratch_loss;
            mlp_grad(params, x + start * kDim, labels + start, bs, grads, loss, T, s);
            adamw(params, grads, m, v, kParams, ++t, *opts, s);
        }
    }
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_kmeanspp(const hn_index *ix, int32_t n_anchor, const double *u,
                           int64_t *anchors, void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (n_anchor < 1 || n_anchor > (1 << 20))
        return fail(HN_ERR_INVALID_ARG, "n_anchor must be in [1, 2^20]");
    if (!u || !anchors) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = ix->n;
    const int n_blocks = (int)((n + 255) / 256);
    Arena *ar = nullptr;
    int rc = arena_for(stream, (size_t)n * 8 + (size_t)n_blocks * 8 + 4096, &ar, 1);
    if (rc) return rc;
    double *dist = ar->take<double>(n);
    unsigned long long *sums = ar->take<unsigned long long>(n_blocks);
    {
        ProfScope prof_(s, "kmeanspp");
        hipLaunchKernelGGL(km_first, dim3(1), dim3(64), 0, s, u, n, anchors);
        for (int t = 1; t < n_anchor; ++t) {
            hipLaunchKernelGGL(km_update, dim3(n_blocks), dim3(256), 0, s, ix->rows, n, anchors, t,
                               t == 1 ? 1 : 0, dist, sums);
            hipLaunchKernelGGL(km_select, dim3(1), dim3(1024), 0, s, dist, n, sums, n_blocks, u, t,
                               anchors);
        }
    }
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_seed_labels(const hn_index *ix, const int64_t *anchors, int32_t n_anchor,
                              const float *queries, int64_t q, int32_t *labels, void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (n_anchor < 1 || n_anchor > (1 << 20))
        return fail(HN_ERR_INVALID_ARG, "n_anchor must be in [1, 2^20]");
    if (q < 0) return fail(HN_ERR_INVALID_ARG, "q must be >= 0");
    if (q == 0) return HN_OK;
    if (!anchors || !queries || !labels) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_anchors_host(anchors, n_anchor, ix->n, s);
    if (rc) return rc;
    Arena *ar = nullptr;
    rc = arena_for(stream, (size_t)q * 16 + 4096, &ar, 1);
    if (rc) return rc;
    int64_t *nn = ar->take<int64_t>(q);
    double *nn_sim = ar->take<double>(q);
    rc = hn_search_top1(ix, queries, q, nn, nn_sim, nullptr, nullptr, nullptr, stream);
    if (rc) return rc;
    {
        ProfScope prof_(s, "seed_labels");
        hipLaunchKernelGGL(label_kernel, dim3(blocks_of(q, 4)), dim3(256), 0, s, ix->rows, nn, q,
                           anchors, n_anchor, labels);
    }
    HN_HIP(hipGetLastError());
    return HN_OK;
}

extern "C" int hn_set_seed_model(hn_index *ix, const float *params, const int64_t *anchors,
                                 int32_t n_anchor, void *stream) {
    clear_error();
    if (!ix) return fail(HN_ERR_INVALID_ARG, "null index");
    if (n_anchor != kOut)
        return fail(HN_ERR_INVALID_ARG, "n_anchor must equal the model's %d outputs", kOut);
    if (!params || !anchors) return fail(HN_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_anchors_host(anchors, n_anchor, ix->n, s);
    if (rc) return rc;
    std::vector<int64_t> h((size_t)n_anchor);
    HN_HIP(hipMemcpy(h.data(), anchors, sizeof(int64_t) * n_anchor, hipMemcpyDeviceToHost));
    std::vector<int32_t> h32(h.begin(), h.end());
    if (!ix->seed_w) {
        if (dev_alloc(&ix->seed_w, kWeights * sizeof(uint16_t)) != hipSuccess ||
            dev_alloc(&ix->seed_b, kBiases * sizeof(float)) != hipSuccess ||
            dev_alloc(&ix->seed_anchor, kOut * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            // all or nothing: a later call allocates the three again
            dev_free(ix->seed_w);
            dev_free(ix->seed_b);
            dev_free(ix->seed_anchor);
            ix->seed_w = nullptr;
            ix->seed_b = nullptr;
            ix->seed_anchor = nullptr;
            return fail(HN_ERR_OOM, "seed model allocation failed");
        }
    }
    hipLaunchKernelGGL(round_weights, dim3(blocks_of(kWeights)), dim3(256), 0, s, params,
                       ix->seed_w, ix->seed_b);
    HN_HIP(hipMemcpyAsync(ix->seed_anchor, h32.data(), sizeof(int32_t) * kOut,
                          hipMemcpyHostToDevice, s));
    HN_HIP(hipStreamSynchronize(s));
    ix->n_anchor = n_anchor;
    return HN_OK;
}
