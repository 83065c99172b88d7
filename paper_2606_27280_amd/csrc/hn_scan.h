// Major-prefix scan kernels (the hot loop of Algorithm 1's Phase 1 and of
// its bound test), written for CDNA4 MFMA.
//
// Tile: one wave computes an R-entry x C-query block of scan scores with one
// MFMA shape, entries as the A operand (rows) and queries as the B operand
// (columns).  Two shapes are used: 16x16 (R = C = 16, 4 scores per lane, the
// K dimension split over four 16-lane groups) and 32x32 (R = C = 32, 16 scores
// per lane, K split over two 32-lane groups).  Lane group g reads a contiguous
// slice of each entry row, so an R-entry block of a [n][W] stream is one
// contiguous R * W element read per wave.  The dot product is a sum over k and
// the same k -> (step, lane group) bijection is applied to both operands, so
// any contiguous slicing gives the same set of products; their summation order
// inside the MFMA is covered by the scan's rounding slack, never relied upon.
//
// Work decomposition: a work-group of 4 waves owns one query block (WQ query
// sub-blocks of NQ C-query tiles) and one chunk of entry blocks; the 4 / WQ
// waves that share a sub-block interleave over the chunk's entry blocks.
// Work items (query block, chunk) are numbered chunk-major and split into 8
// contiguous ranges, one per XCD (blockIdx % 8), so the work-groups of one XCD
// pass every query block over the same chunk while it sits in that XCD's L2.
// Filter launches whose waves each own a query sub-block (WQ = 4) with
// several query blocks split the items further: each wave claims (item,
// sub-block) pairs on its own.
// Control flow that decides barriers is kept provably wave-uniform.
#pragma once

#include <algorithm>
#include <climits>

#include "hn_internal.h"

namespace hn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

enum ScanMode { kArgmax = 0, kFilter = 1, kWindow = 2, kStore = 3 };

struct ScanArgs {
    const void *x;      // entry stream, row stride x_stride elements
    int64_t x_stride;
    const void *qs;     // query operands, row stride q_stride elements
    int64_t q_stride;
    int64_t n;          // valid entries
    int32_t n_blocks;   // ceil(n / R)
    int32_t chunk_blocks, n_chunks;
    int32_t n_qb, n_items;
    int32_t q_count, q_pad;
    float *part_val;    // argmax / window: [n_chunks][q_pad]
    int32_t *part_idx;  // argmax: winning lane group, span * G + g (span = kArgSpan blocks)
    const float *thr;   // filter: T_q; window: window width; [q_pad]
    int2 *pairs;        // filter / window: (query, entry)
    float *pair_val;    // window: scan score of the pair
    unsigned long long *counter;
    int64_t cap;
    int32_t *qflag;     // set when a query's pair did not fit
    float *scores;      // store: [q_count][n]
    int *redo;          // items to re-run (capacity n_items)
    unsigned *redo_count;  // zero before the launch
    unsigned *item_ctr;    // kXcds item counters, zero before the launch; NULL: static order
    const float *init_best;  // window: starting running maximum per query, or NULL
    int32_t q_base;     // added to the query of every emitted pair (several
                        // databases sharing one pair list and flag array)
    // filter: rescoring fused into the flush (psim != NULL).  Each stored
    // pair gets its canonical float64 sim in psim and raises best_key of its
    // query; with rs_major32 the float32 major dot is re-checked against
    // rs_thr32 first (-inf when it fails, as the separate rescoring does).
    double *psim;
    unsigned long long *best_key;
    int32_t *cnt;           // survivor counts per query, or NULL
    const float *rs_queries, *rs_rows;  // float32 [q][128], [n][128]
    const float *rs_major32;            // re-check stream [n_pad][rs_kp], or NULL
    const float *rs_thr32;
    int32_t rs_kp, rs_k;
};

// ------------------------------------------------------------ tile shapes

// 16x16 output: lane l holds column l % 16 and rows 4 (l / 16) + v.
struct Shape16 {
    static constexpr int kRows = 16, kCols = 16, kGroups = 4, kAcc = 4;
    static constexpr bool kIntScores = false;  // exact integer sums (mma_i)
    static constexpr bool kFused = false;      // filter flush may rescore (psim)
    static constexpr bool kDenseFilter = false;  // filter flushes as it goes (direct)
    typedef v4f Acc;
    __device__ __forceinline__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
// 32x32 output: lane l holds column l % 32 and rows 8 (v / 4) + 4 (l / 32) + v % 4.
struct Shape32 {
    static constexpr int kRows = 32, kCols = 32, kGroups = 2, kAcc = 16;
    static constexpr bool kIntScores = false;  // exact integer sums (mma_i)
    static constexpr bool kFused = false;      // filter flush may rescore (psim)
    static constexpr bool kDenseFilter = false;  // filter flushes as it goes (direct)
    typedef v16f Acc;
    __device__ __forceinline__ static int out_row(int lane, int v) {
        return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    }
};

template <int N>
struct Regs {  // N consecutive 32-bit values, loaded with the widest loads
    uint32_t v[N];
    __device__ __forceinline__ void load(const void *p) {
        if constexpr (N == 1) {
            v[0] = *reinterpret_cast<const uint32_t *>(p);
        } else if constexpr (N == 2) {
            uint2 a = *reinterpret_cast<const uint2 *>(p);
            v[0] = a.x;
            v[1] = a.y;
        } else {
#pragma unroll
            for (int c = 0; c < N / 4; ++c) {
                uint4 a = reinterpret_cast<const uint4 *>(p)[c];
                v[4 * c + 0] = a.x;
                v[4 * c + 1] = a.y;
                v[4 * c + 2] = a.z;
                v[4 * c + 3] = a.w;
            }
        }
    }
    // The same values through a buffer descriptor: `off` is a byte offset
    // from the descriptor's base; the hardware returns zeros for bytes past
    // its range instead of reading them.
    __device__ __forceinline__ void load_buf(__amdgpu_buffer_rsrc_t r, int off) {
        if constexpr (N == 1) {
            v[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        } else if constexpr (N == 2) {
            const auto a = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            v[0] = a[0];
            v[1] = a[1];
        } else {
#pragma unroll
            for (int c = 0; c < N / 4; ++c) {
                const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * c, 0, 0);
                v[4 * c + 0] = a[0];
                v[4 * c + 1] = a[1];
                v[4 * c + 2] = a[2];
                v[4 * c + 3] = a[3];
            }
        }
    }
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = 0u;
    }
};

// Fourth word of a raw (unstructured, stride 0) buffer descriptor on CDNA:
// 32-bit data format, no swizzle.
constexpr int kRawBufferWord3 = 0x00020000;

// The query operand of a tile is held as loaded (QFrag = Frag) unless the
// tile decodes it once at load time.
#define HN_SAME_Q_OPERAND                                                              \
    static constexpr int kQRegs = kFragRegs;                                           \
    typedef Frag QFrag;                                                                \
    __device__ __forceinline__ static void load_q(QFrag &f, const Elem *p) { f.load(p); } \
    __device__ __forceinline__ static void zero_q(QFrag &f) { f.zero(); }

// float32 stream of width W on 16x16x4 MFMA (4 lane groups, W/4 each).
template <int W>
struct F32Tile : Shape16 {
    typedef float Elem;
    static constexpr int kSlice = W / 4;        // elements per lane group
    static constexpr int kFragRegs = kSlice;
    typedef Regs<kFragRegs> Frag;
    HN_SAME_Q_OPERAND
    static constexpr bool kFused = true;  // the filter's flushes may rescore (psim)
    __device__ __forceinline__ static Acc mma(const Frag &x, const Frag &q) {
        Acc acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m = 0; m < kSlice; ++m)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.v[m]),
                                                       __uint_as_float(q.v[m]), acc, 0, 0, 0);
        return acc;
    }
};

// float32 stream of width W on 32x32x2 MFMA (2 lane groups, W/2 each).
template <int W>
struct F32Tile32 : Shape32 {
    typedef float Elem;
    static constexpr int kSlice = W / 2;
    static constexpr int kFragRegs = kSlice;
    typedef Regs<kFragRegs> Frag;
    HN_SAME_Q_OPERAND
    static constexpr bool kFused = true;  // the filter's flushes may rescore (psim)
    __device__ __forceinline__ static Acc mma(const Frag &x, const Frag &q) {
        Acc acc = {};
#pragma unroll
        for (int m = 0; m < kSlice; ++m)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(x.v[m]),
                                                       __uint_as_float(q.v[m]), acc, 0, 0, 0);
        return acc;
    }
};

// bfloat16 stream of width W on 16x16 MFMA: 16x16x16 for W = 16 (4 values per
// lane group), 16x16x32 steps of 8 values above.
template <int W>
struct BF16Tile : Shape16 {
    typedef uint16_t Elem;
    static constexpr int kSlice = W / 4;
    static constexpr int kFragRegs = kSlice / 2;
    typedef Regs<kFragRegs> Frag;
    HN_SAME_Q_OPERAND
    static constexpr bool kFused = true;  // the filter's flushes may rescore (psim)
    __device__ __forceinline__ static Acc mma(const Frag &x, const Frag &q) {
        Acc acc = {0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (kSlice == 4) {
            v4s a, b;
            __builtin_memcpy(&a, x.v, 8);
            __builtin_memcpy(&b, q.v, 8);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        } else {
#pragma unroll
            for (int c = 0; c < kSlice / 8; ++c) {
                v8bf a, b;
                __builtin_memcpy(&a, x.v + 4 * c, 16);
                __builtin_memcpy(&b, q.v + 4 * c, 16);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
        }
        return acc;
    }
};

// bfloat16 stream of width W on 32x32x16 MFMA (2 lane groups, W/2 values
// each, in steps of 8).
template <int W>
struct BF16Tile32 : Shape32 {
    typedef uint16_t Elem;
    static constexpr int kSlice = W / 2;
    static constexpr int kFragRegs = kSlice / 2;
    typedef Regs<kFragRegs> Frag;
    HN_SAME_Q_OPERAND
    static constexpr bool kFused = true;  // the filter's flushes may rescore (psim)
    __device__ __forceinline__ static Acc mma(const Frag &x, const Frag &q) {
        Acc acc = {};
#pragma unroll
        for (int c = 0; c < kSlice / 8; ++c) {
            v8bf a, b;
            __builtin_memcpy(&a, x.v + 4 * c, 16);
            __builtin_memcpy(&b, q.v + 4 * c, 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        return acc;
    }
};

// FP8 (OCP E4M3FN codes) stream of width W (2 lane groups, W/2 codes each).
// Every E4M3 value is exactly a bfloat16 value, so the codes are decoded in
// registers (v_cvt_scalef32_pk_bf16_fp8 with scale 1, two per instruction) and
// contracted on the 32x32x16 bf16 MFMA: the stream is half the bf16 bytes and
// the accumulation is the bf16 matrix core's.  (The native fp8 32x32x16
// instruction was measured to lose low-order product bits while summing, far
// beyond float32 rounding, which no admissible slack could cover cheaply.)
// The query operand is decoded once, at load.
template <int W>
struct FP8Tile32 : Shape32 {
    // the fp8 slack keeps many more pairs than the other precisions (for
    // K = 8, thousands per query): most items would overflow their staging
    // buffers and be re-run, so the filter flushes whenever a buffer fills
    static constexpr bool kDenseFilter = true;
    typedef uint8_t Elem;
    static constexpr int kSlice = W / 2;           // codes per lane group
    static constexpr int kFragRegs = kSlice / 4;   // entry operand: 4 codes per register
    static constexpr int kQRegs = kSlice / 2;      // query operand: 2 bf16 per register
    typedef Regs<kFragRegs> Frag;
    struct QFrag {
        uint32_t v[kQRegs];
    };
    __device__ __forceinline__ static void decode(uint32_t codes, uint32_t &lo, uint32_t &hi) {
        const v2bf a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(codes, 1.0f, false);
        const v2bf b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(codes, 1.0f, true);
        __builtin_memcpy(&lo, &a, 4);
        __builtin_memcpy(&hi, &b, 4);
    }
    __device__ __forceinline__ static void load_q(QFrag &f, const Elem *p) {
        Frag c;
        c.load(p);
#pragma unroll
        for (int i = 0; i < kFragRegs; ++i) decode(c.v[i], f.v[2 * i], f.v[2 * i + 1]);
    }
    __device__ __forceinline__ static void zero_q(QFrag &f) {
#pragma unroll
        for (int i = 0; i < kQRegs; ++i) f.v[i] = 0u;
    }
    __device__ __forceinline__ static Acc mma(const Frag &x, const QFrag &q) {
        Acc acc = {};
#pragma unroll
        for (int c = 0; c < kSlice / 8; ++c) {
            uint32_t d[4];
            decode(x.v[2 * c], d[0], d[1]);
            decode(x.v[2 * c + 1], d[2], d[3]);
            v8bf a, b;
            __builtin_memcpy(&a, d, 16);
            __builtin_memcpy(&b, q.v + 4 * c, 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        return acc;
    }
};

// INT8 fixed-point stream of width W on 32x32x16 MFMA (2 lane groups, W/2
// codes each, in steps of 8), summed exactly in int32; the sums are converted
// to float32 for the shared epilogue (exact: |sum| < 2^24).
typedef int v16i __attribute__((ext_vector_type(16)));
template <int W>
struct I8Tile32 : Shape32 {
    typedef int8_t Elem;
    static constexpr int kSlice = W / 2;
    static constexpr int kFragRegs = kSlice / 4;
    typedef Regs<kFragRegs> Frag;
    HN_SAME_Q_OPERAND
    static constexpr bool kFused = true;  // the filter's flushes may rescore (psim)
    // The filter compares these exact int32 sums with integer thresholds; the
    // other modes take them as float32 (exact: |sum| < 2^24).
    static constexpr bool kIntScores = true;
    __device__ __forceinline__ static v16i mma_i(const Frag &x, const Frag &q) {
        v16i acc = {};
#pragma unroll
        for (int c = 0; c < kSlice / 8; ++c) {
            const long a = (long)((unsigned long)x.v[2 * c] | ((unsigned long)x.v[2 * c + 1] << 32));
            const long b = (long)((unsigned long)q.v[2 * c] | ((unsigned long)q.v[2 * c + 1] << 32));
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b, acc, 0, 0, 0);
        }
        return acc;
    }
    __device__ __forceinline__ static Acc mma(const Frag &x, const Frag &q) {
        const v16i acc = mma_i(x, q);
        Acc out;
#pragma unroll
        for (int v = 0; v < 16; ++v) out[v] = (float)acc[v];
        return out;
    }
};

// Registers one tile of a configuration holds per lane (scores + query
// operand); a configuration is compiled when NQ times this stays within budget.
template <class Tile>
constexpr int tile_cost() { return Tile::kAcc + Tile::kQRegs; }
constexpr int kTileBudget = 96;

// ------------------------------------------------------------ helpers

__device__ __forceinline__ unsigned lane_prefix(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <class Acc, int N>
__device__ __forceinline__ float acc_max(const Acc &a) {
    float m = a[0];
#pragma unroll
    for (int v = 1; v < N; ++v) m = fmaxf(m, a[v]);
    return m;
}

// The same, continuing a running maximum m.
template <class Acc, int N>
__device__ __forceinline__ float acc_max_from(float m, const Acc &a) {
#pragma unroll
    for (int v = 0; v < N; ++v) m = fmaxf(m, a[v]);
    return m;
}

// The emission's groups of 4 slots (bit g: slots 4g..4g+3) in which some
// lane holds a score >= t: computed only on the rare tiles with a survivor,
// from each group's maximum (two max operations and one ballot per group),
// so that emit_pairs ballots and counts the slots of those groups alone.
// (fmaxf: the NaN scores of rows past the end never hide a passing one.)
__device__ __forceinline__ float slot_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ int slot_max(int a, int b) { return max(a, b); }
template <int N, class AccT, class T>
__device__ __forceinline__ unsigned group_mask(const AccT &a, T t) {
    unsigned groups = 0;
#pragma unroll
    for (int g = 0; g < (N + 3) / 4; ++g) {
        T x = a[4 * g];
#pragma unroll
        for (int v = 4 * g + 1; v < 4 * g + 4 && v < N; ++v) x = slot_max(x, a[v]);
        if (__ballot(x >= t)) groups |= 1u << g;
    }
    return groups;
}

// Argmax spans: the argmax mode reduces the scores of kArgSpan consecutive
// blocks into one running maximum per lane before comparing it with the
// best so far, so a winning lane group is (span, g): kArgSpan x the group's
// rows of one block.  Chunks hold whole spans (make_plan).
constexpr int kArgSpan = 4;

// Survivor staging.  In the hot loop each wave appends (query, entry) pairs to
// its own LDS buffer only, so the loop issues no global stores (which would
// make the compiler drain the loads in flight); the buffer is flushed to the
// global list with one atomic per wave at the end of the work item.  A wave
// whose buffer fills marks the item for a re-run by scan_redo_kernel, which
// flushes whenever its buffer fills (Direct); the set of pairs is the same.
#ifndef HN_EMIT_CAP
#define HN_EMIT_CAP 1024
#endif
constexpr int kEmitCap = HN_EMIT_CAP;  // pairs per wave buffer (>= 64 lanes x 4 slots)
// Wave-level filter items carry fewer than this many pairs to the wave's
// next item instead of flushing them (float32 filter -1% on 10,000 queries
// over 2^20 entries, where a wave's item holds about 50 pairs; carrying up
// to a full buffer made every wave end on a long flush, 25% slower).
constexpr int kCarryPairs = 128;
static_assert(kEmitCap >= 256, "a flush must always fit four ballots of 64 lanes");

struct EmitBuf {
    int2 *pairs;  // LDS [kEmitCap]
    float *vals;  // LDS [kEmitCap] (window mode)
    int count;    // wave-uniform
    bool full;    // wave-uniform: a pair did not fit (non-direct mode)
};

// Fused rescoring of one stored pair (filter flushes with psim set): the
// float32 re-check of a low-precision scan, then the canonical float64 sim,
// the running key of the query and the survivor count.  The batched form
// loads the pair's key, threshold and re-check prefix together and reads
// one 128-byte line of both rows per step of the float64 sum, so the pair
// waits on few dependent loads; the single-database filters take it (bf16
// 0.78 to 0.75 ms, float32 2.86 to 2.82 ms on 10,000 queries over 2^20
// entries).  The multi-database filter keeps the per-group loads, with which
// it measured 7% faster (1.22 against 1.30 ms on 64 databases).
__device__ __forceinline__ void rescore_pair_batched(const ScanArgs &A, const int2 pr,
                                                     const unsigned long long pos) {
    const float *qv = A.rs_queries + (int64_t)pr.x * kDim;
    const unsigned long long bk = A.best_key[pr.x];
    bool keep = true;
    if (A.rs_major32) {
        const float thr = A.rs_thr32[pr.x];
        const float *xm = A.rs_major32 + (int64_t)pr.y * A.rs_kp;
        float sm = 0.0f;
        for (int j0 = 0; j0 < A.rs_k; j0 += 16) {
            float4 x4[4], q4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = j0 + 4 * u < A.rs_k;
                x4[u] = ok ? *reinterpret_cast<const float4 *>(xm + j0 + 4 * u)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
                q4[u] = ok ? *reinterpret_cast<const float4 *>(qv + j0 + 4 * u)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (j0 + 4 * u < A.rs_k) {
                    sm = fmaf(q4[u].x, x4[u].x, sm);
                    sm = fmaf(q4[u].y, x4[u].y, sm);
                    sm = fmaf(q4[u].z, x4[u].z, sm);
                    sm = fmaf(q4[u].w, x4[u].w, sm);
                }
            }
        }
        keep = sm >= thr;
    }
    double sv = -INFINITY;
    if (keep) {
        sv = sim64<8>(qv, A.rs_rows + (int64_t)pr.y * kDim);
        // best_key starts at the seed's key and only grows: most
        // survivors are below it and need no atomic
        const unsigned long long kk = key_of(sv);
        if (kk > bk) atomicMax(&A.best_key[pr.x], kk);
    }
    A.psim[pos] = sv;
    if (A.cnt) atomicAdd(&A.cnt[pr.x], 1);
}

__device__ __forceinline__ void rescore_pair(const ScanArgs &A, const int2 pr,
                                             const unsigned long long pos) {
    const float *qv = A.rs_queries + (int64_t)pr.x * kDim;
    bool keep = true;
    if (A.rs_major32) {
        const float *xm = A.rs_major32 + (int64_t)pr.y * A.rs_kp;
        float sm = 0.0f;
        for (int j = 0; j < A.rs_k; j += 4) {
            const float4 x4 = *reinterpret_cast<const float4 *>(xm + j);
            const float4 q4 = *reinterpret_cast<const float4 *>(qv + j);
            sm = fmaf(q4.x, x4.x, sm);
            sm = fmaf(q4.y, x4.y, sm);
            sm = fmaf(q4.z, x4.z, sm);
            sm = fmaf(q4.w, x4.w, sm);
        }
        keep = sm >= A.rs_thr32[pr.x];
    }
    double sv = -INFINITY;
    if (keep) {
        sv = sim64(qv, A.rs_rows + (int64_t)pr.y * kDim);
        // the key only grows from the seed's: most survivors need no atomic
        const unsigned long long kk = key_of(sv);
        if (kk > A.best_key[pr.x]) atomicMax(&A.best_key[pr.x], kk);
    }
    A.psim[pos] = sv;
    if (A.cnt) atomicAdd(&A.cnt[pr.x], 1);
}

template <bool WithVal, bool Fused, bool Batch = true>
__device__ __forceinline__ void flush_pairs(const ScanArgs &A, EmitBuf &B) {
    if (B.count == 0) return;
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (__lane_id() == 0) base = atomicAdd(A.counter, (unsigned long long)B.count);
    base = __shfl(base, 0);
    for (int i = (int)__lane_id(); i < B.count; i += 64) {
        const int2 pr = B.pairs[i];
        const unsigned long long pos = base + (unsigned)i;
        if ((int64_t)pos < A.cap) {
            A.pairs[pos] = pr;
            if (WithVal) A.pair_val[pos] = B.vals[i];
            if (Fused && !WithVal && A.psim) {
                if constexpr (Batch)
                    rescore_pair_batched(A, pr, pos);
                else
                    rescore_pair(A, pr, pos);
            }
        } else {
            A.qflag[pr.x] = 1;
        }
    }
    __builtin_amdgcn_wave_barrier();
    B.count = 0;
}

// Append the lane's entries with score >= t, in groups of 4 accumulator
// slots: ballot per slot, positions by popcount + mbcnt prefix counts.  Rows
// past the database end are never appended: the scan sets their scores to
// NaN, which compares false with every threshold (-inf included).
// Padding queries never pass: the caller's threshold for them is +inf (or a
// window limit of +inf / NaN), so the slot test is one comparison, whose lane
// mask is the ballot itself.
template <class Tile, bool WithVal, bool Direct, bool Batch, class AccT, class T>
__device__ __forceinline__ void emit_pairs(const ScanArgs &A, EmitBuf &B, const AccT &a, T t,
                                           int q, int eblk, unsigned groups = ~0u) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int v0 = 0; v0 < Tile::kAcc; v0 += 4) {
        if (!((groups >> (v0 / 4)) & 1u)) continue;  // wave-uniform: no lane's group passes
        bool pv[4];
        unsigned long long mv[4];
        int c[4];
        int total = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pv[u] = a[v0 + u] >= t;
            mv[u] = __ballot(pv[u]);
            c[u] = __popcll(mv[u]);
            total += c[u];
        }
        if (total == 0) continue;
        if (B.count + total > kEmitCap) {
            if constexpr (Direct) {
                flush_pairs<WithVal, Tile::kFused, Batch>(A, B);
            } else {
                B.full = true;
                return;
            }
        }
        int off = B.count;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (pv[u]) {
                const int pos = off + (int)lane_prefix(mv[u]);
                B.pairs[pos] = make_int2(A.q_base + q, eblk + Tile::out_row(lane, v0 + u));
                if constexpr (WithVal) B.vals[pos] = a[v0 + u];
            }
            off += c[u];
        }
        B.count += total;
    }
}

// Lexicographic (value desc, index asc) merge; idx < 0 marks "none".
__device__ __forceinline__ void lex_merge(float &v, int &i, float ov, int oi) {
    if (oi >= 0 && (i < 0 || ov > v || (ov == v && oi < i))) {
        v = ov;
        i = oi;
    }
}

// ------------------------------------------------------------ the scan kernel

// One work item: query block qb x entry chunk `chunk`.  redo_id is what an
// overflowing item records for its re-run (its index in the launch's list).
// sub_block >= 0: this wave alone scans that query sub-block of the item
// (wave-level items, WQ = kWaves); else the wave's place in the work-group
// decides.
template <class Tile, int NQ, int WQ, int MODE, bool Direct, bool Batch = true, bool Carry = false>
__device__ __forceinline__ void scan_item(const ScanArgs &A, const int item, const int redo_id,
                                          float (*sh_val)[NQ * Tile::kCols],
                                          int (*sh_idx)[NQ * Tile::kCols], int *sh_full,
                                          EmitBuf &eb, const int sub_block = -1) {
    typedef typename Tile::Elem Elem;
    typedef typename Tile::Frag Frag;
    typedef typename Tile::QFrag QFrag;
    typedef typename Tile::Acc Acc;
    constexpr int R = Tile::kRows, C = Tile::kCols, G = Tile::kGroups, NA = Tile::kAcc;
    constexpr int NS = kWaves / WQ;  // waves sharing one query sub-block
    const int chunk = item / A.n_qb, qb = item % A.n_qb;
    const int wave =
        sub_block >= 0 ? sub_block : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = lane / R, r = lane % R;  // lane group (K slice) and row / column
    const int wq = wave % WQ, ws = wave / WQ;
    const int tile0 = (qb * WQ + wq) * NQ;

    const Elem *xs = reinterpret_cast<const Elem *>(A.x);
    const Elem *qsrc = reinterpret_cast<const Elem *>(A.qs);
    QFrag qf[NQ];
    int qid[NQ];
    float thr[NQ], best[NQ];
    int bblk[NQ];      // argmax: span of the best score so far
    float smax[NQ];    // argmax: running maximum of the current span
    int cur_span = -1;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        qid[t] = (tile0 + t) * C + r;
        if (qid[t] < A.q_count)
            Tile::load_q(qf[t], qsrc + (int64_t)qid[t] * A.q_stride + g * Tile::kSlice);
        else
            Tile::zero_q(qf[t]);
        // padding queries: a filter threshold of +inf, a window threshold of
        // -inf (limit best + inf): neither ever passes
        thr[t] = MODE == kFilter   ? (qid[t] < A.q_count ? A.thr[qid[t]] : INFINITY)
                 : MODE == kWindow ? (qid[t] < A.q_count ? A.thr[qid[t]] : -INFINITY)
                                   : 0.0f;
        best[t] = (MODE == kWindow && A.init_best) ? A.init_best[qid[t]] : -INFINITY;
        bblk[t] = -1;
        smax[t] = -INFINITY;
    }
    // argmax: fold the current span into the best (NaN scores of rows past
    // the end never win a comparison)
    auto close_span = [&]() {
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            if (smax[t] > best[t]) {
                best[t] = smax[t];
                bblk[t] = cur_span;
            }
            smax[t] = -INFINITY;
        }
    };

    const int blk0 = chunk * A.chunk_blocks;
    const int blk1 = min(blk0 + A.chunk_blocks, A.n_blocks);
    // The item's entry rows through one buffer descriptor based at its first
    // row and ending at its last row (or the database end): a block's load
    // is the lane's fixed byte offset plus the block's, with no per-lane
    // address arithmetic, and rows past the database end read as zeros.
    // make_plan keeps a chunk within 2^30 bytes.
    const int64_t row0 = (int64_t)blk0 * R;
    const int row_bytes = A.x_stride * (int)sizeof(Elem);
    const int64_t rows_in = min((int64_t)blk1 * R, A.n) - row0;
    const __amdgpu_buffer_rsrc_t xrsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(xs + row0 * A.x_stride), (short)0, (int)(rows_in * row_bytes), kRawBufferWord3);
    const int lane_off = r * row_bytes + g * Tile::kSlice * (int)sizeof(Elem);
    const int full_blocks = (int)(A.n / R);  // blocks with no row past the end
    // Two register groups of PF entry blocks each: while one group is being
    // computed the other one is loading.  Every slot is loaded on every step
    // (past the item's end the address is clamped to its last block), so the
    // loads in flight at any point are a fixed, whole group.
#ifndef HN_PF_WIDE
#define HN_PF_WIDE 1
#endif
    constexpr int PF = Tile::kFragRegs <= 2 ? 8 : (Tile::kFragRegs <= 4 ? 4 : HN_PF_WIDE);
    // Loads past the item's end (the last group's prefetch) fall outside the
    // descriptor's range and read zeros without touching memory; they are
    // never used.
    const int blk_step = R * row_bytes;
    auto load_group = [&](Frag (&xg)[PF], int gbase) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            // block offset in a scalar register: one vector add per load
            const int boff =
                __builtin_amdgcn_readfirstlane((gbase - blk0 + j * NS) * blk_step);
            xg[j].load_buf(xrsrc, lane_off + boff);
        }
    };
    // integer filter: the float threshold t as the least integer >= t
    // (clamped to +-2^24, beyond every exact int8 sum); padding queries
    // (t = +inf) never pass
    constexpr bool kIntFilter = MODE == kFilter && Tile::kIntScores;
    int thri[NQ];
    if constexpr (kIntFilter) {
#pragma unroll
        for (int t = 0; t < NQ; ++t)
            thri[t] = (int)fminf(fmaxf(ceilf(thr[t]), -16777216.0f), 16777216.0f);
    }
    auto compute_group = [&](const Frag (&xg)[PF], int gbase) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int blk = gbase + j * NS;
            if (blk >= blk1) break;
            if constexpr (kIntFilter) {
                v16i ai[NQ];
#pragma unroll
                for (int t = 0; t < NQ; ++t) ai[t] = Tile::mma_i(xg[j], qf[t]);
                const int eblk = blk * R;
                if (blk >= full_blocks) {
#pragma unroll
                    for (int t = 0; t < NQ; ++t)
#pragma unroll
                        for (int v = 0; v < NA; ++v)
                            if (eblk + Tile::out_row(lane, v) >= A.n) ai[t][v] = INT_MIN;
                }
                int mi[NQ];
                bool any = false;
#pragma unroll
                for (int t = 0; t < NQ; ++t) {
                    int m = ai[t][0];
#pragma unroll
                    for (int v = 1; v < NA; ++v) m = max(m, ai[t][v]);
                    mi[t] = m;
                    any = any || (m >= thri[t]);
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int t = 0; t < NQ; ++t)
                        if (__ballot(mi[t] >= thri[t]))
                            emit_pairs<Tile, false, Direct, Batch>(A, eb, ai[t], thri[t], qid[t], eblk,
                                                                   group_mask<NA>(ai[t], thri[t]));
                }
                continue;
            }
            Acc acc[NQ];
#pragma unroll
            for (int t = 0; t < NQ; ++t) acc[t] = Tile::mma(xg[j], qf[t]);
            const int eblk = blk * R;
            if (blk >= full_blocks) {
#pragma unroll
                for (int t = 0; t < NQ; ++t)
#pragma unroll
                    for (int v = 0; v < NA; ++v)
                        if (eblk + Tile::out_row(lane, v) >= A.n) acc[t][v] = __builtin_nanf("");
            }
            float mx[NQ];
            if constexpr (MODE != kArgmax) {
                // from -inf: the tree is max3 operations only (no separate
                // quieting of the first scores)
#pragma unroll
                for (int t = 0; t < NQ; ++t) mx[t] = acc_max_from<Acc, NA>(-INFINITY, acc[t]);
            }
            if constexpr (MODE == kArgmax) {
                const int sp = blk / kArgSpan;
                if (sp != cur_span) {
                    close_span();
                    cur_span = sp;
                }
#pragma unroll
                for (int t = 0; t < NQ; ++t) smax[t] = acc_max_from<Acc, NA>(smax[t], acc[t]);
            } else if constexpr (MODE == kFilter) {
                bool any = false;
#pragma unroll
                for (int t = 0; t < NQ; ++t) any = any || (mx[t] >= thr[t]);
                if (__ballot(any)) {
#pragma unroll
                    for (int t = 0; t < NQ; ++t) {
                        if (!__ballot(mx[t] >= thr[t])) continue;
                        emit_pairs<Tile, false, Direct, Batch>(A, eb, acc[t], thr[t], qid[t], eblk,
                                                               group_mask<NA>(acc[t], thr[t]));
                    }
                }
            } else if constexpr (MODE == kWindow) {
                float lim[NQ];
                bool any = false;
#pragma unroll
                for (int t = 0; t < NQ; ++t) {
                    best[t] = fmaxf(best[t], mx[t]);
                    lim[t] = best[t] - thr[t];
                    any = any || (mx[t] >= lim[t]);
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int t = 0; t < NQ; ++t)
                        if (__ballot(mx[t] >= lim[t]))
                            emit_pairs<Tile, true, Direct, Batch>(A, eb, acc[t], lim[t], qid[t],
                                                           eblk);
                }
            } else {
#pragma unroll
                for (int t = 0; t < NQ; ++t) {
                    if (qid[t] < A.q_count) {
#pragma unroll
                        for (int v = 0; v < NA; ++v) {
                            const int e = eblk + Tile::out_row(lane, v);
                            if (e < A.n) A.scores[(int64_t)qid[t] * A.n + e] = acc[t][v];
                        }
                    }
                }
            }
        }
    };
    constexpr int kStep = PF * NS;  // blocks per group for this wave
    // The scheduling barriers keep each group's loads ahead of the other
    // group's compute, so they have a whole compute phase to land.  A wave
    // whose query tiles are all padding (a small batch in a large query
    // block) skips the scan: its scores could never pass or be used, and the
    // SIMD goes to the other waves.  The test is uniform in the wave.
    Frag xa[PF], xb[PF];
    const bool live = tile0 * C < A.q_count;
    if (live) load_group(xa, blk0 + ws);
    for (int base = blk0 + ws; live && base < blk1; base += 2 * kStep) {
        load_group(xb, base + kStep);
        __builtin_amdgcn_sched_barrier(0);
        compute_group(xa, base);
        __builtin_amdgcn_sched_barrier(0);
        if (base + kStep >= blk1) break;
        load_group(xa, base + 2 * kStep);
        __builtin_amdgcn_sched_barrier(0);
        compute_group(xb, base + kStep);
        __builtin_amdgcn_sched_barrier(0);
    }

    if constexpr (MODE == kFilter || MODE == kWindow) {
        if constexpr (Direct) {
            // a wave that runs item after item (Carry) keeps fewer than
            // kCarryPairs pairs for its next item's flush, so that a flush
            // fills its lanes; it flushes the rest after its last item
            if (!Carry || eb.count >= kCarryPairs)
                flush_pairs<MODE == kWindow, Tile::kFused, Batch>(A, eb);
        } else {
            // flush only if no wave of the item overflowed; else re-run it.
            // The decision is made uniform explicitly: a branch the compiler
            // took as divergent would structure the item loop (which holds
            // barriers) as a divergent loop.
            if (lane == 0) sh_full[wave] = eb.full ? 1 : 0;
            __syncthreads();
            const bool redo =
                __builtin_amdgcn_readfirstlane(sh_full[0] | sh_full[1] | sh_full[2] | sh_full[3]) != 0;
            if (!redo) {
                flush_pairs<MODE == kWindow, Tile::kFused, Batch>(A, eb);
            } else if (threadIdx.x == 0) {
                A.redo[atomicAdd(A.redo_count, 1u)] = redo_id;
            }
            eb.count = 0;
            eb.full = false;
        }
    }

    if constexpr (MODE == kArgmax) close_span();
    if constexpr (MODE == kArgmax || MODE == kWindow) {
        // per query: merge the lane groups, then the NS waves of the sub-block.
        // The argmax index is the winning lane group, span * G + g.
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            float v = best[t];
            int i = (MODE == kArgmax) ? (bblk[t] >= 0 ? bblk[t] * G + g : -1)
                                      : (v > -INFINITY ? 0 : -1);
#pragma unroll
            for (int o = R; o < 64; o <<= 1) {
                float ov = __shfl_xor(v, o);
                int oi = __shfl_xor(i, o);
                lex_merge(v, i, ov, oi);
            }
            if (g == 0) {
                sh_val[wave][t * C + r] = v;
                sh_idx[wave][t * C + r] = i;
            }
        }
        __syncthreads();
        if (ws == 0 && g == 0) {
#pragma unroll
            for (int t = 0; t < NQ; ++t) {
                float v = sh_val[wave][t * C + r];
                int i = sh_idx[wave][t * C + r];
                for (int s = 1; s < NS; ++s)
                    lex_merge(v, i, sh_val[wave + s * WQ][t * C + r],
                              sh_idx[wave + s * WQ][t * C + r]);
                const int q = qid[t];
                if (q < A.q_pad) {
                    A.part_val[(int64_t)chunk * A.q_pad + q] = v;
                    if (MODE == kArgmax) A.part_idx[(int64_t)chunk * A.q_pad + q] = i;
                }
            }
        }
    }
}

#define HN_SCAN_SHARED(Tile, NQ, MODE)                                                    \
    __shared__ float sh_val[kWaves][NQ * Tile::kCols];                                    \
    __shared__ int sh_idx[kWaves][NQ * Tile::kCols];                                      \
    __shared__ int sh_full[kWaves];                                                       \
    constexpr bool kEmits = MODE == kFilter || MODE == kWindow;                           \
    __shared__ int2 sh_pairs[kEmits ? kWaves : 1][kEmits ? kEmitCap : 1];                 \
    __shared__ float sh_pval[MODE == kWindow ? kWaves : 1][MODE == kWindow ? kEmitCap : 1]; \
    EmitBuf eb;                                                                           \
    eb.pairs = sh_pairs[kEmits ? (threadIdx.x >> 6) : 0];                                 \
    eb.vals = sh_pval[MODE == kWindow ? (threadIdx.x >> 6) : 0];                          \
    eb.count = 0;                                                                         \
    eb.full = false;

// Persistent scan with a static, XCD-ranged item assignment: the items are
// split into 8 contiguous ranges, one per XCD (blockIdx % 8), and the
// work-groups of an XCD take their range round-robin, so at any time they work
// on neighbouring items, which share entry chunks (see make_plan) in that XCD's
// L2.  The item loop depends only on blockIdx and gridDim: it is uniform, so
// the barriers inside scan_item are reached by every wave the same number of
// times.
// Optional occupancy request for the scan kernels (waves per SIMD).
#ifdef HN_WAVES_PER_EU
#define HN_SCAN_ATTR __attribute__((amdgpu_waves_per_eu(HN_WAVES_PER_EU)))
#else
#define HN_SCAN_ATTR
#endif

template <class Tile, int NQ, int WQ, int MODE>
__global__ __launch_bounds__(256) HN_SCAN_ATTR void scan_kernel(ScanArgs A) {
    HN_SCAN_SHARED(Tile, NQ, MODE)
    // The single-pass window keeps a few percent of the entries, more than a
    // wave's staging buffer holds for nearly every item: it flushes whenever
    // the buffer fills (direct mode) instead of re-running the items that
    // overflowed.  The two-pass filter's survivors are sparse: it flushes once
    // per item and re-runs the rare overflowing item, except with a tile
    // whose slack keeps dense survivors (kDenseFilter).
    constexpr bool kDirect = MODE == kWindow || (MODE == kFilter && Tile::kDenseFilter);
    const int groups_per_xcd = (int)gridDim.x / kXcds;
    const int x = (int)(blockIdx.x % kXcds), w = (int)(blockIdx.x / kXcds);
    const int per = (A.n_items + kXcds - 1) / kXcds;
    const int lo = x * per, hi = min(A.n_items, lo + per);
    if constexpr (MODE == kFilter && WQ == kWaves && !Tile::kIntScores) {
        if (A.item_ctr) {
            // Wave-level items: with one query sub-block per wave the four
            // waves of a work-group share nothing but the entry chunk, so
            // each wave claims (item, sub-block) pairs alone, one atomic
            // each, and flushes whenever its staging buffer fills (and after
            // an item that leaves kCarryPairs pairs or more, the rest after
            // its last item).  No wave waits at a barrier for another one's
            // survivors.  The counters
            // count sub-block items, kWaves per item, in the same per-XCD
            // ranges as the items.  (Measured with 10,000 queries on 2^20
            // entries: +3% float32 and bf16; the int8 filter, whose integer
            // emission does not take the inline flushes well, ran at half
            // speed and keeps work-group items.)
            const int nw = A.n_items * kWaves;
            const int wper = (nw + kXcds - 1) / kXcds;
            const int wlo = x * wper, whi = min(nw, wlo + wper);
            auto claim_sub = [&]() {
                unsigned v = 0;
                if (__lane_id() == 0) v = atomicAdd(A.item_ctr + x, 1u);
                return wlo + (int)__builtin_amdgcn_readfirstlane(v);
            };
            for (int wi = claim_sub(); wi < whi; wi = claim_sub())
                scan_item<Tile, NQ, WQ, MODE, true, true, true>(A, wi / kWaves, wi / kWaves, sh_val,
                                                                sh_idx, sh_full, eb, wi % kWaves);
            flush_pairs<false, Tile::kFused>(A, eb);
            return;
        }
    }
    if (A.item_ctr) {
        // Dynamic order: the XCD's groups take its items in list order from
        // a counter, so items whose survivors cost more (queries with weak
        // lower bounds) do not pile up on the groups a static stride would
        // give them to.  Thread 0 claims the next item and shares it through
        // LDS; the claim is the loop's condition (before the first item and
        // after each), which the compiler keeps uniform, so every wave
        // reaches the barriers inside the loop the same number of times (a
        // claim at the head of the loop body made it structure the loop as
        // divergent).
        __shared__ int sh_item;
        auto claim = [&]() {
            if (threadIdx.x == 0) sh_item = lo + (int)atomicAdd(A.item_ctr + x, 1u);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(sh_item);
            __syncthreads();
            return it;
        };
        for (int item = claim(); item < hi; item = claim())
            scan_item<Tile, NQ, WQ, MODE, kDirect>(A, item, item, sh_val, sh_idx, sh_full, eb);
        return;
    }
    for (int item = lo + w; item < hi; item += groups_per_xcd)
        scan_item<Tile, NQ, WQ, MODE, kDirect>(A, item, item, sh_val, sh_idx, sh_full, eb);
}

// Re-runs the items whose survivor buffers overflowed, flushing as it goes.
template <class Tile, int NQ, int WQ, int MODE>
__global__ __launch_bounds__(256) void scan_redo_kernel(ScanArgs A) {
    HN_SCAN_SHARED(Tile, NQ, MODE)
    const unsigned n = __builtin_amdgcn_readfirstlane(*A.redo_count);
    for (unsigned r = blockIdx.x; r < n; r += gridDim.x) {
        const int item = __builtin_amdgcn_readfirstlane(A.redo[r]);
        scan_item<Tile, NQ, WQ, MODE, true>(A, item, item, sh_val, sh_idx, sh_full, eb);
    }
}

// Several databases in one launch: items[i] = (database, its local item);
// every database has its own arguments (same tile and configuration).  The
// list is ordered database by database, chunk-major inside each, and split
// into 8 XCD ranges as in scan_kernel.  Overflowing items record their list
// index in the redo list every database of the launch shares.
template <class Tile, int NQ, int WQ, int MODE>
__global__ __launch_bounds__(256) void scan_multi_kernel(const ScanArgs *__restrict__ dbs,
                                                         const int2 *__restrict__ items,
                                                         int n_items, unsigned *item_ctr) {
    HN_SCAN_SHARED(Tile, NQ, MODE)
    const int groups_per_xcd = (int)gridDim.x / kXcds;
    const int x = (int)(blockIdx.x % kXcds), w = (int)(blockIdx.x / kXcds);
    const int per = (n_items + kXcds - 1) / kXcds;
    const int lo = x * per, hi = min(n_items, lo + per);
    constexpr bool kDirect = MODE == kFilter && Tile::kDenseFilter;  // as in scan_kernel
    auto run = [&](int item) {
        const int2 it = items[item];
        const int d = __builtin_amdgcn_readfirstlane(it.x);
        const int local = __builtin_amdgcn_readfirstlane(it.y);
        const ScanArgs A = dbs[d];
        scan_item<Tile, NQ, WQ, MODE, kDirect, false>(A, local, item, sh_val, sh_idx, sh_full, eb);
    };
    if (item_ctr) {
        // device work queue: items of databases of very different sizes and
        // query counts are claimed in list order per XCD (as in scan_kernel)
        __shared__ int sh_item;
        auto claim = [&]() {
            if (threadIdx.x == 0) sh_item = lo + (int)atomicAdd(item_ctr + x, 1u);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(sh_item);
            __syncthreads();
            return it;
        };
        for (int item = claim(); item < hi; item = claim()) run(item);
        return;
    }
    for (int item = lo + w; item < hi; item += groups_per_xcd) run(item);
}

template <class Tile, int NQ, int WQ, int MODE>
__global__ __launch_bounds__(256) void scan_multi_redo_kernel(const ScanArgs *__restrict__ dbs,
                                                              const int2 *__restrict__ items,
                                                              const int *__restrict__ redo,
                                                              const unsigned *redo_count) {
    HN_SCAN_SHARED(Tile, NQ, MODE)
    const unsigned n = __builtin_amdgcn_readfirstlane(*redo_count);
    for (unsigned r = blockIdx.x; r < n; r += gridDim.x) {
        const int item = __builtin_amdgcn_readfirstlane(redo[r]);
        const int2 it = items[item];
        const int d = __builtin_amdgcn_readfirstlane(it.x);
        const int local = __builtin_amdgcn_readfirstlane(it.y);
        const ScanArgs A = dbs[d];
        scan_item<Tile, NQ, WQ, MODE, true, false>(A, local, item, sh_val, sh_idx, sh_full, eb);
    }
}

// ------------------------------------------------------------ host side

// Shape of a launch: query tiles per wave (NQ) x query sub-blocks per group
// (WQ), tile width C, entries per block R.
struct Plan {
    int nq = 4, wq = 4, cols = 16, rows = 16;
    int qb_size() const { return nq * wq * cols; }
    int32_t n_qb = 0, n_blocks = 0, chunk_blocks = 0, n_chunks = 0, n_items = 0;
    int64_t q_pad = 0;
};

// Configurations compiled for each tile: (NQ, WQ).
constexpr int kNumCfg = 6;
constexpr int kCfgNQ[kNumCfg] = {1, 2, 4, 2, 4, 8};
constexpr int kCfgWQ[kNumCfg] = {1, 1, 1, 4, 4, 4};

// Smallest configuration whose query block covers q (largest if none),
// within the register budget.  forced_nq > 0 restricts NQ to the largest
// compiled value not above it.  -1 if none fits.
inline int pick_cfg(int64_t q, int cols, int cost, int forced_nq) {
    if (forced_nq > 0) {
        int nq = 0;
        for (int c = 0; c < kNumCfg; ++c)
            if (kCfgNQ[c] * cost <= kTileBudget && kCfgNQ[c] <= forced_nq && kCfgNQ[c] > nq)
                nq = kCfgNQ[c];
        forced_nq = nq;
        if (nq == 0) return -1;
    }
    // Unforced, the 32x32 shape keeps at most 2 tiles per wave: its 16
    // scores per tile make larger NQ cost occupancy (measured: NQ = 2 beats 4).
    const int auto_cap = cols == 32 ? 2 : 8;
    int best = -1;
    for (int c = 0; c < kNumCfg; ++c) {
        if (kCfgNQ[c] * cost > kTileBudget) continue;
        if (forced_nq > 0 && kCfgNQ[c] != forced_nq) continue;
        if (forced_nq <= 0 && kCfgNQ[c] > auto_cap) continue;
        best = c;
        if ((int64_t)kCfgNQ[c] * kCfgWQ[c] * cols >= q) break;
    }
    return best;
}

// Entry chunks: chunk_blocks if given, else about target_items items.  With
// `slots` (the launch's resident work-groups, a multiple of 8) the chunk count
// is chosen so the items fill whole rounds of the persistent grid: n_items <=
// rounds * slots, so no work-group runs a round more than the others (the
// XCD ranges hold at most rounds * slots / 8 items each).  min_chunks raises
// the chunk count where a caller needs that many partials per query.
inline Plan make_plan(int64_t n, int64_t q, int cfg, int chunk_blocks, int rows, int cols,
                      int64_t target_items = 8192, int64_t slots = 0, int64_t min_chunks = 1) {
    Plan p;
    p.nq = kCfgNQ[cfg];
    p.wq = kCfgWQ[cfg];
    p.rows = rows;
    p.cols = cols;
    const int64_t qb = p.qb_size();
    p.n_qb = (int32_t)((q + qb - 1) / qb);
    p.q_pad = (int64_t)p.n_qb * qb;
    p.n_blocks = (int32_t)((n + rows - 1) / rows);
    if (chunk_blocks <= 0) {
        // chunks of at least 32 blocks (a work item's fixed costs, its query
        // tiles and its flush, then stay small against its scan), unless that
        // leaves fewer than 256 items; never below 8 blocks
        const int64_t max_chunks = std::max<int64_t>(
            1, std::max<int64_t>(p.n_blocks / 32, std::min<int64_t>(p.n_blocks / 8, 256)));
        int64_t want;
        if (slots >= kXcds) {
            const int64_t rounds = std::max<int64_t>(1, (target_items + slots / 2) / slots);
            want = std::max<int64_t>(1, rounds * slots / p.n_qb);
        } else {
            want = std::max<int64_t>(1, (target_items + p.n_qb - 1) / p.n_qb);
        }
        want = std::min(std::max(want, min_chunks), max_chunks);
        chunk_blocks = (int32_t)((p.n_blocks + want - 1) / want);
    }
    // a chunk is addressed through one buffer descriptor with 32-bit offsets:
    // at most 2^30 bytes for rows of up to 128 float32 values, which leaves
    // room for the prefetch past its end
    const int32_t max_chunk =
        (int32_t)(((int64_t)1 << 30) / ((int64_t)rows * 512)) / kArgSpan * kArgSpan;
    // whole argmax spans per chunk, so a winning lane group lies in one chunk
    chunk_blocks = (chunk_blocks + kArgSpan - 1) / kArgSpan * kArgSpan;
    chunk_blocks = std::min(chunk_blocks, max_chunk);
    p.chunk_blocks = std::min<int32_t>(chunk_blocks, p.n_blocks);
    p.n_chunks = (p.n_blocks + p.chunk_blocks - 1) / p.chunk_blocks;
    p.n_items = p.n_qb * p.n_chunks;
    return p;
}

inline int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

// Persistent grid: every resident work-group slot once, at most one per item
// of the largest XCD range (rounded to whole XCD rounds).  The occupancy is
// the launched kernel's own (single- or multi-database scan); only that
// kernel is instantiated, so each scan kernel lives in one translation unit.
template <class Tile, int NQ, int WQ, int MODE, bool Multi = false>
inline unsigned persistent_grid(int n_items) {
    static const int per_cu = [] {
        const void *kernel;
        if constexpr (Multi)
            kernel = reinterpret_cast<const void *>(&scan_multi_kernel<Tile, NQ, WQ, MODE>);
        else
            kernel = reinterpret_cast<const void *>(&scan_kernel<Tile, NQ, WQ, MODE>);
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, 256, 0) != hipSuccess) {
            (void)hipGetLastError();
            b = 1;
        }
        return b < 1 ? 1 : b;
    }();
    int64_t g = (int64_t)cu_count() * per_cu;
    const int64_t need = ((int64_t)n_items + kXcds - 1) / kXcds * kXcds;  // 8 x range size
    g = std::min(g, need);
    g = (g + kXcds - 1) / kXcds * kXcds;
    return (unsigned)std::max<int64_t>(g, kXcds);
}

template <class Tile, int MODE, int C>
inline void launch_one(const Plan &p, const ScanArgs &A, hipStream_t s) {
    if constexpr (kCfgNQ[C] * tile_cost<Tile>() <= kTileBudget) {
        hipLaunchKernelGGL((scan_kernel<Tile, kCfgNQ[C], kCfgWQ[C], MODE>),
                           dim3(persistent_grid<Tile, kCfgNQ[C], kCfgWQ[C], MODE>(p.n_items)),
                           dim3(256), 0, s, A);
        if constexpr (MODE == kFilter || MODE == kWindow)
            hipLaunchKernelGGL((scan_redo_kernel<Tile, kCfgNQ[C], kCfgWQ[C], MODE>),
                               dim3(persistent_grid<Tile, kCfgNQ[C], kCfgWQ[C], MODE>(p.n_items)),
                               dim3(256), 0, s, A);
    }
}

template <class Tile, int MODE>
inline void launch_cfgs(int cfg, const Plan &p, const ScanArgs &A, hipStream_t s) {
    switch (cfg) {
        case 0: launch_one<Tile, MODE, 0>(p, A, s); break;
        case 1: launch_one<Tile, MODE, 1>(p, A, s); break;
        case 2: launch_one<Tile, MODE, 2>(p, A, s); break;
        case 3: launch_one<Tile, MODE, 3>(p, A, s); break;
        case 4: launch_one<Tile, MODE, 4>(p, A, s); break;
        case 5: launch_one<Tile, MODE, 5>(p, A, s); break;
    }
}

// Instantiated modes: argmax and filter for every tile and configuration;
// store (the score buffer) for configuration 0; the window mode (the
// single-pass forms and the exhaustive scan) where the tile family asks for it.
// Returns nonzero if the requested combination is not compiled.
template <class Tile, bool Window>
inline int launch_tile(int mode, int cfg, const Plan &p, const ScanArgs &A, hipStream_t s) {
    if (cfg < 0 || cfg >= kNumCfg || kCfgNQ[cfg] * tile_cost<Tile>() > kTileBudget) return 1;
    switch (mode) {
        case kArgmax: launch_cfgs<Tile, kArgmax>(cfg, p, A, s); return 0;
        case kFilter: launch_cfgs<Tile, kFilter>(cfg, p, A, s); return 0;
        case kStore:
            if (cfg != 0) return 1;
            launch_one<Tile, kStore, 0>(p, A, s);
            return 0;
        case kWindow:
            if constexpr (Window) {
                launch_cfgs<Tile, kWindow>(cfg, p, A, s);
                return 0;
            }
            return 1;
    }
    return 1;
}

// Resident work-groups of the kernel a launch_tile call with the same mode and
// configuration would start (its persistent grid for an unbounded item count);
// 0 if not compiled.
template <class Tile, int MODE, int C>
inline unsigned slots_one() {
    if constexpr (kCfgNQ[C] * tile_cost<Tile>() <= kTileBudget)
        return persistent_grid<Tile, kCfgNQ[C], kCfgWQ[C], MODE>(1 << 30);
    return 0;
}
template <class Tile, int MODE>
inline unsigned slots_cfgs(int cfg) {
    switch (cfg) {
        case 0: return slots_one<Tile, MODE, 0>();
        case 1: return slots_one<Tile, MODE, 1>();
        case 2: return slots_one<Tile, MODE, 2>();
        case 3: return slots_one<Tile, MODE, 3>();
        case 4: return slots_one<Tile, MODE, 4>();
        case 5: return slots_one<Tile, MODE, 5>();
    }
    return 0;
}
template <class Tile, bool Window>
inline unsigned tile_slots(int mode, int cfg) {
    if (cfg < 0 || cfg >= kNumCfg) return 0;
    switch (mode) {
        case kArgmax: return slots_cfgs<Tile, kArgmax>(cfg);
        case kFilter: return slots_cfgs<Tile, kFilter>(cfg);
        case kWindow:
            if constexpr (Window) return slots_cfgs<Tile, kWindow>(cfg);
            return 0;
    }
    return 0;
}

// Several databases in one launch (argmax and filter modes).  The grid is
// sized by the occupancy of the single-database kernel of the same tile.
// item_ctr: kXcds item counters, zero before the launch (NULL: static order).
template <class Tile, int MODE, int C>
inline void launch_multi_one(const ScanArgs *dbs, const int2 *items, int n_items,
                             const int *redo, const unsigned *redo_count, unsigned *item_ctr,
                             hipStream_t s) {
    if constexpr (kCfgNQ[C] * tile_cost<Tile>() <= kTileBudget) {
        hipLaunchKernelGGL((scan_multi_kernel<Tile, kCfgNQ[C], kCfgWQ[C], MODE>),
                           dim3(persistent_grid<Tile, kCfgNQ[C], kCfgWQ[C], MODE, true>(n_items)),
                           dim3(256), 0, s, dbs, items, n_items, item_ctr);
        if constexpr (MODE == kFilter)
            hipLaunchKernelGGL((scan_multi_redo_kernel<Tile, kCfgNQ[C], kCfgWQ[C], MODE>),
                               dim3(persistent_grid<Tile, kCfgNQ[C], kCfgWQ[C], MODE, true>(n_items)),
                               dim3(256), 0, s, dbs, items, redo, redo_count);
    }
}

template <class Tile>
inline int launch_tile_multi(int mode, int cfg, const ScanArgs *dbs, const int2 *items,
                             int n_items, const int *redo, const unsigned *redo_count,
                             unsigned *item_ctr, hipStream_t s) {
    if (cfg < 0 || cfg >= kNumCfg || kCfgNQ[cfg] * tile_cost<Tile>() > kTileBudget) return 1;
    if (mode != kArgmax && mode != kFilter) return 1;
#define HN_MULTI_CASE(C)                                                   \
    case C:                                                                \
        if (mode == kArgmax)                                                           \
            launch_multi_one<Tile, kArgmax, C>(dbs, items, n_items, redo, redo_count,   \
                                               item_ctr, s);                            \
        else                                                                           \
            launch_multi_one<Tile, kFilter, C>(dbs, items, n_items, redo, redo_count,   \
                                               item_ctr, s);                            \
        return 0;
    switch (cfg) {
        HN_MULTI_CASE(0)
        HN_MULTI_CASE(1)
        HN_MULTI_CASE(2)
        HN_MULTI_CASE(3)
        HN_MULTI_CASE(4)
        HN_MULTI_CASE(5)
    }
#undef HN_MULTI_CASE
    return 1;
}

// Tile families: for each precision, a stream of width W up to 32 runs on the
// 32x32 shape, wider streams on the 16x16 shape (fp8 streams are 16 or 32).  cost = tile_cost<Tile>().
struct TileInfo {
    int rows, cols, cost, groups;
};
inline TileInfo tile_info(int precision, int w) {
    if (precision == HN_PREC_FP8) return TileInfo{32, 32, 16 + w / 4, 2};
    if (precision == HN_PREC_INT8) return TileInfo{32, 32, 16 + w / 8, 2};
    if (precision == HN_PREC_FP32) {
        if (w <= 32) return TileInfo{32, 32, 16 + w / 2, 2};
        return TileInfo{16, 16, 4 + w / 4, 4};
    }
    if (w <= 32) return TileInfo{32, 32, 16 + w / 4, 2};
    return TileInfo{16, 16, 4 + w / 8, 4};
}

// Per-precision launchers, each compiled in its own translation unit.
int launch_scan_f32_narrow(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                           hipStream_t s);  // widths 4, 8, 16, 32 (32x32 tiles)
int launch_scan_f32_wide(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                         hipStream_t s);    // widths 64, 128 (16x16 tiles)
int launch_scan_bf16(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                     hipStream_t s);        // widths 16, 32 (32x32), 64, 128 (16x16)
int launch_scan_fp8(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                    hipStream_t s);         // widths 16, 32 (32x32)
int launch_scan_int8(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                     hipStream_t s);        // widths 16, 32 (32x32)
// Resident work-groups of the scan kernel of (mode, width, configuration), 0
// if not compiled: one function per launcher above.
unsigned slots_scan_f32_narrow(int mode, int w, int cfg);
unsigned slots_scan_f32_wide(int mode, int w, int cfg);
unsigned slots_scan_bf16(int mode, int w, int cfg);
unsigned slots_scan_fp8(int mode, int w, int cfg);
unsigned slots_scan_int8(int mode, int w, int cfg);
// Several databases of one stream width in one launch: float32 widths 8, 16,
// 32; bf16 and fp8 widths 16, 32.  Nonzero if not compiled.
int launch_scan_multi(int precision, int mode, int w, int cfg, const ScanArgs *dbs,
                      const int2 *items, int n_items, const int *redo,
                      const unsigned *redo_count, unsigned *item_ctr, hipStream_t s);
#define HN_MULTI_DECL(name)                                                                    \
    int launch_scan_multi_##name(int mode, int w, int cfg, const ScanArgs *dbs,             \
                                 const int2 *items, int n_items, const int *redo,          \
                                 const unsigned *redo_count, unsigned *item_ctr,           \
                                 hipStream_t s);
HN_MULTI_DECL(f32)   // widths 8, 16, 32
HN_MULTI_DECL(bf16)  // widths 16, 32
HN_MULTI_DECL(fp8)   // widths 16, 32
HN_MULTI_DECL(i8)    // widths 16, 32
#undef HN_MULTI_DECL

}  // namespace hn
