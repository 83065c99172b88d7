/*
 * hnsearch: exact top-1 inner-product search over hierarchically normalised
 * (HN) vectors on AMD Instinct MI355X (gfx950).
 *
 * The method (Sections 3.1-3.3 of "Exact and Deterministic Patch Descriptor
 * Retrieval via Hierarchical Normalization"): every D = 128 vector carries a
 * K-dim major prefix of norm sqrt(1-alpha) and a (D-K)-dim minor part of norm
 * sqrt(alpha) (Eq. 1).  By Eq. 2 and Cauchy-Schwarz (Eq. 3) the full inner
 * product is at most dot_K + alpha, so after one major-prefix scan only the
 * entries whose bound reaches a known similarity need the full product
 * (Algorithm 1).  The result equals exhaustive search (Theorem 1) and is
 * deterministic (Theorem 2).
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are device memory owned by the caller; they must
 *    stay valid until the work enqueued on `stream` has completed.  Host
 *    pointers are read or written before the call returns.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously unless stated otherwise.
 *  - Every function returns HN_OK (0) or a negative hn_status and never
 *    throws.  On error no output is written and hn_last_error() returns a
 *    message for the calling thread.
 *  - Arrays of 128-value float32 rows (databases, queries, HN-layer inputs
 *    and outputs) are read and written with 16-byte accesses: their base
 *    pointers must be 16-byte aligned, else HN_ERR_INVALID_ARG.
 *  - Indices are 0-based int64 positions in the database as given to the
 *    build; ties in similarity go to the smallest index.
 *  - Similarities are the canonical float64 sim: acc = 0; for j = 0..127:
 *    acc += (double)q[j] * (double)x[j], ascending j, round-to-nearest.
 */
#ifndef HNSEARCH_H
#define HNSEARCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hn_index hn_index; /* opaque; owns its device copies */

typedef enum {
    HN_OK = 0,
    HN_ERR_INVALID_ARG = -1,  /* bad size, pointer or option */
    HN_ERR_NOT_NORMALIZED = -2, /* a row violates the HN block norms (Eq. 1) */
    HN_ERR_OOM = -3,          /* device allocation failed */
    HN_ERR_DEVICE = -4,       /* a HIP call failed */
    HN_ERR_UNSUPPORTED = -5   /* valid but not implemented (e.g. n >= 2^31) */
} hn_status;

/* Scan precision of the major-prefix pass.  FP32 scans the float32 prefix;
 * BF16 scans round-to-nearest-even bfloat16 copies of both operands; FP8
 * scans OCP E4M3FN copies (round to nearest even) of x[:k] / s_x and
 * q[:k] / s_q, with power-of-two scales s_x (one per index, from max |x[:k]|)
 * and s_q (one per query), and is available for k <= 32.  INT8 (k <= 32)
 * scans fixed-point codes round(x[:k] / s_x) and round(q[:k] / s_q) in
 * [-127, 127] with power-of-two scales, summed exactly in int32.  All keep
 * the search exact: the bound slack covers the rounding (bf16, fp8, int8: by
 * the measured residual norms of the copies), and the low-precision survivors
 * pass a float32 re-check before float64 rescoring. */
enum { HN_PREC_FP32 = 0, HN_PREC_BF16 = 1, HN_PREC_FP8 = 2, HN_PREC_INT8 = 3 };

/* How each query's initial lower bound L_q is found (Algorithm 1 step 2).
 *   PLAIN    two scans: the argmax scan gives the seed b (largest scan score),
 *            L_q = sim(q, x_b); the filter scan keeps s~ >= T_q.
 *   LEARNED  one scan: L_q from the index's seed model (hn_set_seed_model), the
 *            best canonical sim among the anchors of the model's 4 largest
 *            outputs; the scan keeps s~ >= max(T_q, m - w_q), m the running
 *            scan maximum of its work item and w_q = 2 (alpha + eps_q): the
 *            entry scoring m has sim >= m - alpha - eps_q, so anything below
 *            the window cannot beat it.  Survivors are re-filtered against the
 *            final maximum, then rescored.
 *   WINDOW   one scan with the window only (L_q = -inf): the comparison form
 *            without a seed. */
enum { HN_SEED_PLAIN = 0, HN_SEED_LEARNED = 1, HN_SEED_WINDOW = 2 };

/* Precision of the plain seed's argmax scan (Algorithm 1 step 1).  Any entry
 * whose scan score is near-maximal is an admissible seed (its canonical sim
 * is the bound), so the argmax scan may run on the bf16 copy whatever the
 * filter's precision: BF16 (the default) contracts four times faster than
 * FP32 on the matrix cores; FP32 runs the argmax on the float32 prefix, the
 * all-float32 form of the search.  The result is the same either way. */
enum { HN_SEED_SCAN_BF16 = 0, HN_SEED_SCAN_FP32 = 1 };

/* The seed model: an MLP 128 -> 256 -> 256 -> 512 with exact GELU
 * (x Phi(x)) after the two hidden layers, bf16 weights, float32 biases,
 * float32 accumulation, one output per anchor entry.  Its parameters are one
 * float32 vector of HN_MLP_PARAMS values: W1 [256][128], b1 [256],
 * W2 [256][256], b2 [256], W3 [512][256], b3 [512], weights row-major
 * (output-major).  Forward passes round the weights to bf16 (nearest even). */
enum { HN_MLP_IN = 128, HN_MLP_H = 256, HN_MLP_OUT = 512, HN_MLP_PARAMS = 230400 };

/* Build flags (any other bit: HN_ERR_INVALID_ARG).  Every build makes the
 * float32 prefix stream, the BF16 copy and, for k <= 32, the FP8 and INT8
 * copies (4, 2, 1 and 1 bytes per prefix element) beside the float32 rows. */
enum {
    HN_BUILD_NO_VALIDATE = 1u << 0 /* skip the block-norm check (bounds stay
                                      rigorous: they use measured norms) */
};

typedef struct {
    int32_t precision;    /* HN_PREC_*; FP32 by default */
    int32_t seed;         /* HN_SEED_*; plain by default */
    int32_t query_tiles;  /* MFMA query tiles per wave (16 or 32 queries each,
                             by K and precision); 0 = a fixed heuristic of q,
                             K and precision (the smallest query block that
                             covers q, within the register budget); values the
                             build does not compile fall to the largest
                             smaller one */
    int32_t chunk_blocks; /* entry blocks (16 or 32 entries) per work item;
                             0 = a fixed heuristic (whole rounds of the
                             persistent grid, about 8192 items) */
    int64_t survivor_cap; /* capacity of the survivor list in (query, entry)
                             pairs; 0 = automatic.  Queries whose survivors
                             do not fit are finished exactly by a second
                             pass (see hn_search_top1). */
    double beta;          /* < 0: exact search (bound alpha).  0 <= beta <
                             alpha: soft mode of Section 7, which replaces
                             alpha by beta in the skip test and is no longer
                             exact. */
    int32_t seed_scan;    /* HN_SEED_SCAN_*: precision of the plain seed's
                             argmax scan; BF16 (0) by default */
} hn_search_opts;

/* Optional per-query device outputs (any member may be NULL). */
typedef struct {
    int64_t *seed_idx;  /* seed entry b (plain seed)                        */
    double *seed_sim;   /* L_q: the seed's canonical sim (initial bound)    */
    float *threshold;   /* T_q: survivor test on the scan is s~ >= T_q (FP8:
                           in scan units, T_q / (s_q s_x))                 */
    int32_t *survivors; /* entries that passed the first-pass filter        */
    double *slack;      /* eps_q: rounding slack used for the bound         */
} hn_search_aux;

/* Host-side totals of one call (filled after the call synchronises). */
typedef struct {
    int64_t survivors;        /* sum over queries of first-pass survivors  */
    int64_t overflow_queries; /* queries finished by the exact fallback    */
} hn_search_stats;

/*
 * Build an index over n HN-normalised vectors (Eq. 1, Section 3.1).
 *   db     device, float32 [n][d] row-major (d must be 128).  Copied; the
 *          caller may free it once the call returns (the call synchronises).
 *   k      major prefix length, 1 <= k <= 127.
 *   alpha  minor energy, 0 <= alpha < 1.
 *   flags  HN_BUILD_* bits.
 *   out    receives the index; release it with hn_free_index.
 * Validation: every row must satisfy | ||x[:k]|| - sqrt(1-alpha) | <=
 * 2^-13 sqrt(1-alpha) and | ||x[k:]|| - sqrt(alpha) | <= 2^-13 sqrt(alpha)
 * (alpha = 0: ||x[k:]|| <= 2^-20), with finite entries, else
 * HN_ERR_NOT_NORMALIZED.  Exactness does not depend on this tolerance: the
 * bound slack uses the measured block-norm maxima.
 */
int hn_build_index(const float *db, int64_t n, int32_t d, int32_t k, double alpha,
                   uint32_t flags, void *stream, hn_index **out);

void hn_free_index(hn_index *ix);

/* Index properties (host outputs, any may be NULL).  norms[3] receives the
 * rigorous upper bounds {max ||x[:k]||, max ||x[k:]||, max ||x||}. */
int hn_index_info(const hn_index *ix, int64_t *n, int32_t *k, double *alpha,
                  double *norms);

/*
 * Exact top-1 for q queries (Algorithm 1, Section 3.3, as a GPU pipeline):
 * a major-prefix scan finds each query's seed b (largest scan score, smallest
 * index on ties); its canonical sim L_q is the initial bound; a second scan
 * keeps the entries with s~ >= T_q = round_down_f32(L_q - alpha - eps_q),
 * where eps_q covers the scan's rounding, the float32 storage of the norms
 * and the float64 evaluation (Eq. 3 made admissible in floating point); the
 * survivors are rescored in float64 and reduced by the key (sim desc, index
 * asc).
 *   queries  device, float32 [q][128]; q >= 0 (q = 0 is a no-op).
 *   out_idx  device, int64 [q];  out_sim  device, double [q].
 *   opts     NULL = defaults.  aux, stats: NULL allowed; a non-NULL stats
 *            makes the call synchronise `stream`.  The survivor list holds
 *            max(4096, n / 256) pairs per query by default (at least 2^20, at
 *            most 2^28 in all).  With the plain seed on the FP32 and BF16
 *            scans the call never synchronises: queries whose survivors
 *            overflow the list are finished by an exhaustive float64 pass
 *            (slow when many do: raise survivor_cap for such data).  The fp8
 *            and int8 scans and the single-pass seeds keep many more pairs:
 *            they synchronise once per query batch and search their
 *            overflowing queries again by a float32 filter pass seeded with
 *            the best candidate each reached, with a list sized from the
 *            first pass's pair count (the plain seed) or the default rule.
 * A query with a non-finite component gets idx -1 and sim NaN.
 */
int hn_search_top1(const hn_index *ix, const float *queries, int64_t q, int64_t *out_idx,
                   double *out_sim, const hn_search_opts *opts, const hn_search_aux *aux,
                   hn_search_stats *stats, void *stream);

/*
 * The search of hn_search_top1 for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, with every scratch buffer
 * carved from one statically allocated device array of
 * HN_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds
 * until the process ends.  The call allocates and frees nothing and never
 * synchronises.
 *   opts   the plain seed with precision FP32 or BF16 (others:
 *          HN_ERR_UNSUPPORTED); survivor_cap 0 sizes the pair list to what the
 *          array leaves after the per-query buffers (queries whose survivors
 *          do not fit are finished exactly by the exhaustive float64 pass);
 *          a survivor_cap beyond that is HN_ERR_INVALID_ARG.
 *   aux    as for hn_search_top1; there are no stats.
 * The per-query buffers grow with q and with n / 16 (argmax partials): a call
 * whose buffers besides a minimal pair list of 65,536 pairs exceed the array
 * returns HN_ERR_INVALID_ARG and enqueues nothing; split the queries.  At
 * n = 2^20 and K = 16, q = 10,000 fits.  The index's device must be current.
 * Every call on one GPU uses the same array: calls that overlap in time on one
 * GPU (on different streams, or from several threads) race and give wrong
 * results; serialise them.
 */
#define HN_NOALLOC_SCRATCH_BYTES (64ll << 20)
int hn_search_top1_noalloc(const hn_index *ix, const float *queries, int64_t q,
                           int64_t *out_idx, double *out_sim, const hn_search_opts *opts,
                           const hn_search_aux *aux, void *stream);

/*
 * Exact top-k (k = topk) per query: the topk entries of largest canonical
 * sim, ordered by (sim desc, index asc) — Algorithm 1 with the running best
 * replaced by the topk-th best.  The seed bound L is the topk-th best sim
 * among the winning lane groups of the best scan chunks (distinct real
 * entries, so L is at most the true topk-th best); every entry with
 * s~ >= round_down_f32(L - alpha - eps_q) is rescored in float64 and the
 * topk best are selected per query.  Synchronises `stream` once (and runs the
 * filter again with a list large enough if the survivors did not fit).
 *   topk     1 <= topk <= 128.
 *   out_idx  device int64 [q][topk]; out_sim device double [q][topk].  Places
 *            beyond the database size get index -1 and sim -inf; a query
 *            with a non-finite component gets -1 and NaN throughout.
 *   opts     precision, launch shape, survivor_cap (initial), beta; the seed
 *            must be HN_SEED_PLAIN.
 */
int hn_search_topk(const hn_index *ix, const float *queries, int64_t q, int32_t topk,
                   int64_t *out_idx, double *out_sim, const hn_search_opts *opts, void *stream);

/*
 * The survivor set of the bound test for given lower bounds (Algorithm 1's
 * skip test against a fixed s_best, Eq. 3):
 *   { (q, i) : s~(q, i) >= round_down_f32(L[q] - alpha - eps_q) }.
 *   lower    device, double [q]: L per query.
 *   pairs    device, int32 [cap][2]: (query, entry) pairs, unordered.
 *   count    host, receives the total number of survivors (may exceed cap;
 *            only the first cap are written).  The call synchronises.
 *   slack    device, double [q] or NULL: receives eps_q.
 */
int hn_filter_survivors(const hn_index *ix, const float *queries, int64_t q,
                        const double *lower, int32_t *pairs, int64_t cap, int64_t *count,
                        double *slack, const hn_search_opts *opts, void *stream);

/*
 * Phase 1 of Algorithm 1 with its score buffer: the scan scores
 * s~(q, i) = dot_K(q, x_i) (Eq. 2) as the search kernels compute them, for
 * every query and entry.
 *   precision  HN_PREC_FP32, HN_PREC_BF16, HN_PREC_FP8 or HN_PREC_INT8 (the
 *              last two k <= 32, else HN_ERR_UNSUPPORTED); FP8 and INT8
 *              scores are returned rescaled by s_q s_x (exact: powers of two).
 *   scores     device, float32 [q][n] row-major.
 */
int hn_scan_scores(const hn_index *ix, const float *queries, int64_t q, int32_t precision,
                   float *scores, void *stream);

/*
 * Exhaustive GPU top-1 over raw vectors (the paper's brute-force 128-dim
 * baseline, Section 6.2): a float32 scan of all n x 128 products with the
 * running maximum, then float64 rescoring of every candidate within the
 * float32 error band of the maximum, so the result is exact.
 *   db       device, float32 [n][d] (d = 128), any values (finite).
 *   queries  device, float32 [q][d].
 *   out_idx, out_sim  device [q].
 */
int hn_bruteforce_top1(const float *db, int64_t n, int32_t d, const float *queries,
                       int64_t q, int64_t *out_idx, double *out_sim, void *stream);

/*
 * Kernel timing for measurement.  Between hn_profile_begin(stream) and
 * hn_profile_end(stream, ...) every kernel this library enqueues on `stream`
 * is bracketed by HIP events (enqueued asynchronously, no synchronisation).
 * hn_profile_end synchronises `stream`, sums the elapsed times per kernel
 * name and ends the session.
 *   names   host, receives up to `max` pointers to static kernel names.
 *   ms      host double [max]: total milliseconds per kernel name.
 *   counts  host int64 [max]: launches per kernel name.
 *   n_out   host, receives the number of distinct kernel names.
 */
int hn_profile_begin(void *stream);
int hn_profile_end(void *stream, const char **names, double *ms, int64_t *counts, int32_t max,
                   int32_t *n_out);

/* ---------------------------------------------------------------- seed model
 * Not part of the paper: the learned-seed form of the search.  Anchors are
 * chosen by k-means++ D^2 seeding, a query's label is the anchor closest to
 * its exact nearest neighbour, and the MLP is trained with softmax
 * cross-entropy and AdamW.  All pointers are device memory. */

typedef struct {
    double lr, beta1, beta2, eps, weight_decay; /* AdamW, decoupled decay:
        w -= lr (m^ / (sqrt(v^) + eps) + weight_decay w) */
} hn_adamw_opts;

/* logits [b][512] = MLP(x [b][128]) for the float32 parameter vector
 * `params` (weights rounded to bf16).  0 <= b <= 2^24. */
int hn_mlp_forward(const float *params, const float *x, int64_t b, float *logits, void *stream);

/* Gradient of the mean softmax cross-entropy of MLP(x) against labels
 * (int32 [b], each in [0, 512); another value makes the loss NaN) with
 * respect to the parameters: grads [HN_MLP_PARAMS] in the parameter layout,
 * loss: one float.  The forward rounds the weights to bf16; the gradient is
 * taken through that forward (straight through to the float32 weights).
 * 1 <= b <= 2^20. */
int hn_mlp_grad(const float *params, const float *x, const int32_t *labels, int64_t b,
                float *grads, float *loss, void *stream);

/* One AdamW step on n parameters with step count t >= 1 (bias corrections
 * 1 / (1 - beta^t)); m and v are the moment buffers (zero at t = 1). */
int hn_mlp_adamw(float *params, const float *grads, float *m, float *v, int64_t n, int32_t t,
                 const hn_adamw_opts *opts, void *stream);

/* Train in place: `epochs` passes over (x [n][128], labels [n]) in order, in
 * batches of `batch` (the last one ragged), one AdamW step per batch with
 * fresh moments.  losses: NULL or float [epochs * ceil(n / batch)], the mean
 * loss of every step. */
int hn_seed_train(float *params, const float *x, const int32_t *labels, int64_t n,
                  int32_t batch, int32_t epochs, const hn_adamw_opts *opts, float *losses,
                  void *stream);

/* k-means++ D^2 seeding over the index rows (no Lloyd iterations):
 * anchors[0] = floor(u[0] n) (n - 1 if that is n); for t >= 1, with
 * D(x) = min over chosen anchors a of 2 - 2 sim(a, x) and integer weights
 * w(x) = floor(max(0, D(x)) 2^30), anchors[t] is the first entry whose
 * running weight sum exceeds floor(u[t] * total) (n - 1 if none).
 *   u        double [n_anchor], uniform draws in [0, 1) (the caller's random
 *            numbers).
 *   anchors  int64 [n_anchor].  Exact integer arithmetic: deterministic. */
int hn_kmeanspp(const hn_index *ix, int32_t n_anchor, const double *u, int64_t *anchors,
                void *stream);

/* Training labels: labels[i] = the a in [0, n_anchor) maximising
 * sim(x_nn(i), x_anchors[a]) (ties to the smaller a), where nn(i) is query
 * i's exact top-1 (hn_search_top1); -1 for a query with a non-finite
 * component.  Anchors are checked to be entries (synchronises). */
int hn_seed_labels(const hn_index *ix, const int64_t *anchors, int32_t n_anchor,
                   const float *queries, int64_t q, int32_t *labels, void *stream);

/* Install a seed model in the index for HN_SEED_LEARNED: the parameters are
 * copied (weights rounded to bf16), anchors int64 [n_anchor] with n_anchor =
 * HN_MLP_OUT, each an entry of the index.  Replaces an earlier model;
 * synchronises `stream`. */
int hn_set_seed_model(hn_index *ix, const float *params, const int64_t *anchors,
                      int32_t n_anchor, void *stream);

/* ---------------------------------------------------------------- HN layer
 * Eq. 1 (Section 3.1) as a batched layer and its vector-Jacobian product:
 * the step that places embeddings on the split sphere before they are
 * indexed.  Rows are float32 [b][128]; block norms in float64; every output
 * rounded once to float32. */

/* out[r] = ( sqrt(1-alpha) f[r,:k] / ||f[r,:k]||, sqrt(alpha) f[r,k:] /
 * ||f[r,k:]|| ); at alpha = 0 the minor block is 0.  A block that cannot be
 * normalised (zero, or a non-finite component in the row) comes out 0 and
 * status[r] (int32 [b], may be NULL) says why: 0 ok, 1 zero major block,
 * 2 zero minor block with alpha > 0, 3 non-finite component. */
int hn_layer_forward(const float *f, int64_t b, int32_t d, int32_t k, double alpha, float *out,
                     int32_t *status, void *stream);

/* grad[r] = (dL/dout[r]) . d out[r] / d f[r] given g = dL/dout: per block of
 * norm scale c, (c / ||u||) (g - v (v . g)) with u the block of f and
 * v = u / ||u||; 0 for blocks that cannot be normalised and for one-element
 * blocks (whose output is the constant +-c). */
int hn_layer_backward(const float *f, const float *g, int64_t b, int32_t d, int32_t k,
                      double alpha, float *grad, void *stream);

/* ---------------------------------------------------------- many databases
 * Ragged query batches against many indexes in one search: every scan is a
 * single persistent launch over the work items of all databases of one stream
 * width (bf16 and fp8: one launch for all k <= 16), the per-query kernels look
 * up their database, and results are exactly those of hn_search_top1 on each
 * index.  A plan owns all buffers and tables: hn_multi_search allocates
 * nothing and never synchronises, and with use_graph it replays a HIP graph
 * captured on the first call (captured again when a pointer changes). */
typedef struct hn_multi_plan hn_multi_plan; /* opaque */

/* Plan a search of q_counts[d] queries (host int64 [n_db], >= 0) against
 * ixs[d] (each k <= 32, all on the current device) with the given options
 * (precision, query_tiles, chunk_blocks, survivor_cap, beta; the seed must be
 * HN_SEED_PLAIN, else HN_ERR_UNSUPPORTED; a plan runs its argmax scan in its
 * own precision and ignores seed_scan).  Synchronises.  The indexes must
 * outlive the plan. */
int hn_multi_plan_create(const hn_index *const *ixs, int32_t n_db, const int64_t *q_counts,
                         const hn_search_opts *opts, hn_multi_plan **out);

/* Run a plan: queries device float32 [sum q_counts][128] (16-byte aligned),
 * database by database in order; out_idx int64 and out_sim double [sum
 * q_counts] in the same order (indices into each query's own database).
 * use_graph != 0: launch the plan's captured graph on `stream`. */
int hn_multi_search(hn_multi_plan *plan, const float *queries, int64_t *out_idx,
                    double *out_sim, int32_t use_graph, void *stream);

/* Plan facts (host outputs, any may be NULL): total queries, scan work items
 * (both scan passes together), scan launches per search. */
int hn_multi_plan_info(const hn_multi_plan *plan, int64_t *total_queries, int64_t *work_items,
                       int32_t *scan_launches);

/* Per-batch latency of the plan's last search, from device timestamps taken
 * inside it (the constant-rate clock, 100 MHz on MI355X): ms[d] (host, n_db
 * values) is the time from the start of the search's first kernel to the
 * last write of database d's results; 0 for a database without queries.
 * Every batch's results are written by the search's last kernel, so the
 * values sit close to the whole search's time.  Synchronises `stream` (the
 * stream the search ran on). */
int hn_multi_batch_times(const hn_multi_plan *plan, double *ms, void *stream);

void hn_multi_plan_free(hn_multi_plan *plan);

/* ------------------------------------------------------------ device memory
 * Not part of the paper: the library's own device allocations (index copies,
 * seed models, per-stream scratch arenas, multi-database plans) counted
 * against an optional budget, for processes that share a GPU and for tests of
 * the out-of-memory paths.  Scratch arenas are kept per (device, stream) and
 * grow on demand; two host threads must not enqueue on the same stream at
 * once, since their calls would share one arena. */

/* Cap the bytes the library holds at once in device allocations: a request
 * that would exceed it fails with HN_ERR_OOM, as a full device does, and the
 * failing call releases what it had taken.  max_bytes = 0 removes the cap
 * (the default); max_bytes < 0 is HN_ERR_INVALID_ARG.  Holdings above a new
 * cap are not released. */
int hn_set_memory_budget(int64_t max_bytes);

/* Bytes the library holds now in device allocations (all devices). */
int64_t hn_memory_held(void);

/* Release the scratch arenas kept for `stream` on the current device, after
 * synchronising it.  Later calls on that stream allocate them again. */
int hn_release_scratch(void *stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *hn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HNSEARCH_H */
