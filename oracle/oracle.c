/*
 * CPU FP64 oracle for hierarchical-normalisation (HN) exact top-1 search.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library and includes none of its files.
 *
 * Everything here is plain and sequential per query: no blocking, no fusion,
 * no reordering of a sum.  Queries are split across POSIX threads in
 * contiguous static ranges; every query is computed by one thread from start
 * to finish, so results do not depend on the thread count (Theorem 2,
 * Section 3.3).
 *
 * Definitions followed:
 *  - sim(q, x): the full inner product of Eq. 2 (Section 3.2), evaluated as
 *    the canonical float64 sum  acc = 0; for j = 0..D-1: acc += (double)q_j *
 *    (double)x_j  in ascending j with round-to-nearest.  Each float32 x
 *    float32 product is exact in float64, so a fused or unfused multiply-add
 *    gives the same bits; only the order of the additions matters.
 *  - top-1: the smallest index among the entries whose sim is maximal
 *    ("ties by index", Algorithm 1 step 1 and Theorem 2).
 *  - dot_K(q, x): the major-prefix product of Eq. 2, the same canonical sum
 *    over j < K.
 *  - Branch and bound: Algorithm 1 (Section 3.3) in float64 with the
 *    lexicographic (sim desc, index asc) key and the admissible bound of
 *    Eq. 3 widened by a rounding slack (see or_bnb_top1).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_U64 (1.0 / 9007199254740992.0) /* 2^-53, float64 unit roundoff */

/* Higham's gamma_n(u) = n u / (1 - n u). */
static double or_gamma(int n, double u) { return (double)n * u / (1.0 - (double)n * u); }

double or_sim(const float *q, const float *x, int d) {
    double acc = 0.0;
    for (int j = 0; j < d; ++j) acc = acc + (double)q[j] * (double)x[j];
    return acc;
}

double or_dot_prefix(const float *q, const float *x, int k) { return or_sim(q, x, k); }

/* Euclidean norm of v[lo:hi) in float64 (sequential sum of squares). */
double or_norm(const float *v, int lo, int hi) {
    double acc = 0.0;
    for (int j = lo; j < hi; ++j) acc = acc + (double)v[j] * (double)v[j];
    return sqrt(acc);
}

/* Largest block norms over the database: out[0] = max ||x[:k]||,
 * out[1] = max ||x[k:]||, out[2] = max ||x||. */
void or_db_max_norms(const float *db, int64_t n, int d, int k, double *out) {
    double mM = 0.0, mm = 0.0, mf = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const float *x = db + i * (int64_t)d;
        double a = or_norm(x, 0, k), b = or_norm(x, k, d), c = or_norm(x, 0, d);
        if (a > mM) mM = a;
        if (b > mm) mm = b;
        if (c > mf) mf = c;
    }
    out[0] = mM;
    out[1] = mm;
    out[2] = mf;
}

/* ---------------------------------------------------------------- threads */

typedef void (*or_query_fn)(void *ctx, int64_t qi);

struct or_range {
    or_query_fn fn;
    void *ctx;
    int64_t lo, hi;
};

static void *or_range_main(void *p) {
    struct or_range *r = (struct or_range *)p;
    for (int64_t qi = r->lo; qi < r->hi; ++qi) r->fn(r->ctx, qi);
    return NULL;
}

static void or_parallel_queries(int64_t nq, int nthreads, or_query_fn fn, void *ctx) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > nq) nthreads = nq > 0 ? (int)nq : 1;
    struct or_range rs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) {
        rs[t].fn = fn;
        rs[t].ctx = ctx;
        rs[t].lo = nq * t / nthreads;
        rs[t].hi = nq * (t + 1) / nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, or_range_main, &rs[t]);
    or_range_main(&rs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------ brute force */

struct or_bf_ctx {
    const float *db, *qs;
    int64_t n;
    int d;
    int64_t *out_idx;
    double *out_sim;
};

static void or_bf_one(void *p, int64_t qi) {
    struct or_bf_ctx *c = (struct or_bf_ctx *)p;
    const float *q = c->qs + qi * (int64_t)c->d;
    int64_t best = -1;
    double bs = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
        double s = or_sim(q, c->db + i * (int64_t)c->d, c->d);
        if (best < 0 || s > bs) { /* strict: the earlier (smaller) index keeps a tie */
            bs = s;
            best = i;
        }
    }
    c->out_idx[qi] = best;
    c->out_sim[qi] = bs;
}

/* Exhaustive top-1 under the canonical sim, ties to the smallest index. */
void or_bruteforce_top1(const float *db, int64_t n, int d, const float *qs, int64_t nq,
                        int nthreads, int64_t *out_idx, double *out_sim) {
    struct or_bf_ctx c = {db, qs, n, d, out_idx, out_sim};
    or_parallel_queries(nq, nthreads, or_bf_one, &c);
}

/* --------------------------------------------------------- branch & bound */

struct or_bnb_ctx {
    const float *db, *qs;
    int64_t n;
    int d, k;
    double alpha, beta;
    double muM, mum, mu; /* database block-norm maxima */
    int64_t *out_idx, *out_seed_idx, *out_phase2;
    double *out_sim, *out_seed_sim, *out_slack;
};

/* Rounding slack for the float64 bound test of one query: with the bound of
 * Eq. 3 written as s_i + alpha, the gap between it and the float64 canonical
 * sim of entry i is covered by
 *   max(0, ||q_m|| mu_m - alpha)        Cauchy-Schwarz with the stored norms
 * + gamma_K(2^-53)   ||q_M|| mu_M       float64 evaluation of dot_K
 * + gamma_D(2^-53)   ||q||   mu         float64 evaluation of the full sim
 * + 2^-48                               evaluation of the test itself. */
double or_bnb_slack(const float *q, int d, int k, double alpha, double muM, double mum,
                    double mu) {
    double nM = or_norm(q, 0, k), nm = or_norm(q, k, d), nf = or_norm(q, 0, d);
    double e = nm * mum - alpha;
    if (e < 0.0) e = 0.0;
    e += or_gamma(k, OR_U64) * nM * muM * 1.0000001;
    e += or_gamma(d, OR_U64) * nf * mu * 1.0000001;
    e += ldexp(1.0, -48);
    return e;
}

static void or_bnb_one(void *p, int64_t qi) {
    struct or_bnb_ctx *c = (struct or_bnb_ctx *)p;
    const int d = c->d, k = c->k;
    const float *q = c->qs + qi * (int64_t)d;
    const int64_t n = c->n;
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    /* Phase 1: store every major score; seed b = first index of the maximum. */
    int64_t b = 0;
    for (int64_t i = 0; i < n; ++i) {
        s[i] = or_dot_prefix(q, c->db + i * (int64_t)d, k);
        if (s[i] > s[b]) b = i;
    }
    /* Seed: one full evaluation. */
    double best = or_sim(q, c->db + b * (int64_t)d, d);
    int64_t bi = b;
    c->out_seed_idx[qi] = b;
    c->out_seed_sim[qi] = best;
    double slack = or_bnb_slack(q, d, k, c->alpha, c->muM, c->mum, c->mu);
    c->out_slack[qi] = slack;
    /* Phase 2: index order; skip only when the widened bound is strictly
     * below the running best, so an entry that could tie is evaluated. */
    int64_t evaluated = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == b) continue;
        if (s[i] + c->beta + slack < best) continue;
        ++evaluated;
        double v = or_sim(q, c->db + i * (int64_t)d, d);
        if (v > best || (v == best && i < bi)) {
            best = v;
            bi = i;
        }
    }
    free(s);
    c->out_idx[qi] = bi;
    c->out_sim[qi] = best;
    c->out_phase2[qi] = evaluated;
}

/* Algorithm 1 per query.  beta < 0 means beta = alpha (exact).  Outputs:
 * top-1 index and sim, the seed b and sim(q, x_b), the number of entries
 * Phase 2 evaluated in full (Algorithm 1's Phase2% numerator) and the slack
 * used.  db_norms = {mu_M, mu_m, mu} from or_db_max_norms. */
void or_bnb_top1(const float *db, int64_t n, int d, int k, double alpha, double beta,
                 const double *db_norms, const float *qs, int64_t nq, int nthreads,
                 int64_t *out_idx, double *out_sim, int64_t *out_seed_idx,
                 double *out_seed_sim, int64_t *out_phase2, double *out_slack) {
    struct or_bnb_ctx c;
    c.db = db;
    c.qs = qs;
    c.n = n;
    c.d = d;
    c.k = k;
    c.alpha = alpha;
    c.beta = beta < 0.0 ? alpha : beta;
    c.muM = db_norms[0];
    c.mum = db_norms[1];
    c.mu = db_norms[2];
    c.out_idx = out_idx;
    c.out_sim = out_sim;
    c.out_seed_idx = out_seed_idx;
    c.out_seed_sim = out_seed_sim;
    c.out_phase2 = out_phase2;
    c.out_slack = out_slack;
    or_parallel_queries(nq, nthreads, or_bnb_one, &c);
}

/* ------------------------------------------------------- survivor sets */

struct or_surv_ctx {
    const float *db, *qs;
    int64_t n;
    int d, k;
    double alpha;
    const double *lo; /* per query: count entries with s_i + alpha >= lo[q] */
    const double *hi; /* per query: count entries with s_i + alpha >= hi[q] */
    int64_t *cnt_lo, *cnt_hi;
};

static void or_surv_one(void *p, int64_t qi) {
    struct or_surv_ctx *c = (struct or_surv_ctx *)p;
    const float *q = c->qs + qi * (int64_t)c->d;
    int64_t a = 0, b = 0;
    for (int64_t i = 0; i < c->n; ++i) {
        double v = or_dot_prefix(q, c->db + i * (int64_t)c->d, c->k) + c->alpha;
        if (v >= c->lo[qi]) ++a;
        if (v >= c->hi[qi]) ++b;
    }
    c->cnt_lo[qi] = a;
    c->cnt_hi[qi] = b;
}

/* Sizes of the seed-threshold survivor sets S(q, L) = {i : dot_K + alpha >= L}
 * at two levels per query (float64 dot_K). */
void or_survivor_counts(const float *db, int64_t n, int d, int k, double alpha,
                        const float *qs, int64_t nq, const double *lo, const double *hi,
                        int nthreads, int64_t *cnt_lo, int64_t *cnt_hi) {
    struct or_surv_ctx c = {db, qs, n, d, k, alpha, lo, hi, cnt_lo, cnt_hi};
    or_parallel_queries(nq, nthreads, or_surv_one, &c);
}

/* Indices of S(q, L) for one query, ascending; returns the set size (writes
 * at most cap indices). */
int64_t or_survivor_list(const float *db, int64_t n, int d, int k, double alpha,
                         const float *q, double L, int64_t *out, int64_t cap) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        double v = or_dot_prefix(q, db + i * (int64_t)d, k) + alpha;
        if (v >= L) {
            if (m < cap) out[m] = i;
            ++m;
        }
    }
    return m;
}

/* ----------------------------------------------------------------- top-k */

struct or_topk_ctx {
    const float *db, *qs;
    int64_t n;
    int d, kk;
    int64_t *out_idx;
    double *out_sim;
};

static void or_topk_one(void *p, int64_t qi) {
    struct or_topk_ctx *c = (struct or_topk_ctx *)p;
    const float *q = c->qs + qi * (int64_t)c->d;
    int64_t *I = c->out_idx + qi * (int64_t)c->kk;
    double *S = c->out_sim + qi * (int64_t)c->kk;
    int m = 0;
    for (int64_t i = 0; i < c->n; ++i) {
        double v = or_sim(q, c->db + i * (int64_t)c->d, c->d);
        /* insertion into a list kept in (sim desc, index asc) order; a later
         * index never displaces an equal sim */
        int pos = m;
        while (pos > 0 && v > S[pos - 1]) --pos;
        if (pos >= c->kk) continue;
        int last = m < c->kk ? m : c->kk - 1;
        for (int t = last; t > pos; --t) {
            S[t] = S[t - 1];
            I[t] = I[t - 1];
        }
        S[pos] = v;
        I[pos] = i;
        if (m < c->kk) ++m;
    }
    for (int t = m; t < c->kk; ++t) {
        S[t] = -INFINITY;
        I[t] = -1;
    }
}

/* Exhaustive top-k (k = kk) under the canonical sim, ordered by (sim desc,
 * index asc). */
void or_topk(const float *db, int64_t n, int d, const float *qs, int64_t nq, int kk,
             int nthreads, int64_t *out_idx, double *out_sim) {
    struct or_topk_ctx c = {db, qs, n, d, kk, out_idx, out_sim};
    or_parallel_queries(nq, nthreads, or_topk_one, &c);
}

/* ------------------------------------------------------ anchor selection */

/* k-means++ (D^2) seeding on the database, no Lloyd steps, so that anchors are
 * real entries.  D_i is the smallest distance 2 - 2 sim(a, x_i) over the
 * anchors chosen so far (squared Euclidean distance between unit vectors).
 * The draw u[t] in [0, 1) picks an entry by inverse CDF over the weights.
 * Weights are quantised to integers w_i = floor(max(0, D_i) * 2^30) so that
 * the cumulative sums are exact and independent of summation order; entry i
 * is chosen when prefix(i-1) <= floor(u * total) < prefix(i).  The first pick
 * is floor(u[0] * n).  A chosen entry keeps only its float32 storage
 * residue as weight (about 1e-7 of a typical one). */
void or_kmeanspp(const float *db, int64_t n, int d, int n_anchor, const double *u,
                 int64_t *out) {
    double *dist = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t first = (int64_t)floor(u[0] * (double)n);
    if (first >= n) first = n - 1;
    out[0] = first;
    for (int64_t i = 0; i < n; ++i) dist[i] = INFINITY;
    for (int t = 1; t <= n_anchor; ++t) {
        const float *a = db + out[t - 1] * (int64_t)d;
        uint64_t total = 0;
        for (int64_t i = 0; i < n; ++i) {
            double v = 2.0 - 2.0 * or_sim(a, db + i * (int64_t)d, d);
            if (v < dist[i]) dist[i] = v;
            double w = dist[i] > 0.0 ? dist[i] : 0.0;
            total += (uint64_t)floor(ldexp(w, 30));
        }
        if (t == n_anchor) break;
        uint64_t target = (uint64_t)floor(u[t] * (double)total);
        uint64_t run = 0;
        int64_t pick = n - 1;
        for (int64_t i = 0; i < n; ++i) {
            double w = dist[i] > 0.0 ? dist[i] : 0.0;
            run += (uint64_t)floor(ldexp(w, 30));
            if (run > target) {
                pick = i;
                break;
            }
        }
        out[t] = pick;
    }
    free(dist);
}
