/*
 * Drives every entry point of the CPU oracle (oracle/oracle.c) once on small
 * seeded HN-like inputs so that the test suite can build both into one
 * executable with AddressSanitizer and UndefinedBehaviorSanitizer.  It checks
 * a few facts the paper fixes (B&B equals brute force, Theorem 1; top-k's
 * first column is the top-1; survivor counts match the survivor lists), but
 * its purpose is the sanitizer run: any out-of-bounds access, leak, use after
 * free or undefined operation in the oracle ends it with a report and a
 * non-zero status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double or_sim(const float *q, const float *x, int d);
double or_norm(const float *v, int lo, int hi);
void or_db_max_norms(const float *db, int64_t n, int d, int k, double *out);
void or_bruteforce_top1(const float *db, int64_t n, int d, const float *qs, int64_t nq,
                        int nthreads, int64_t *out_idx, double *out_sim);
double or_bnb_slack(const float *q, int d, int k, double alpha, double muM, double mum,
                    double mu);
void or_bnb_top1(const float *db, int64_t n, int d, int k, double alpha, double beta,
                 const double *db_norms, const float *qs, int64_t nq, int nthreads,
                 int64_t *out_idx, double *out_sim, int64_t *out_seed_idx,
                 double *out_seed_sim, int64_t *out_phase2, double *out_slack);
void or_survivor_counts(const float *db, int64_t n, int d, int k, double alpha,
                        const float *qs, int64_t nq, const double *lo, const double *hi,
                        int nthreads, int64_t *cnt_lo, int64_t *cnt_hi);
int64_t or_survivor_list(const float *db, int64_t n, int d, int k, double alpha,
                         const float *q, double L, int64_t *out, int64_t cap);
void or_topk(const float *db, int64_t n, int d, const float *qs, int64_t nq, int kk,
             int nthreads, int64_t *out_idx, double *out_sim);
void or_kmeanspp(const float *db, int64_t n, int d, int n_anchor, const double *u,
                 int64_t *out);

/* xorshift64* with a Box-Muller normal: only an input generator */
static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double uniform01(void) {
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}
static double normal(void) {
    double u = uniform01(), v = uniform01();
    if (u < 1e-300) u = 1e-300;
    return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

/* rows scaled block-wise to norms sqrt(1 - alpha) and sqrt(alpha) */
static void hn_rows(float *out, int64_t n, int d, int k, double alpha) {
    for (int64_t i = 0; i < n; ++i) {
        double v[128], a = 0, b = 0;
        for (int j = 0; j < d; ++j) v[j] = normal();
        for (int j = 0; j < k; ++j) a += v[j] * v[j];
        for (int j = k; j < d; ++j) b += v[j] * v[j];
        for (int j = 0; j < d; ++j)
            out[i * d + j] = (float)(j < k ? v[j] * sqrt((1 - alpha) / a)
                                           : (alpha > 0 ? v[j] * sqrt(alpha / b) : 0.0));
    }
}

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

int main(void) {
    const int d = 128, k = 16, nq = 23, kk = 5, na = 7;
    const int64_t n = 701;
    const double alpha = 0.125;
    float *db = malloc(sizeof(float) * n * d), *qs = malloc(sizeof(float) * nq * d);
    hn_rows(db, n, d, k, alpha);
    for (int q = 0; q < nq; ++q) /* perturbed copies of entries */
        for (int j = 0; j < d; ++j) qs[q * d + j] = db[(q * 31 % n) * d + j] + 0.01f * (float)normal();
    for (int j = 0; j < d; ++j) db[(n - 1) * d + j] = db[j]; /* an exact duplicate: a tie */

    double norms[3];
    or_db_max_norms(db, n, d, k, norms);
    CHECK(fabs(norms[0] - sqrt(1 - alpha)) < 1e-5 && fabs(norms[1] - sqrt(alpha)) < 1e-5);
    CHECK(fabs(or_norm(db, 0, d) - 1.0) < 1e-5);

    int64_t *bi = malloc(sizeof(int64_t) * nq), *ri = malloc(sizeof(int64_t) * nq);
    double *bs = malloc(sizeof(double) * nq), *rs = malloc(sizeof(double) * nq);
    int64_t *seed = malloc(sizeof(int64_t) * nq), *p2 = malloc(sizeof(int64_t) * nq);
    double *ss = malloc(sizeof(double) * nq), *sl = malloc(sizeof(double) * nq);
    or_bruteforce_top1(db, n, d, qs, nq, 3, bi, bs);
    for (int threads = 1; threads <= 4; threads += 3) {
        or_bnb_top1(db, n, d, k, alpha, -1.0, norms, qs, nq, threads, ri, rs, seed, ss, p2, sl);
        for (int q = 0; q < nq; ++q) CHECK(ri[q] == bi[q] && rs[q] == bs[q]);
    }
    or_bnb_top1(db, n, d, k, alpha, 0.25 * alpha, norms, qs, nq, 2, ri, rs, seed, ss, p2, sl);
    for (int q = 0; q < nq; ++q) CHECK(rs[q] <= bs[q] && rs[q] >= ss[q]);
    CHECK(or_bnb_slack(qs, d, k, alpha, norms[0], norms[1], norms[2]) > 0.0);

    double *lo = malloc(sizeof(double) * nq), *hi = malloc(sizeof(double) * nq);
    int64_t *clo = malloc(sizeof(int64_t) * nq), *chi = malloc(sizeof(int64_t) * nq);
    for (int q = 0; q < nq; ++q) {
        lo[q] = bs[q] - 0.3;
        hi[q] = bs[q];
    }
    or_survivor_counts(db, n, d, k, alpha, qs, nq, lo, hi, 3, clo, chi);
    int64_t *list = malloc(sizeof(int64_t) * n);
    for (int q = 0; q < nq; ++q) {
        CHECK(or_survivor_list(db, n, d, k, alpha, qs + q * d, lo[q], list, n) == clo[q]);
        CHECK(or_survivor_list(db, n, d, k, alpha, qs + q * d, hi[q], list, 2) == chi[q]);
    }

    int64_t *ti = malloc(sizeof(int64_t) * nq * kk);
    double *ts = malloc(sizeof(double) * nq * kk);
    or_topk(db, n, d, qs, nq, kk, 2, ti, ts);
    for (int q = 0; q < nq; ++q) CHECK(ti[q * kk] == bi[q] && ts[q * kk] == bs[q]);
    int64_t *small_i = malloc(sizeof(int64_t) * (n + 3));
    double *small_s = malloc(sizeof(double) * (n + 3));
    or_topk(db, n, d, qs, 1, (int)n + 3, 1, small_i, small_s);
    CHECK(small_i[n] == -1 && isinf(small_s[n + 2]));

    double u[7];
    int64_t anchors[7];
    for (int t = 0; t < na; ++t) u[t] = uniform01();
    or_kmeanspp(db, n, d, na, u, anchors);
    for (int t = 0; t < na; ++t) CHECK(anchors[t] >= 0 && anchors[t] < n);
    CHECK(or_sim(qs, db, d) == or_sim(qs, db, d));

    free(db); free(qs); free(bi); free(ri); free(bs); free(rs); free(seed); free(p2);
    free(ss); free(sl); free(lo); free(hi); free(clo); free(chi); free(list); free(ti);
    free(ts); free(small_i); free(small_s);
    printf("oracle sanitizer run: ok\n");
    return 0;
}
