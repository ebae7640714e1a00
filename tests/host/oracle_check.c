/* The CPU oracle (oracle/sj_oracle.c) built with the address and
 * undefined-behaviour sanitizers by tests/test_host_sanitizers.py: its modes
 * run on random and adversarial inputs (zero extents, shared edges, signed
 * zeros, coordinates outside the domain, one and many threads), must agree
 * with one another and must not touch memory they do not own. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_bruteforce(const float *R, int64_t nR, const float *S, int64_t nS, int32_t **out);
int64_t oracle_sweep(const float *R, int64_t nR, const float *S, int64_t nS, int32_t **out);
int64_t oracle_pbsm(const float *R, int64_t nR, const float *S, int64_t nS, int K,
                    const float *domain, int threads, int32_t **out, double *t_part, double *t_join);
int64_t oracle_gbda(const float *R, int64_t nR, const float *S, int64_t nS, int K,
                    const float *domain, int32_t **out);
int64_t oracle_partition_ids(const float *A, int64_t n, int K, const float *domain, int64_t *off,
                             int32_t **ids);
int64_t oracle_distance_brute(const float *P, int64_t nP, const float *Q, int64_t nQ, float eps,
                              int32_t **out);
int64_t oracle_distance_refine(const float *P, const float *Q, float eps, int32_t *pairs, int64_t n);
void oracle_free(void *p);

static uint64_t state = 88172645463325252ull;
static double urand(void) { /* xorshift64 */
    state ^= state << 13, state ^= state >> 7, state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static void rects(float *A, int64_t n, int K) {
    for (int64_t i = 0; i < n; i++) {
        int kind = (int)(urand() * 5);
        float x = (float)urand(), y = (float)urand();
        if (kind == 1) x = (float)((int)(urand() * (K + 2)) - 1) / K, y = (float)((int)(urand() * (K + 2)) - 1) / K;
        if (kind == 2) x = urand() < 0.5 ? -0.0f : 0.0f, y = urand() < 0.5 ? -0.0f : 0.0f;
        float w = kind == 3 ? 0.0f : (float)(urand() * 0.3), h = kind == 3 ? 0.0f : (float)(urand() * 0.3);
        A[4 * i] = x, A[4 * i + 1] = y, A[4 * i + 2] = x + w, A[4 * i + 3] = y + h;
        if (kind == 4 && i > 0) memcpy(A + 4 * i, A + 4 * (i - 1 - (int64_t)(urand() * i)), 16);
    }
}

static int cmp_pair(const void *a, const void *b) {
    const int32_t *x = a, *y = b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return (x[1] > y[1]) - (x[1] < y[1]);
}

static int same(int32_t *a, int64_t na, int32_t *b, int64_t nb) {
    if (na != nb) return 0;
    if (na == 0) return 1;
    qsort(a, (size_t)na, 8, cmp_pair);
    qsort(b, (size_t)nb, 8, cmp_pair);
    return memcmp(a, b, (size_t)na * 8) == 0;
}

int main(void) {
    int fails = 0;
    for (int round = 0; round < 30; round++) {
        int K = 1 + (int)(urand() * 20);
        int64_t nR = (int64_t)(urand() * 300), nS = (int64_t)(urand() * 300);
        float *R = malloc((size_t)(nR + 1) * 16), *S = malloc((size_t)(nS + 1) * 16);
        rects(R, nR, K);
        rects(S, nS, K);
        int32_t *ref = NULL, *got = NULL;
        int64_t n = oracle_bruteforce(R, nR, S, nS, &ref);
        int32_t *tmp = NULL;
        int64_t m = oracle_sweep(R, nR, S, nS, &tmp);
        if (!same(tmp, m, ref, n)) { fprintf(stderr, "sweep differs, round %d\n", round); fails++; }
        oracle_free(tmp);
        for (int threads = 1; threads <= 4; threads += 3) {
            int32_t *ref2 = malloc((size_t)(n + 1) * 8);
            memcpy(ref2, ref, (size_t)n * 8);
            got = NULL;
            m = oracle_pbsm(R, nR, S, nS, K, NULL, threads, &got, NULL, NULL);
            if (!same(got, m, ref2, n)) { fprintf(stderr, "pbsm differs, round %d\n", round); fails++; }
            oracle_free(got);
            free(ref2);
        }
        float dom[4] = {-0.5f, -0.5f, 1.5f, 1.5f};
        got = NULL;
        m = oracle_gbda(R, nR, S, nS, K, dom, &got);
        if (!same(got, m, ref, n)) { fprintf(stderr, "gbda differs, round %d\n", round); fails++; }
        oracle_free(got);
        int64_t *off = malloc((size_t)K * K * 8 + 8);
        int32_t *ids = NULL;
        int64_t e = oracle_partition_ids(R, nR, K, NULL, off, &ids);
        if (e < nR || off[(int64_t)K * K] != e) { fprintf(stderr, "partition, round %d\n", round); fails++; }
        oracle_free(ids);
        free(off);
        /* distance join of the lower corners: brute force vs the refinement
         * of every pair */
        float *P = malloc((size_t)(nR + 1) * 8), *Q = malloc((size_t)(nS + 1) * 8);
        for (int64_t i = 0; i < nR; i++) P[2 * i] = R[4 * i], P[2 * i + 1] = R[4 * i + 1];
        for (int64_t j = 0; j < nS; j++) Q[2 * j] = S[4 * j], Q[2 * j + 1] = S[4 * j + 1];
        int32_t *dref = NULL;
        int64_t dn = oracle_distance_brute(P, nR, Q, nS, 0.1f, &dref);
        int32_t *all = malloc((size_t)(nR * nS + 1) * 8);
        for (int64_t i = 0, k = 0; i < nR; i++)
            for (int64_t j = 0; j < nS; j++, k++) all[2 * k] = (int32_t)i, all[2 * k + 1] = (int32_t)j;
        int64_t kept = oracle_distance_refine(P, Q, 0.1f, all, nR * nS);
        if (!same(all, kept, dref, dn)) { fprintf(stderr, "distance, round %d\n", round); fails++; }
        free(all);
        oracle_free(dref);
        free(P);
        free(Q);
        oracle_free(ref);
        free(R);
        free(S);
    }
    if (fails) return 1;
    printf("oracle checks passed\n");
    return 0;
}
