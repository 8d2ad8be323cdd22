/* Drives the C cascade oracle (oracle/cascade.c) on small seeded inputs and edge cases, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer.  Prints one line per case; exits non-zero
 * when an entry point reports an error or two entry points disagree on a case. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oc_search(const float *T, int64_t n, const float *Q, int32_t m, int32_t r, int32_t nthreads,
              int64_t *best_idx, double *best_dist, int64_t *counters);
int oc_search_many(const float *T, int64_t n, const float *Q, int32_t m, const int32_t *r_in, int32_t nq,
                   int32_t nthreads, int64_t *best_idx, double *best_dist, int64_t *counters);
int oc_dtw_starts(const float *T, int64_t n, const float *Q, int32_t m, int32_t r, const int64_t *starts,
                  int64_t count, int32_t nthreads, double *out);

/* 64-bit linear congruential generator (Knuth's MMIX constants), uniform in [-0.5, 0.5). */
static uint64_t lcg_state = 12345;
static double uni(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) / 9007199254740992.0 - 0.5;
}

static int run_case(const char *name, const float *T, int64_t n, const float *Q, int32_t m, int32_t r) {
    int64_t idx = -1, cnt[6];
    double d = 0.0;
    if (oc_search(T, n, Q, m, r, 2, &idx, &d, cnt) != 0) {
        printf("%s: oc_search failed\n", name);
        return 1;
    }
    int64_t idx2 = -1;
    double d2 = 0.0;
    const int32_t rr[2] = {r, r};
    int64_t idxs[2];
    double ds[2];
    float *Q2 = (float *)malloc(sizeof(float) * 2 * (size_t)m);
    for (int j = 0; j < m; ++j) Q2[j] = Q2[m + j] = Q[j];
    if (oc_search_many(T, n, Q2, m, rr, 2, 2, idxs, ds, cnt) != 0) {
        printf("%s: oc_search_many failed\n", name);
        free(Q2);
        return 1;
    }
    idx2 = idxs[1];
    d2 = ds[1];
    free(Q2);
    double full = NAN;
    if (idx >= 0 && oc_dtw_starts(T, n, Q, m, r, &idx, 1, 1, &full) != 0) {
        printf("%s: oc_dtw_starts failed\n", name);
        return 1;
    }
    printf("%s: n=%lld m=%d r=%d best %lld %.9g (many %lld %.9g, full %.9g)\n", name, (long long)n, m, r,
           (long long)idx, d, (long long)idx2, d2, full);
    if (idx != idx2 || d != d2 || (idx >= 0 && fabs(full - d) > 1e-9 * (1.0 + d))) return 1;
    return 0;
}

int main(void) {
    const int64_t n = 20000;
    float *T = (float *)malloc(sizeof(float) * n);
    double x = 0.0;
    for (int64_t i = 0; i < n; ++i) T[i] = (float)(x += uni());
    for (int64_t i = 5000; i < 5400; ++i) T[i] = 3.0f;   /* a flat stretch */
    float Q[300];
    int bad = 0;
    for (int j = 0; j < 300; ++j) Q[j] = T[12000 + j] + 0.1f * (float)uni();
    bad |= run_case("cut m=128 r=6", T, n, Q, 128, 6);
    bad |= run_case("cut m=300 r=30", T, n, Q, 300, 30);
    bad |= run_case("band wider than the query", T, n, Q, 64, 500);
    bad |= run_case("band 0", T, n, Q, 100, 0);
    bad |= run_case("m = 1", T, n, Q, 1, 0);
    bad |= run_case("m = 2", T, n, Q, 2, 1);
    bad |= run_case("series as long as the query", T, 128, Q, 128, 12);
    float flat[64];
    for (int j = 0; j < 64; ++j) flat[j] = 7.0f;
    bad |= run_case("flat query", T, n, flat, 64, 6);
    bad |= run_case("flat query on the flat stretch", T + 5000, 400, flat, 64, 6);
    free(T);
    return bad;
}
