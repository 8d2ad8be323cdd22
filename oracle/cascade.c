/*
 * FP64 CPU oracle: exact best-match subsequence search under banded,
 * z-normalised, squared DTW, by the sequential cascade scan the paper builds on.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the GPU search library.
 *
 * Source: Kraeva & Zymbler, arXiv:1812.10302.
 *   - DTW recurrence: Section 2.1, eq. (dtw); Sakoe-Chiba band: Section 2.1.
 *   - z-normalisation: Section 2.2, eq. (Normalization1), population sigma,
 *     computed two-pass per window; sigma <= 1e-8 means a flat window that
 *     normalises to zeros.
 *   - cascade of lower bounds and the best-so-far rule: Section 2.2,
 *     eqs. (bsf), (LB_Kim), (LBKeoghEC), (envelope), (LBKeoghEQ), and the
 *     closing description of the sequential scan: normalise the query, build
 *     its envelope, set bsf to infinity, then for each candidate apply the
 *     bounds in order and compute DTW only for candidates that survive.
 *   - LB_KimFL is taken with squared differences (the printed unsquared form
 *     does not bound squared DTW); envelopes are clipped to the sequence.
 *   - the DTW call carries the current bsf as an early-abandon threshold: a
 *     row of the band whose every cell exceeds it proves DTW > bsf, because
 *     every warping path crosses every row and costs are non-negative.
 *   - threads: the candidates are split into contiguous segments, one per
 *     thread (the paper's static OpenMP partition, Section 3.3).  Threads
 *     share the best-so-far value for pruning through an atomic; each keeps
 *     its own best (distance, index) and the results are reduced by minimum
 *     distance, then lowest index.
 *   - pruning compares with a relative slack of 1e-12 (prune only when
 *     bound > bsf * (1 + 1e-12)), so FP64 rounding in a bound can never drop
 *     a candidate whose distance ties the best.  Slack only weakens pruning.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define SIGMA_FLAT 1e-8
#define SLACK (1.0 + 1e-12)

static void znorm_window(const float *x, int m, double *out) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += (double)x[j];
    double mu = s / m;
    double v = 0.0;
    for (int j = 0; j < m; ++j) { double d = (double)x[j] - mu; v += d * d; }
    double sigma = sqrt(v / m);
    if (sigma <= SIGMA_FLAT) { for (int j = 0; j < m; ++j) out[j] = 0.0; return; }
    for (int j = 0; j < m; ++j) out[j] = ((double)x[j] - mu) / sigma;
}

static void envelope(const double *x, int m, int r, double *U, double *L) {
    for (int i = 0; i < m; ++i) {
        int a = i - r < 0 ? 0 : i - r, b = i + r > m - 1 ? m - 1 : i + r;
        double u = x[a], l = x[a];
        for (int k = a + 1; k <= b; ++k) { if (x[k] > u) u = x[k]; if (x[k] < l) l = x[k]; }
        U[i] = u; L[i] = l;
    }
}

/* eq. (LBKeoghEC) with early abandon once the partial sum exceeds thr. */
static double lb_keogh(const double *x, const double *U, const double *L, int m, double thr) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
        if (x[i] > U[i]) { double d = x[i] - U[i]; s += d * d; }
        else if (x[i] < L[i]) { double d = x[i] - L[i]; s += d * d; }
        if (s > thr) return s;
    }
    return s;
}

/* eq. (dtw) restricted to |i-j| <= r, rolling two rows; returns +inf once a whole row exceeds thr. */
static double dtw_band(const double *x, const double *y, int m, int r, double thr,
                       double *prev, double *cur) {
    if (r > m - 1) r = m - 1;
    /* prev/cur hold d(i, 0..m) (1-based j) */
    for (int j = 0; j <= m; ++j) prev[j] = INFINITY;
    prev[0] = 0.0;
    for (int j = 0; j <= m; ++j) cur[j] = INFINITY;
    for (int i = 1; i <= m; ++i) {
        int jlo = i - r < 1 ? 1 : i - r, jhi = i + r > m ? m : i + r;
        /* cells of row i outside the band are +inf; only the two next to it are ever read */
        cur[jlo - 1] = INFINITY;
        if (jhi + 1 <= m) cur[jhi + 1] = INFINITY;
        double rowmin = INFINITY;
        for (int j = jlo; j <= jhi; ++j) {
            double c = (x[i - 1] - y[j - 1]) * (x[i - 1] - y[j - 1]);
            double a = prev[j], b = cur[j - 1], d = prev[j - 1];
            double mn = a < b ? a : b;
            mn = mn < d ? mn : d;
            cur[j] = c + mn;
            if (cur[j] < rowmin) rowmin = cur[j];
        }
        if (rowmin > thr) return INFINITY;
        double *t = prev; prev = cur; cur = t;
    }
    return prev[m];
}

static inline uint64_t dbits(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }
static inline double bitsd(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }

/* Shared best-so-far (a non-negative double: its bit pattern orders like the value). */
static void publish_bsf(uint64_t *g, double d) {
    uint64_t nb = dbits(d), cur = __atomic_load_n(g, __ATOMIC_RELAXED);
    while (nb < cur && !__atomic_compare_exchange_n(g, &cur, nb, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
}

/* counters[0..5]: candidates, pruned by LB_Kim, by LB_Keogh(query env), by LB_Keogh(candidate env),
 * DTW abandoned, DTW completed. */
int oc_search(const float *T, int64_t n, const float *Q, int32_t m, int32_t r, int32_t nthreads,
              int64_t *best_idx, double *best_dist, int64_t *counters) {
    if (!T || !Q || m < 1 || n < m || r < 0) return -1;
    if (r > m - 1) r = m - 1;
    int64_t N = n - m + 1;
    double *qh = (double *)malloc(sizeof(double) * m * 3);
    double *U = qh + m, *Lq = qh + 2 * m;
    znorm_window(Q, m, qh);
    envelope(qh, m, r, U, Lq);
    uint64_t gbsf = dbits(INFINITY);
    int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
    double gbest = INFINITY;
    int64_t gidx = -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        int p = omp_get_num_threads(), t = omp_get_thread_num();
        int64_t a = N * t / p, b = N * (t + 1) / p;
        double *buf = (double *)malloc(sizeof(double) * (size_t)m * 6 + 16);
        double *ch = buf, *Uc = buf + m, *Lc = buf + 2 * m, *prev = buf + 3 * m, *cur = buf + 4 * m + 2;
        double best = INFINITY;
        int64_t bidx = -1, c[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t i = a; i < b; ++i) {
            c[0]++;
            double bsf = bitsd(__atomic_load_n(&gbsf, __ATOMIC_RELAXED));
            if (best < bsf) bsf = best;
            double thr = bsf * SLACK;
            znorm_window(T + i, m, ch);
            double lk = (m == 1) ? (qh[0] - ch[0]) * (qh[0] - ch[0])
                                 : (qh[0] - ch[0]) * (qh[0] - ch[0]) + (qh[m - 1] - ch[m - 1]) * (qh[m - 1] - ch[m - 1]);
            if (lk > thr) { c[1]++; continue; }
            if (lb_keogh(ch, U, Lq, m, thr) > thr) { c[2]++; continue; }
            envelope(ch, m, r, Uc, Lc);
            if (lb_keogh(qh, Uc, Lc, m, thr) > thr) { c[3]++; continue; }
            double d = dtw_band(qh, ch, m, r, thr, prev, cur);
            if (d == INFINITY) { c[4]++; continue; }
            c[5]++;
            if (d < best) { best = d; bidx = i; publish_bsf(&gbsf, d); }
        }
#pragma omp critical
        {
            if (bidx >= 0 && (best < gbest || (best == gbest && bidx < gidx))) { gbest = best; gidx = bidx; }
            for (int k = 0; k < 6; ++k) cnt[k] += c[k];
        }
        free(buf);
    }
    free(qh);
    *best_idx = gidx;
    *best_dist = gbest;
    if (counters) for (int k = 0; k < 6; ++k) counters[k] = cnt[k];
    return 0;
}

/* FP64 banded DTW (no abandoning) of the normalised query against the normalised candidates at the
 * given starts. */
int oc_dtw_starts(const float *T, int64_t n, const float *Q, int32_t m, int32_t r, const int64_t *starts,
                  int64_t count, int32_t nthreads, double *out) {
    if (!T || !Q || !starts || !out || m < 1 || n < m || r < 0) return -1;
    for (int64_t k = 0; k < count; ++k) if (starts[k] < 0 || starts[k] > n - m) return -1;
    double *qh = (double *)malloc(sizeof(double) * m);
    znorm_window(Q, m, qh);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)m * 3 + 16);
        double *ch = buf, *prev = buf + m, *cur = buf + 2 * m + 1;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < count; ++k) {
            znorm_window(T + starts[k], m, ch);
            out[k] = dtw_band(qh, ch, m, r, INFINITY, prev, cur);
        }
        free(buf);
    }
    free(qh);
    return 0;
}

int oc_num_threads(void) { return omp_get_max_threads(); }
