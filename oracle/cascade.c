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
 *     thread (the paper's static OpenMP partition, Section 3.3).  A thread
 *     scans its segment in two passes, every 64th start first, then the rest,
 *     so that it meets a close match early.  Threads
 *     share the best-so-far value for pruning through an atomic; each keeps
 *     its own best (distance, index) and the results are reduced by minimum
 *     distance, then lowest index.
 *   - a window is normalised point by point as the bounds need it: LB_Kim
 *     takes its moments and its first and last points, LB_Keogh against the
 *     query envelope normalises each point as it adds its term, and only a
 *     survivor of both is normalised in full (the values are the same either
 *     way).  oc_search_many runs several queries of one length in one
 *     scan, sharing each window's moments; every query keeps its own
 *     best-so-far and cascade, so each result is oc_search's.
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

/* Mean and population sigma of x[0..m) (eq. (Normalization1)), two passes in FP64: the mean first,
 * then the mean squared deviation.  Each pass keeps eight partial sums (elements j = k mod 8), added
 * in a fixed order at the end; that is only another rounding order of the same sums. */
__attribute__((target_clones("avx2", "default")))
static void window_moments(const float *x, int m, double *mu_out, double *sigma_out) {
    double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int j = 0;
    for (; j + 8 <= m; j += 8)
        for (int k = 0; k < 8; ++k) p[k] += (double)x[j + k];
    for (; j < m; ++j) p[j & 7] += (double)x[j];
    double mu = (((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]))) / m;
    for (int k = 0; k < 8; ++k) p[k] = 0.0;
    for (j = 0; j + 8 <= m; j += 8)
        for (int k = 0; k < 8; ++k) { double d = (double)x[j + k] - mu; p[k] += d * d; }
    for (; j < m; ++j) { double d = (double)x[j] - mu; p[j & 7] += d * d; }
    double v = (((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]))) / m;
    *mu_out = mu;
    *sigma_out = sqrt(v);
}

/* 1 / sigma, or 0 for a flat window (sigma <= 1e-8): a flat window normalises to zeros */
static inline double inv_sigma(double sigma) { return sigma <= SIGMA_FLAT ? 0.0 : 1.0 / sigma; }

/* normalised value of one point, (t - mu) / sigma as (t - mu) * (1 / sigma) */
static inline double znorm_point(float t, double mu, double inv) { return ((double)t - mu) * inv; }

static void znorm_window(const float *x, int m, double *out) {
    double mu, sigma;
    window_moments(x, m, &mu, &sigma);
    const double inv = inv_sigma(sigma);
    for (int j = 0; j < m; ++j) out[j] = znorm_point(x[j], mu, inv);
}

static void envelope(const double *x, int m, int r, double *U, double *L) {
    for (int i = 0; i < m; ++i) {
        int a = i - r < 0 ? 0 : i - r, b = i + r > m - 1 ? m - 1 : i + r;
        double u = x[a], l = x[a];
        for (int k = a + 1; k <= b; ++k) { if (x[k] > u) u = x[k]; if (x[k] < l) l = x[k]; }
        U[i] = u; L[i] = l;
    }
}

/* eq. (LBKeoghEC) for the window x[0..m) normalised with (mu, sigma) point by point as it goes,
 * with early abandon once the partial sum exceeds thr (the values are znorm_point's). */
static double lb_keogh_window(const float *x, double mu, double inv, const double *U, const double *L, int m,
                              double thr) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
        double c = znorm_point(x[i], mu, inv);
        if (c > U[i]) { double d = c - U[i]; s += d * d; }
        else if (c < L[i]) { double d = c - L[i]; s += d * d; }
        if (s > thr) return s;
    }
    return s;
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

/* Position number `it` of a thread's scan of its segment [a, b): first every SCAN_STRIDE-th start
 * (a, a + SCAN_STRIDE, ...), then the others in order.  Any order gives the same exact result
 * (ties are resolved by index); sampling the whole segment first finds a close match, and with it
 * a tight best-so-far, early. */
#define SCAN_STRIDE 64
static inline int64_t scan_position(int64_t a, int64_t b, int64_t it) {
    const int64_t len = b - a, first = (len + SCAN_STRIDE - 1) / SCAN_STRIDE;
    if (it < first) return a + it * SCAN_STRIDE;
    it -= first;   /* the it-th start that is not a multiple of the stride past a */
    return a + (it / (SCAN_STRIDE - 1)) * SCAN_STRIDE + 1 + it % (SCAN_STRIDE - 1);
}

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
        for (int64_t it = 0; it < b - a; ++it) {
            const int64_t i = scan_position(a, b, it);
            c[0]++;
            double bsf = bitsd(__atomic_load_n(&gbsf, __ATOMIC_RELAXED));
            if (best < bsf) bsf = best;
            double thr = bsf * SLACK;
            /* LB_Kim needs only the window's moments and its first and last points; the whole
             * window is normalised once the candidate survives it */
            double mu, sigma;
            window_moments(T + i, m, &mu, &sigma);
            const double inv = inv_sigma(sigma);
            double c0 = znorm_point(T[i], mu, inv), cl = znorm_point(T[i + m - 1], mu, inv);
            double lk = (m == 1) ? (qh[0] - c0) * (qh[0] - c0)
                                 : (qh[0] - c0) * (qh[0] - c0) + (qh[m - 1] - cl) * (qh[m - 1] - cl);
            if (lk > thr) { c[1]++; continue; }
            if (lb_keogh_window(T + i, mu, inv, U, Lq, m, thr) > thr) { c[2]++; continue; }
            for (int j = 0; j < m; ++j) ch[j] = znorm_point(T[i + j], mu, inv);
            envelope(ch, m, r, Uc, Lc);
            if (lb_keogh(qh, Uc, Lc, m, thr) > thr) { c[3]++; continue; }
            double d = dtw_band(qh, ch, m, r, thr, prev, cur);
            if (d == INFINITY) { c[4]++; continue; }
            c[5]++;
            if (d < best || (d == best && i < bidx)) { best = d; bidx = i; publish_bsf(&gbsf, d); }
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

/* The same search for nq queries of one length m against one series (queries back to back in Q,
 * band r[k] for query k): every window's moments are computed once and serve all the queries; each
 * query keeps its own best-so-far and its own cascade, exactly as oc_search.  best_idx[k] and
 * best_dist[k] receive query k's result; counters as oc_search, summed over the queries. */
int oc_search_many(const float *T, int64_t n, const float *Q, int32_t m, const int32_t *r_in, int32_t nq,
                   int32_t nthreads, int64_t *best_idx, double *best_dist, int64_t *counters) {
    if (!T || !Q || !r_in || nq < 1 || m < 1 || n < m) return -1;
    for (int k = 0; k < nq; ++k) if (r_in[k] < 0) return -1;
    int64_t N = n - m + 1;
    int *r = (int *)malloc(sizeof(int) * nq);
    double *qh = (double *)malloc(sizeof(double) * (size_t)m * 3 * nq);
    uint64_t *gbsf = (uint64_t *)malloc(sizeof(uint64_t) * nq);
    double *gbest = (double *)malloc(sizeof(double) * nq);
    int64_t *gidx = (int64_t *)malloc(sizeof(int64_t) * nq);
    for (int k = 0; k < nq; ++k) {
        r[k] = r_in[k] > m - 1 ? m - 1 : r_in[k];
        double *q = qh + (size_t)3 * m * k;
        znorm_window(Q + (size_t)m * k, m, q);
        envelope(q, m, r[k], q + m, q + 2 * m);
        gbsf[k] = dbits(INFINITY);
        gbest[k] = INFINITY;
        gidx[k] = -1;
    }
    int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        int p = omp_get_num_threads(), t = omp_get_thread_num();
        int64_t a = N * t / p, b = N * (t + 1) / p;
        double *buf = (double *)malloc(sizeof(double) * (size_t)m * 6 + 16);
        double *best = (double *)malloc(sizeof(double) * nq);
        int64_t *bidx = (int64_t *)malloc(sizeof(int64_t) * nq);
        double *ch = buf, *Uc = buf + m, *Lc = buf + 2 * m, *prev = buf + 3 * m, *cur = buf + 4 * m + 2;
        int64_t c[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < nq; ++k) { best[k] = INFINITY; bidx[k] = -1; }
        for (int64_t it = 0; it < b - a; ++it) {
            const int64_t i = scan_position(a, b, it);
            double mu, sigma;
            window_moments(T + i, m, &mu, &sigma);
            const double inv = inv_sigma(sigma);
            double c0 = znorm_point(T[i], mu, inv), cl = znorm_point(T[i + m - 1], mu, inv);
            int full = 0;   /* ch holds the normalised window */
            for (int k = 0; k < nq; ++k) {
                const double *q = qh + (size_t)3 * m * k, *U = q + m, *Lq = q + 2 * m;
                c[0]++;
                double bsf = bitsd(__atomic_load_n(&gbsf[k], __ATOMIC_RELAXED));
                if (best[k] < bsf) bsf = best[k];
                double thr = bsf * SLACK;
                double lk = (m == 1) ? (q[0] - c0) * (q[0] - c0)
                                     : (q[0] - c0) * (q[0] - c0) + (q[m - 1] - cl) * (q[m - 1] - cl);
                if (lk > thr) { c[1]++; continue; }
                if (lb_keogh_window(T + i, mu, inv, U, Lq, m, thr) > thr) { c[2]++; continue; }
                if (!full) {
                    for (int j = 0; j < m; ++j) ch[j] = znorm_point(T[i + j], mu, inv);
                    full = 1;
                }
                envelope(ch, m, r[k], Uc, Lc);
                if (lb_keogh(q, Uc, Lc, m, thr) > thr) { c[3]++; continue; }
                double d = dtw_band(q, ch, m, r[k], thr, prev, cur);
                if (d == INFINITY) { c[4]++; continue; }
                c[5]++;
                if (d < best[k] || (d == best[k] && i < bidx[k])) { best[k] = d; bidx[k] = i; publish_bsf(&gbsf[k], d); }
            }
        }
#pragma omp critical
        {
            for (int k = 0; k < nq; ++k)
                if (bidx[k] >= 0 && (best[k] < gbest[k] || (best[k] == gbest[k] && bidx[k] < gidx[k]))) {
                    gbest[k] = best[k];
                    gidx[k] = bidx[k];
                }
            for (int k = 0; k < 6; ++k) cnt[k] += c[k];
        }
        free(buf);
        free(best);
        free(bidx);
    }
    for (int k = 0; k < nq; ++k) { best_idx[k] = gidx[k]; best_dist[k] = gbest[k]; }
    if (counters) for (int k = 0; k < 6; ++k) counters[k] = cnt[k];
    free(r); free(qh); free(gbsf); free(gbest); free(gidx);
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
