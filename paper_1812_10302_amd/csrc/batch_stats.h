// Per-candidate normalisation parameters for the batched kernels: from the blocked FP64 prefix of
// the series (any window length) or from per-window arrays of one length.
#pragma once
#include "device.h"

namespace dtws {

// Mean and population sigma of T[i .. i+m) from the blocked prefix (FP64).  Windows whose prefix
// difference may have lost relative precision (short windows, heavy cancellation) are recomputed
// two-pass from the series.
struct StatsPrefix {
    const float *T;
    const double *P1, *P2, *anc, *tot1, *tot2;
    int m;
    double inv_m;
    // mean and variance of window i
    __device__ void window(int64_t i, double &mu, double &var) const {
        const int64_t e = i + m;
        const int64_t b0 = i / kPB, b1 = (e - 1) / kPB;
        double e1, e2;
        if (e == (b1 + 1) * kPB) {
            e1 = tot1[b1];
            e2 = tot2[b1];
        } else {
            e1 = P1[e];
            e2 = P2[e];
        }
        double S1, S2;
        if (b0 == b1) {
            S1 = e1 - P1[i];
            S2 = e2 - P2[i];
        } else {
            const double delta = anc[b1] - anc[b0];
            const double c2 = (double)(e - b1 * kPB);
            S1 = (tot1[b0] - P1[i]) + e1 + c2 * delta;
            S2 = (tot2[b0] - P2[i]) + e2 + 2.0 * delta * e1 + c2 * delta * delta;
        }
        const double md = S1 * inv_m, msq = S2 * inv_m;
        var = msq - md * md;
        mu = anc[b0] + md;
        if (m <= 64 || !(var > 4e-6 * msq)) {
            const float *w = T + i;
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += (double)w[j];
            mu = s / m;
            double q = 0.0;
            for (int j = 0; j < m; ++j) {
                const double d = (double)w[j] - mu;
                q += d * d;
            }
            var = q / m;
        }
        if (!(var > 0.0)) var = 0.0;
    }
    // The scale is stored in FP32 anyway, so 1/sigma comes from the FP32 reciprocal square root
    // of the FP64 variance (relative error ~2^-23); flat windows (sigma <= 1e-8) get scale 0.
    __device__ void operator()(int64_t i, float &mu32, float &s, float &o) const {
        double mu, var;
        window(i, mu, var);
        mu32 = (float)mu;
        s = var <= kSigmaFlat * kSigmaFlat ? 0.0f : rsqrtf((float)var);
        o = (float)(-(mu - (double)mu32)) * s;
    }
};

struct StatsArr {
    const float *mu, *s, *o;   // already offset to the query's statistics slot
    __device__ void operator()(int64_t i, float &m, float &sg, float &off) const {
        m = mu[i];
        sg = s[i];
        off = o[i];
    }
};

// Query of wave w of DTW bucket c in the survivor segments (segments are query-major).
__device__ inline int wave_query(const BatchArgs &a, int c, int64_t w, int32_t &wq0) {
    int lo = a.bucket_j[2 * c], hi = a.bucket_j[2 * c + 1];   // wstart[lo] <= w < wstart[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.wstart[mid] <= w) lo = mid;
        else hi = mid;
    }
    wq0 = a.wstart[lo];
    return a.qorder[lo];
}

}  // namespace dtws
