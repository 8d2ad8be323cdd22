// Per-candidate normalisation parameters for the batched kernels: from the blocked FP64 prefix of
// the series (any window length) or from per-window arrays of one length.
#pragma once
#include "device.h"

namespace dtws {

// Mean and population sigma of T[i .. i+m) from the blocked prefix (FP64).  Windows whose prefix
// difference may have lost relative precision (short windows, heavy cancellation) are recomputed
// two-pass from the series.
struct StatsPrefix {
    static constexpr bool kRuns = true;   // the cascade may walk items as chains (see cascade)
    const float *T;
    Prefix pre;
    int m;
    double inv_m;
    // Sums of (T - a0) and of its square over window i, a0 = the anchor of the window's first block
    // (m <= 2048 < kPB: the window ends in its first block or the next; branch free, the lookups
    // past the last block hit sentinels).
    __device__ void sums(int64_t i, double &a0, double &S1, double &S2) const {
        sums_from(i, pre.at(i), pre.at(i + m), a0, S1, S2);
    }
    // The same for a group of 64 consecutive windows that share the block b0 of their starts and
    // whether they end past it (both wave-uniform: m and the group start are multiples of 64 and
    // kPB is a multiple of 64); el = e - (b0 + 1) kPB for this lane's window end e.  The block's
    // anchor a_lo = anc[b0], the next one a_hi = anc[b0 + 1] and the block totals t = tot[b0] are
    // passed in (the caller loads them for both groups of a step together).
    __device__ void sums_group(bool cross, int el, double2 p0, double2 pe, double a_lo, double a_hi, double2 t,
                               double &S1, double &S2) const {
        if (cross) {
            const double delta = a_hi - a_lo;
            const double c2 = (double)el;
            S1 = (t.x - p0.x) + pe.x + c2 * delta;
            S2 = (t.y - p0.y) + pe.y + 2.0 * delta * pe.x + c2 * delta * delta;
        } else {
            S1 = pe.x - p0.x;
            S2 = pe.y - p0.y;
        }
    }
    // the same from the prefix entries p0 = PP[i] and pe = PP[i + m]
    __device__ void sums_from(int64_t i, double2 p0, double2 pe, double &a0, double &S1, double &S2) const {
        const int64_t e = i + m;
        const int64_t b0 = i / kPB, e0 = (b0 + 1) * kPB;
        const bool cross = e >= e0;
        // unconditional loads (the entry past the last block exists), selected afterwards
        const double2 t = pre.tot[b0];
        a0 = pre.anc[b0];
        const double a1 = pre.anc[b0 + 1];
        const double delta = cross ? a1 - a0 : 0.0;
        const double c2 = (double)(e - e0);
        const double cS1 = (t.x - p0.x) + pe.x + c2 * delta;
        const double cS2 = (t.y - p0.y) + pe.y + 2.0 * delta * pe.x + c2 * delta * delta;
        S1 = cross ? cS1 : pe.x - p0.x;
        S2 = cross ? cS2 : pe.y - p0.y;
    }
    // Normalisation parameters from anchored sums.  Windows whose sums may have lost relative
    // precision (short windows, heavy cancellation) are recomputed two-pass from the series.  The
    // scale is stored in FP32 anyway, so 1/sigma comes from the FP32 reciprocal square root of the
    // FP64 variance (relative error ~2^-23); flat windows (sigma <= 1e-8) get scale 0.
    __device__ void finish(int64_t i, double a0, double S1, double S2, float &mu32, float &s, float &o) const {
        const double md = S1 * inv_m, msq = S2 * inv_m;
        double var = msq - md * md, mu = a0 + md;
        if (m <= 64 || !(var > 4e-6 * msq)) {
            const float *w = T + i;
            double sm = 0.0;
            for (int j = 0; j < m; ++j) sm += (double)w[j];
            mu = sm / m;
            double q = 0.0;
            for (int j = 0; j < m; ++j) {
                const double d = (double)w[j] - mu;
                q += d * d;
            }
            var = q / m;
        }
        mu32 = (float)mu;
        // var > kSigmaFlat^2 is a normal FP32 number: the hardware reciprocal square root needs no
        // denormal scaling; anything else (flat, negative from rounding, NaN) gets scale 0
        s = var > kSigmaFlat * kSigmaFlat ? __builtin_amdgcn_rsqf((float)var) : 0.0f;
        o = (float)(-(mu - (double)mu32)) * s;
    }
    __device__ void operator()(int64_t i, float &mu32, float &s, float &o) const {
        double a0, S1, S2;
        sums(i, a0, S1, S2);
        finish(i, a0, S1, S2, mu32, s, o);
    }
};

struct StatsArr {
    static constexpr bool kRuns = false;
    const float *mu, *s, *o;   // already offset to the query's statistics slot
    __device__ void operator()(int64_t i, float &m, float &sg, float &off) const {
        m = mu[i];
        sg = s[i];
        off = o[i];
    }
};

// Appends the survivors of one wave (alive lanes, start i, query q) to the batch's survivor list;
// an append past the capacity raises the overflow flag instead (the batch then falls back).
struct EmitBatch {
    int32_t *surv_q, *surv_i;
    float *surv_lb;
    uint32_t *count, *qcnt, *overflow;
    int64_t cap;
    int q;
    // lb: the survivor's query-envelope LB_Keogh sum, kept for the DTW's abandoning test
    __device__ void operator()(bool alive, int64_t i, float lb) const {
        const uint64_t mask = __ballot(alive);
        if (!mask) return;
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((unsigned long long)mask) - 1;
        const uint32_t pc = (uint32_t)__popcll(mask);
        uint32_t base = 0;
        if (lane == leader) {
            base = atomicAdd(count, pc);
            if ((int64_t)base + pc > cap) atomicOr(overflow, 1u);
            else atomicAdd(&qcnt[q * kCntStride], pc);
        }
        base = __shfl(base, leader, 64);
        const int64_t pos = (int64_t)base + __popcll(mask & lanemask_lt());
        if (alive && (int64_t)base + pc <= cap) {
            surv_q[pos] = q;
            surv_i[pos] = (int32_t)i;
            surv_lb[pos] = lb;
        }
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
