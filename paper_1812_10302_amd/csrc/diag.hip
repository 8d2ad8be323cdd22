// Banded DTW of one candidate by one wave, along anti-diagonals (latency schedule).
//
// The recurrence is eq. (dtw) with the Sakoe-Chiba band of Section 2.1; the three predecessors of
// cell (i, j) lie on the two previous anti-diagonals d - 1 and d - 2 (d = i + j), so all cells of
// one anti-diagonal are independent.  On a diagonal of parity p = (d + r) & 1 the band holds the
// cells with i - j = -r + 2k + p; slot k lives in lane k % 64 of register k / 64 (CPL registers,
// r <= 64 CPL - 1).  The predecessors of slot k are, on an even diagonal, slots k - 1 (up) and k
// (left) of the previous diagonal and, on an odd one, slots k (up) and k + 1 (left); slot k of the
// diagonal before that is the diagonal neighbour.  Neighbouring slots move with DPP wave shifts.
//
// Each wave copies the normalised query and candidate into LDS with padding of huge values of
// opposite sign, so a cell with i or j outside [0, m) costs infinity without a bounds test, and
// consecutive diagonals need one new query or candidate value per lane.  A lane-per-candidate
// kernel needs m steps of 16 NC cells per candidate but runs 64 candidates per wave; this kernel
// needs 2m steps of CPL cells, so it wins whenever few candidates are left.
#include "batch_stats.h"

namespace dtws {

// Kernel instances by the most slot registers per lane they serve (MAXCPL): 4 for bands up to
// r = 255, 16 for bands up to r = 1023.  Pads around the staged arrays, for r < 64 MAXCPL: the
// first diagonals read the query down to index -(r + 1) / 2 and the candidate down to -64 MAXCPL;
// the last ones read the query up to m + 64 MAXCPL and the candidate up to m + r / 2 + 1.
template <int MAXCPL>
struct DiagPads {
    static constexpr int QLo = 32 * MAXCPL + 1, QHi = 64 * MAXCPL + 2;
    static constexpr int CLo = 64 * MAXCPL, CHi = 32 * MAXCPL + 2;
    static constexpr int All = QLo + QHi + CLo + CHi;
};

template <typename F> struct DiagTraits;
template <> struct DiagTraits<float> {
    static constexpr float big = 1e20f;   // (2e20)^2 overflows to infinity
};
template <> struct DiagTraits<double> {
    static constexpr double big = 1e200;
};

// DPP wave shifts: shr gives lane l the value of lane l - 1 (lane 0 gets `fill`), shl the value of
// lane l + 1 (lane 63 gets `fill`).
__device__ __forceinline__ float wave_shr(float fill, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_shl(float fill, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double wave_shr(double fill, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_shl(double fill, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// cost + min of the predecessors; FP32 fused, FP64 rounded as (diff * diff) + min like the
// reference recurrence
__device__ __forceinline__ float cell_value(float diff, float mn) { return fmaf(diff, diff, mn); }
__device__ __forceinline__ double cell_value(double diff, double mn) { return __dadd_rn(__dmul_rn(diff, diff), mn); }

// One anti-diagonal: p1 = previous diagonal, p2 = the one before; dd = the difference of query and
// candidate value of each slot's cell, plus a huge value for slots outside the band on this parity
// (its square overflows to infinity, so those slots stay infinite without a step on the chain).
template <int CPL, bool ODD, typename F>
__device__ __forceinline__ void diag_step(F (&p1)[CPL], F (&p2)[CPL], const F (&dd)[CPL]) {
    const F inf = (F)INFINITY;
    F nv[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        F up, left;
        if (!ODD) {
            const F fill = c == 0 ? inf : lane_value(p1[c - 1], 63);
            up = wave_shr(fill, p1[c]);
            left = p1[c];
        } else {
            const F fill = c == CPL - 1 ? inf : lane_value(p1[c + 1], 0);
            up = p1[c];
            left = wave_shl(fill, p1[c]);
        }
        const F mn = fmin(fmin(up, left), p2[c]);
        nv[c] = cell_value(dd[c], mn);
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        p2[c] = p1[c];
        p1[c] = nv[c];
    }
}

// DTW of the wave's staged pair (qb[0..m), cb[0..m) with the paddings around them), band r <=
// 64 CPL - 1.  With ABANDON the wave stops once every cell of two consecutive diagonals exceeds
// the threshold (every warping path meets one of any two consecutive anti-diagonals, costs are
// non-negative); the threshold is min(thr0, the query's best-so-far), refreshed every 32 pairs from
// a read issued 32 pairs earlier.
// Returns the distance (wave-uniform); pairs = diagonal pairs computed.
template <int CPL, bool ABANDON, typename F>
__device__ F diag_dtw(const F *qb, const F *cb, int m, int r, const uint64_t *key, float thr0, bool &alive,
                      int &pairs) {
    const int lane = threadIdx.x & 63;
    const int s0 = r >> 1;   // slot of i == j on the diagonals of parity r & 1
    const F inf = (F)INFINITY;
    const F big = DiagTraits<F>::big;
    F p1[CPL], p2[CPL], penE[CPL], penO[CPL], qv[CPL], cv[CPL];
    const F *qp[CPL], *cp[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int k = lane + 64 * c;
        penE[c] = k <= r ? (F)0 : big;
        penO[c] = k <= r - 1 ? (F)0 : big;
        // diagonal -2 holds only d(-1, -1) = 0; the loop starts at diagonal 0 (r even) or -1 (r odd)
        p1[c] = ((r & 1) && k == s0) ? (F)0 : inf;
        p2[c] = (!(r & 1) && k == s0) ? (F)0 : inf;
        qp[c] = qb - ((r + 1) >> 1) + k;   // i of slot k on the first even diagonal
        cp[c] = cb + (r >> 1) - k;         // j of slot k on the first even diagonal
        qv[c] = qp[c][0];
        cv[c] = cp[c][0];
    }
    float thr = thr0;
    uint32_t kpend = ~0u;   // best-so-far read 32 pairs before it tightens thr (latency hidden)
    if (ABANDON && key) {
        thr = fminf(thr0, threshold_of(load_bsf(key)));
        kpend = load_key_dist_bits(key);
    }
    alive = true;
    // one (even, odd) pair of diagonals; the odd one and the next even one take the query at i + 1
    // and the candidate at j + 1
    auto pair = [&](int t) {
        F qn[CPL], cn[CPL], de[CPL], dn[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            qn[c] = qp[c][t + 1];
            cn[c] = cp[c][t + 1];
            de[c] = (qv[c] - cv[c]) + penE[c];
            dn[c] = (qn[c] - cv[c]) + penO[c];
        }
        diag_step<CPL, false>(p1, p2, de);
        diag_step<CPL, true>(p1, p2, dn);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            qv[c] = qn[c];
            cv[c] = cn[c];
        }
    };
    // blocks of 8 pairs without a branch; with ABANDON a test after each block
    int t = 0;
    for (; t + 8 <= m; t += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) pair(t + u);
        if (ABANDON) {
            if (key && (t & 31) == 24) {
                thr = fminf(thr0, threshold_of(__uint_as_float(kpend)));
                kpend = load_key_dist_bits(key);
            }
            bool any = false;
#pragma unroll
            for (int c = 0; c < CPL; ++c) any |= (float)fmin(p1[c], p2[c]) <= thr;
            if (__ballot(any) == 0) {
                alive = false;
                t += 8;
                break;
            }
        }
    }
    if (alive)
        for (; t < m; ++t) pair(t);
    pairs = t;
    // the last diagonal 2m - 2 has parity r & 1: odd r ends on the odd step (p1), even r on the even
    // step, which the loop's last odd step moved to p2
    F res = inf;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        if (c == (s0 >> 6)) res = (r & 1) ? p1[c] : p2[c];
    return lane_value(res, s0 & 63);
}

// Band cells (|i - j| <= r, 0 <= i, j < m) with i + j <= dl, summed over the wave's lanes (one
// anti-diagonal per lane and step); every lane gets the total.
__device__ inline unsigned long long band_cells_upto(int m, int r, long long dl) {
    unsigned long long n = 0;
    for (long long d = threadIdx.x & 63; d <= dl; d += 64) {
        long long lo = (d - r + 1) >> 1, hi = (d + r) >> 1;   // ceil((d-r)/2), floor((d+r)/2)
        if (lo < 0) lo = 0;
        if (lo < d - (m - 1)) lo = d - (m - 1);
        if (hi > m - 1) hi = m - 1;
        if (hi > d) hi = d;
        if (hi >= lo) n += (unsigned long long)(hi - lo + 1);
    }
    return wave_add_u64(n);
}

// The diagonal loop for the band's slot registers per lane, cpl = r / 64 + 1, rounded up to an
// instantiated count (extra slots lie outside the band and stay infinite).
template <int MAXCPL, bool ABANDON, typename F>
__device__ F diag_dispatch(int cpl, const F *qb, const F *cb, int m, int r, const uint64_t *key, float thr0,
                           bool &alive, int &pairs) {
    if constexpr (MAXCPL > 4) {
        if (cpl > 12) return diag_dtw<16, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
        if (cpl > 8) return diag_dtw<12, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
        if (cpl > 6) return diag_dtw<8, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
        if (cpl > 4) return diag_dtw<6, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
    }
    switch (cpl) {
    case 1: return diag_dtw<1, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
    case 2: return diag_dtw<2, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
    case 3: return diag_dtw<3, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
    default: return diag_dtw<4, ABANDON>(qb, cb, m, r, key, thr0, alive, pairs);
    }
}

// Pads around the staged arrays: query +big, candidate -big.
template <int MAXCPL, typename F>
__device__ inline void stage_pads(F *qb, F *cb, int m) {
    using P = DiagPads<MAXCPL>;
    const int lane = threadIdx.x & 63;
    const F big = DiagTraits<F>::big;
    for (int x = lane; x < P::QLo; x += 64) qb[x - P::QLo] = big;
    for (int x = lane; x < P::QHi; x += 64) qb[m + x] = big;
    for (int x = lane; x < P::CLo; x += 64) cb[x - P::CLo] = -big;
    for (int x = lane; x < P::CHi; x += 64) cb[m + x] = -big;
}

// Batched search, latency schedule: one wave per survivor of the round's list, used when the round
// has at most a.diag_max survivors (the lane-per-candidate kernels exit in that case).
template <bool PREFIX, int MAXCPL>
__global__ __launch_bounds__(128) void k_dtw_diag(BatchArgs a) {
    using P = DiagPads<MAXCPL>;
    extern __shared__ float lds_f[];
    if (*a.overflow) return;
    const uint32_t count = *a.surv_count;
    // small rounds: every survivor here; large rounds: only the wide-band bucket (112 <= r <= 1023),
    // read from its sorted segments, the other buckets go to the lane-per-candidate kernels
    const bool all = count <= a.diag_max;
    if (!all && !a.diag_wide) return;
    constexpr int cw = kMaxChunks + 1;
    const int64_t glo = all ? 0 : (int64_t)a.bucket_w[2 * cw] * 64;
    const int64_t ghi = all ? (int64_t)count : (int64_t)a.bucket_w[2 * cw + 1] * 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    float *qb = lds_f + (int64_t)wid * (2 * a.max_m + P::All) + P::QLo;
    float *cb = qb + a.max_m + P::QHi + P::CLo;
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0, n_lane_cells = 0;
    for (int64_t g = glo + wave; g < ghi; g += nwaves) {
        // wave-uniform values in scalar registers keep the diagonal loop uniform
        int q;
        int64_t start;
        if (all) {
            q = __builtin_amdgcn_readfirstlane(a.surv_q[g]);
            start = __builtin_amdgcn_readfirstlane(a.surv_i[g]);
        } else {
            int32_t wq0;
            q = __builtin_amdgcn_readfirstlane(wave_query(a, cw, g >> 6, wq0));
            if (((g >> 6) - wq0) * 64 + (g & 63) >= (int64_t)a.qcnt[q * kCntStride]) continue;
            start = __builtin_amdgcn_readfirstlane(a.sorted[g]);
        }
        const BatchQ bq = a.bq[q];
        const int m = __builtin_amdgcn_readfirstlane(bq.m), r = __builtin_amdgcn_readfirstlane(bq.r);
        float mu, s, o;
        if (PREFIX) {
            StatsPrefix{a.T, a.pre, m, 1.0 / m}(start, mu, s, o);
        } else {
            const int64_t so = bq.stat_slot * a.slot_stride;
            StatsArr{a.mu + so, a.s + so, a.o + so}(start, mu, s, o);
        }
        wave_sync();
        const float *qh = a.qpad + q * a.qstride + kQPad;
        const float *Tp = a.T + start;
        for (int x = lane; x < m; x += 64) {
            qb[x] = qh[x];
            cb[x] = fmaf(Tp[x] - mu, s, o);
        }
        stage_pads<MAXCPL>(qb, cb, m);
        wave_sync();
        const int cpl = (r >> 6) + 1;
        bool alive;
        int pairs;
        const float D = diag_dispatch<MAXCPL, true>(cpl, qb, cb, m, r, a.keys + q, INFINITY, alive, pairs);
        ++n_started;
        n_lane_cells += (unsigned long long)pairs * 2 * 64 * cpl;
        if (!alive) ++n_aband;
        if (a.counters) n_cells += band_cells_upto(m, r, 2LL * pairs - 1 - (r & 1));
        if (alive && D <= threshold_of(load_bsf(a.keys + q)) && lane == 0) {
            atomicMin((unsigned long long *)(a.keys + q), (unsigned long long)pack_key(D, (uint32_t)start));
            const uint32_t pos = atomicAdd(a.nb_count, 1u);
            if (pos < a.nb_cap) {
                a.nb_d[pos] = D;
                a.nb_idx[pos] = (uint32_t)start;
                a.nb_q[pos] = q;
            }
        }
    }
    if (a.counters && lane == 0) {
        atomicAdd(&a.counters[4], n_started);
        atomicAdd(&a.counters[5], n_aband);
        atomicAdd(&a.counters[6], n_cells);
        atomicAdd(&a.counters[8], n_lane_cells);
        atomicAdd(&a.counters[10], n_cells);
    }
}

// FP64 certification, one wave per selected near-best candidate: two-pass FP64 normalisation of the
// window, then the exact (non-abandoning) recurrence in FP64.
template <int MAXCPL>
__global__ __launch_bounds__(64) void k_cert_diag(BatchArgs a) {
    using P = DiagPads<MAXCPL>;
    extern __shared__ double lds_d[];
    const uint32_t cnt0 = *a.cert_count;
    const uint32_t cnt = cnt0 < a.nb_cap ? cnt0 : a.nb_cap;
    const int lane = threadIdx.x & 63;
    double *qb = lds_d + P::QLo;
    double *cb = qb + a.max_m + P::QHi + P::CLo;
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int q = __builtin_amdgcn_readfirstlane(a.cert_q[e]);
        const BatchQ bq = a.bq[q];
        const int m = __builtin_amdgcn_readfirstlane(bq.m), r = __builtin_amdgcn_readfirstlane(bq.r);
        const float *wv = a.T + a.cert_idx[e];
        double s = 0.0;
        for (int x = lane; x < m; x += 64) s += (double)wv[x];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        const double mu = s / m;
        double v = 0.0;
        for (int x = lane; x < m; x += 64) {
            const double dd = (double)wv[x] - mu;
            v += dd * dd;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        const double sigma = sqrt(v / m);
        const bool flat = sigma <= kSigmaFlat;
        wave_sync();
        const double *qsrc = a.qhat64 + (int64_t)q * a.max_m;
        for (int x = lane; x < m; x += 64) {
            qb[x] = qsrc[x];
            cb[x] = flat ? 0.0 : ((double)wv[x] - mu) / sigma;
        }
        stage_pads<MAXCPL>(qb, cb, m);
        wave_sync();
        bool alive;
        int pairs;
        const double D = diag_dispatch<MAXCPL, false>((r >> 6) + 1, qb, cb, m, r, nullptr, INFINITY, alive,
                                                           pairs);
        if (lane == 0) a.cert_d[e] = D;
    }
}

// Two-pass FP64 mean and sigma of the window by the whole wave, as FP32 normalisation parameters
// (c_j = fma(T[i+j] - mu, s, o), see norm_params).
__device__ inline void wave_norm(const float *w, int m, float &mu, float &s, float &o) {
    const int lane = threadIdx.x & 63;
    double sum = 0.0;
    for (int x = lane; x < m; x += 64) sum += (double)w[x];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    const double mu64 = sum / m;
    double v = 0.0;
    for (int x = lane; x < m; x += 64) {
        const double d = (double)w[x] - mu64;
        v += d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    norm_params(mu64, sqrt(v / m), mu, s, o);
}

// Normalisation parameters of the windows at starts[k] (one wave per start, coalesced loads, FP64
// two-pass), so that the one-lane-per-candidate DTW kernel reads them instead of normalising each
// window in its own lane; starts outside [0, n-m] get zeros (the DTW kernel rejects them).
__global__ __launch_bounds__(256) void k_start_stats(const float *T, int64_t n, int m, const int64_t *starts,
                                                     int64_t count, float *mu, float *sg, float *off) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k = wave; k < count; k += nwaves) {
        const int64_t st = starts[k];
        float a = 0.0f, b = 0.0f, c = 0.0f;
        if (st >= 0 && st <= n - m) wave_norm(T + st, m, a, b, c);
        if (lane == 0) {
            mu[k] = a;
            sg[k] = b;
            off[k] = c;
        }
    }
}

hipError_t launch_start_stats(const float *T, int64_t n, int m, const int64_t *starts, int64_t count, float *mu,
                              float *sg, float *off, int num_cu, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 3) / 4;
    if (blocks > (int64_t)num_cu * 16) blocks = (int64_t)num_cu * 16;
    hipLaunchKernelGGL(k_start_stats, dim3((unsigned)blocks), dim3(256), 0, s, T, n, m, starts, count, mu, sg, off);
    return hipGetLastError();
}

// Plain search and the stage entry point: one wave per start of a DtwArgs list (explicit starts,
// device-side survivors, a range or a single start).  In search mode with a device-side count,
// rounds of more than a.diag_max survivors are left to the lane-per-candidate kernels.
template <bool SEARCH, int MAXCPL>
__global__ __launch_bounds__(128) void k_dtw_diag_list(DtwArgs a) {
    using P = DiagPads<MAXCPL>;
    extern __shared__ float lds_f[];
    int64_t count = a.single >= 0 ? 1 : (a.count_dev ? (int64_t)*a.count_dev : a.count);
    if (a.count_dev && count > a.count) count = a.count;
    if (SEARCH && a.count_dev && count > (int64_t)a.diag_max) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int m = a.m, r = a.r;
    float *qb = lds_f + (int64_t)wid * (2 * m + P::All) + P::QLo;
    float *cb = qb + m + P::QHi + P::CLo;
    const float *qh = a.qpad + kQPad;
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0, n_lane_cells = 0;
    for (int64_t k = wave; k < count; k += nwaves) {
        int64_t start = a.single >= 0 ? a.single
                        : a.starts32 ? (int64_t)a.starts32[k]
                        : a.starts64 ? a.starts64[k] : a.range_first + k;
        start = (int64_t)__builtin_amdgcn_readfirstlane((int)start);
        if (start < 0 || start > a.n - m) {
            if (!SEARCH && lane == 0) a.dist_out[k] = NAN;
            continue;
        }
        float mu, s, o;
        if (a.mu) {
            mu = a.mu[start];
            s = a.s[start];
            o = a.o[start];
        } else {
            wave_norm(a.T + start, m, mu, s, o);
        }
        wave_sync();
        const float *Tp = a.T + start;
        for (int x = lane; x < m; x += 64) {
            qb[x] = qh[x];
            cb[x] = fmaf(Tp[x] - mu, s, o);
        }
        stage_pads<MAXCPL>(qb, cb, m);
        wave_sync();
        bool alive;
        int pairs;
        const float D = diag_dispatch<MAXCPL, true>((r >> 6) + 1, qb, cb, m, r, SEARCH ? a.key : nullptr,
                                                         SEARCH ? INFINITY : a.abandon_at, alive, pairs);
        if (SEARCH) {
            ++n_started;
            n_lane_cells += (unsigned long long)pairs * 2 * 64 * ((r >> 6) + 1);
            if (!alive) ++n_aband;
            if (a.counters) n_cells += band_cells_upto(m, r, 2LL * pairs - 1 - (r & 1));
            if (alive && D <= threshold_of(load_bsf(a.key)) && lane == 0) {
                atomicMin((unsigned long long *)a.key, (unsigned long long)pack_key(D, (uint32_t)start));
                const uint32_t pos = atomicAdd(a.nb_count, 1u);
                if (pos < a.nb_cap) {
                    a.nb_d[pos] = D;
                    a.nb_idx[pos] = (uint32_t)start;
                }
            }
        } else if (lane == 0) {
            a.dist_out[k] = alive ? D : INFINITY;
        }
    }
    if (SEARCH && a.counters && lane == 0) {
        atomicAdd(&a.counters[4], n_started);
        atomicAdd(&a.counters[5], n_aband);
        atomicAdd(&a.counters[6], n_cells);
        atomicAdd(&a.counters[8], n_lane_cells);
        atomicAdd(&a.counters[10], n_cells);
    }
}

// FP64 certification of the plain path, one wave per selected candidate.
template <int MAXCPL>
__global__ __launch_bounds__(64) void k_cert_diag_list(CertArgs c) {
    using P = DiagPads<MAXCPL>;
    extern __shared__ double lds_d[];
    const uint32_t cnt0 = *c.cert_count;
    const uint32_t cnt = cnt0 < c.nb_cap ? cnt0 : c.nb_cap;
    const int lane = threadIdx.x & 63;
    const int m = c.m, r = c.r;
    double *qb = lds_d + P::QLo;
    double *cb = qb + m + P::QHi + P::CLo;
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const float *wv = c.T + __builtin_amdgcn_readfirstlane((int)c.cert_idx[e]);
        double sum = 0.0;
        for (int x = lane; x < m; x += 64) sum += (double)wv[x];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        const double mu = sum / m;
        double v = 0.0;
        for (int x = lane; x < m; x += 64) {
            const double dd = (double)wv[x] - mu;
            v += dd * dd;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        const double sigma = sqrt(v / m);
        const bool flat = sigma <= kSigmaFlat;
        wave_sync();
        for (int x = lane; x < m; x += 64) {
            qb[x] = c.qhat64[x];
            cb[x] = flat ? 0.0 : ((double)wv[x] - mu) / sigma;
        }
        stage_pads<MAXCPL>(qb, cb, m);
        wave_sync();
        bool alive;
        int pairs;
        const double D = diag_dispatch<MAXCPL, false>((r >> 6) + 1, qb, cb, m, r, nullptr, INFINITY, alive,
                                                           pairs);
        if (lane == 0) c.cert_d[e] = D;
    }
}

// the instance for a launch's widest band
static bool diag_wide_of(int max_r) { return max_r > kDiagMaxBandNarrow; }

hipError_t launch_dtw_diag_list(const DtwArgs &a, bool search, int blocks, hipStream_t s) {
    const size_t shm = 2 * diag_lds_bytes(a.m, false, a.r);
    if (diag_wide_of(a.r)) {
        if (search)
            hipLaunchKernelGGL((k_dtw_diag_list<true, 16>), dim3(blocks), dim3(128), shm, s, a);
        else
            hipLaunchKernelGGL((k_dtw_diag_list<false, 16>), dim3(blocks), dim3(128), shm, s, a);
    } else {
        if (search)
            hipLaunchKernelGGL((k_dtw_diag_list<true, 4>), dim3(blocks), dim3(128), shm, s, a);
        else
            hipLaunchKernelGGL((k_dtw_diag_list<false, 4>), dim3(blocks), dim3(128), shm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_cert_diag_list(const CertArgs &c, int blocks, hipStream_t s) {
    const size_t shm = diag_lds_bytes(c.m, true, c.r);
    if (diag_wide_of(c.r))
        hipLaunchKernelGGL(k_cert_diag_list<16>, dim3(blocks), dim3(64), shm, s, c);
    else
        hipLaunchKernelGGL(k_cert_diag_list<4>, dim3(blocks), dim3(64), shm, s, c);
    return hipGetLastError();
}

size_t diag_lds_bytes(int max_m, bool fp64, int max_r) {
    const int pads = diag_wide_of(max_r) ? DiagPads<16>::All : DiagPads<4>::All;
    return (size_t)(2 * max_m + pads) * (fp64 ? sizeof(double) : sizeof(float));
}

hipError_t launch_dtw_diag(const BatchArgs &a, bool prefix, int max_r, int blocks, hipStream_t s) {
    const size_t shm = 2 * diag_lds_bytes(a.max_m, false, max_r);
    if (diag_wide_of(max_r)) {
        if (prefix)
            hipLaunchKernelGGL((k_dtw_diag<true, 16>), dim3(blocks), dim3(128), shm, s, a);
        else
            hipLaunchKernelGGL((k_dtw_diag<false, 16>), dim3(blocks), dim3(128), shm, s, a);
    } else {
        if (prefix)
            hipLaunchKernelGGL((k_dtw_diag<true, 4>), dim3(blocks), dim3(128), shm, s, a);
        else
            hipLaunchKernelGGL((k_dtw_diag<false, 4>), dim3(blocks), dim3(128), shm, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_cert_diag(const BatchArgs &a, int max_r, int blocks, hipStream_t s) {
    const size_t shm = diag_lds_bytes(a.max_m, true, max_r);
    if (diag_wide_of(max_r))
        hipLaunchKernelGGL(k_cert_diag<16>, dim3(blocks), dim3(64), shm, s, a);
    else
        hipLaunchKernelGGL(k_cert_diag<4>, dim3(blocks), dim3(64), shm, s, a);
    return hipGetLastError();
}

}  // namespace dtws
