// Banded DTW (eq. (dtw) with the Sakoe-Chiba band of Section 2.1), the best-so-far update
// (eq. (bsf)) and the FP64 certification of the near-best candidates.
//
// Register kernel (band width 2r+1 <= 16 * kMaxChunks): one lane per candidate.  The DP is swept
// column by column over the candidate (DTW is symmetric in its operands, so sweeping the
// candidate index as the outer loop computes the same d(m,m)).  For column j the lane keeps the
// cells of rows i = j - R + k, k in [0, 16*NC), in a register array a[k], where R = 8*NC - 1 is a
// compile-time centre (band r <= R); updating in place in ascending k uses a[k] = d(i-1, j-1),
// a[k+1] = d(i, j-1) and the cell just written below, d(i-1, j):
//     a[k] <- (q_{j-R+k} - c_j)^2 + min(a[k], a[k+1], a[k-1]_new).
// Cells with |k - R| > r lie outside the band: the lanes that supply their query values read the
// sentinel padding instead, so they cost +inf.  With the centre fixed at compile time the start
// cell d(-1,-1) = 0 sits at a[R] before column 0 and the result d(m-1, m-1) at a[R] after the
// last column.
// The query window q_{j-R+k} is the same for every lane of the wave; it is loaded 16 values at
// a time, one value per lane of each 16-lane row, and broadcast to the row with DPP
// row_newbcast, so each cell costs one v_sub, one v_min3 and one v_fma.  Rows outside [0, m) and
// cells above the band read the sentinel query value and cost +inf, which keeps the loop free
// of branches.  A lane is abandoned when every cell of a column exceeds the threshold: every
// warping path crosses every column and costs are non-negative.
#include <utility>

#include "device.h"

namespace dtws {

template <int NC, bool SEARCH>
__global__ __launch_bounds__(256) void k_dtw(DtwArgs a) {
    constexpr int W = 16 * NC;
    extern __shared__ float bound_lds[];   // [kBoundBlocks][256] when the suffix bound is on
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t count = a.single >= 0 ? 1 : (a.count_dev ? (int64_t)*a.count_dev : a.count);
    if (a.count_dev && count > a.count) count = a.count;
    if (SEARCH && a.count_dev && count <= (int64_t)a.diag_max) return;   // the one-wave kernel's round
    const int m = a.m, r = a.r;
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0, n_lane_cells = 0;

    for (int64_t base = wave * 64; base < count; base += nwaves * 64) {
        const int64_t k = base + lane;
        const bool valid = k < count;
        int64_t start = 0;
        bool bad = false;
        if (valid) {
            start = a.single >= 0 ? a.single
                    : a.starts32 ? (int64_t)a.starts32[k]
                    : a.starts64 ? a.starts64[k] : a.range_first + k;
            bad = start < 0 || start > a.n - m;
            if (bad) start = 0;
        }
        float mu, s, o;
        if (a.mu) {
            const int64_t si = a.stats_by_k ? (valid ? k : 0) : start;
            mu = a.mu[si];
            s = a.s[si];
            o = a.o[si];
        } else {
            lane_stats(a.T + start, m, mu, s, o);
        }
        const float *sfx = nullptr;
        int G = 16;
        if constexpr (NC >= kBoundMinNC) {
            if (a.Un) {
                G = bound_block(m);
                bound_suffix(a.T + start, mu, s, o, a.Un, a.Ln, m, G, bound_lds + threadIdx.x);
                sfx = bound_lds + threadIdx.x;
            }
        }
        bool alive;
        float D;
        int jdead, jrun;
        dtw_lanes<NC>(a.T, start, mu, s, o, a.qpad, m, r, valid && !bad, SEARCH ? a.key : nullptr,
                      SEARCH ? INFINITY : a.abandon_at, alive, D, jdead, jrun, sfx, G);
        n_lane_cells += (unsigned long long)jrun * W;
        if (SEARCH) {
            if (valid && !bad) {
                ++n_started;
                if (jdead < m) ++n_aband;
                n_cells += band_cells(m, r, jdead);
            }
            if (valid && !bad && alive) {
                atomicMin((unsigned long long *)a.key, (unsigned long long)pack_key(D, (uint32_t)start));
                const uint32_t pos = atomicAdd(a.nb_count, 1u);
                if (pos < a.nb_cap) {
                    a.nb_d[pos] = D;
                    a.nb_idx[pos] = (uint32_t)start;
                }
            }
        } else if (valid) {
            a.dist_out[k] = bad ? NAN : (alive ? D : INFINITY);
        }
    }
    if (SEARCH && a.counters) {
        n_started = wave_add(n_started);
        n_aband = wave_add(n_aband);
        n_cells = wave_add(n_cells);
        n_lane_cells = wave_add(n_lane_cells);
        if (lane == 0) {
            atomicAdd(&a.counters[4], n_started);
            atomicAdd(&a.counters[5], n_aband);
            atomicAdd(&a.counters[6], n_cells);
            atomicAdd(&a.counters[8], n_lane_cells);
        }
    }
}

// Wide-band fallback (2r+1 > 16 * kMaxChunks): one lane per candidate, rows of the DP in global
// scratch (two rows of m+1 floats per lane), row-by-row sweep as in eq. (dtw).
template <bool SEARCH>
__global__ __launch_bounds__(64) void k_dtw_wide(DtwArgs a, float *rows, int64_t nlanes) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nlanes) return;
    int64_t count = a.single >= 0 ? 1 : (a.count_dev ? (int64_t)*a.count_dev : a.count);
    if (a.count_dev && count > a.count) count = a.count;
    if (SEARCH && a.count_dev && count <= (int64_t)a.diag_max) return;   // the one-wave kernel's round
    const int m = a.m, r = a.r;
    const float *qh = a.qpad + kQPad;
    float *prev = rows + g * 2 * (int64_t)(m + 1), *cur = prev + (m + 1);
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0;
    for (int64_t k = g; k < count; k += nlanes) {
        int64_t start = a.single >= 0 ? a.single
                        : a.starts32 ? (int64_t)a.starts32[k]
                        : a.starts64 ? a.starts64[k] : a.range_first + k;
        if (start < 0 || start > a.n - m) {
            if (!SEARCH) a.dist_out[k] = NAN;
            continue;
        }
        float mu, s, o;
        if (a.mu) {
            mu = a.mu[start];
            s = a.s[start];
            o = a.o[start];
        } else {
            lane_stats(a.T + start, m, mu, s, o);
        }
        const float *Tp = a.T + start;
        float thr = SEARCH ? threshold_of(load_bsf(a.key)) : a.abandon_at;
        for (int x = 0; x <= m; ++x) {
            prev[x] = INFINITY;
            cur[x] = INFINITY;
        }
        prev[0] = 0.0f;
        bool alive = true;
        int idead = m;
        for (int i = 1; i <= m; ++i) {
            const int jlo = i - r < 1 ? 1 : i - r, jhi = i + r > m ? m : i + r;
            cur[jlo - 1] = INFINITY;
            if (jhi + 1 <= m) cur[jhi + 1] = INFINITY;
            const float qi = qh[i - 1];
            float rowmin = INFINITY;
            for (int jj = jlo; jj <= jhi; ++jj) {
                const float c = fmaf(Tp[jj - 1] - mu, s, o);
                const float diff = qi - c;
                const float v = fmaf(diff, diff, fminf(fminf(prev[jj], cur[jj - 1]), prev[jj - 1]));
                cur[jj] = v;
                rowmin = fminf(rowmin, v);
            }
            float *t = prev;
            prev = cur;
            cur = t;
            if ((i & 15) == 0 && SEARCH) thr = threshold_of(load_bsf(a.key));
            if (rowmin > thr) {
                alive = false;
                idead = i;
                break;
            }
        }
        const float D = alive ? prev[m] : INFINITY;   // after the last swap, prev holds row m
        // restore the row roles for the next candidate
        prev = rows + g * 2 * (int64_t)(m + 1);
        cur = prev + (m + 1);
        if (SEARCH) {
            ++n_started;
            if (!alive) ++n_aband;
            n_cells += band_cells(m, r, alive ? m : idead);
            if (alive && D <= thr) {
                atomicMin((unsigned long long *)a.key, (unsigned long long)pack_key(D, (uint32_t)start));
                const uint32_t pos = atomicAdd(a.nb_count, 1u);
                if (pos < a.nb_cap) {
                    a.nb_d[pos] = D;
                    a.nb_idx[pos] = (uint32_t)start;
                }
            }
        } else {
            a.dist_out[k] = D;
        }
    }
    if (SEARCH && a.counters) {
        atomicAdd(&a.counters[4], n_started);
        atomicAdd(&a.counters[5], n_aband);
        atomicAdd(&a.counters[6], n_cells);
        atomicAdd(&a.counters[8], n_cells);
    }
}

// ------------------------------------------------------------------ small fills
// Plain fill kernels instead of hipMemsetAsync, so the same calls can later be captured in a graph.
__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

// Start of a batched search in one launch: empty best-so-far keys, zero counters, work-queue heads,
// near-best and certification counts and the overflow flag.
__global__ void k_reset_batch(uint64_t *keys, int nq, unsigned long long *counters, int ncounters, uint32_t *heads,
                              int nheads, uint32_t *nb_count, uint32_t *cert_count, uint32_t *overflow) {
    for (int i = threadIdx.x; i < nq; i += blockDim.x) keys[i] = kEmptyKey;
    for (int i = threadIdx.x; i < ncounters; i += blockDim.x) counters[i] = 0ull;
    for (int i = threadIdx.x; i < nheads; i += blockDim.x) heads[i] = 0u;
    if (threadIdx.x == 0) {
        *nb_count = 0u;
        *cert_count = 0u;
        *overflow = 0u;
    }
}

hipError_t launch_reset_batch(uint64_t *keys, int nq, unsigned long long *counters, int ncounters, uint32_t *heads,
                              int nheads, uint32_t *nb_count, uint32_t *cert_count, uint32_t *overflow, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_batch, dim3(1), dim3(256), 0, s, keys, nq, counters, ncounters, heads, nheads, nb_count,
                       cert_count, overflow);
    return hipGetLastError();
}

// ------------------------------------------------------------------ best-so-far update
__global__ __launch_bounds__(256) void k_bsf_update(uint64_t *keys, const float *d, const int64_t *idx,
                                                    int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const int64_t k = base + threadIdx.x;
        unsigned long long key = ~0ull;
        if (k < count) key = pack_key(d[k], (uint32_t)idx[k]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off, 64);
            key = o < key ? o : key;
        }
        if ((threadIdx.x & 63) == 0) atomicMin((unsigned long long *)keys, key);
    }
}

// ------------------------------------------------------------------ FP64 certification


__global__ __launch_bounds__(256) void k_certify(CertArgs c) {
    __shared__ double sd[256];
    __shared__ uint32_t si[256];
    __shared__ unsigned int s_cert;
    const int tid = threadIdx.x;
    if (tid == 0) s_cert = 0;
    __syncthreads();
    const float thr = threshold_of(key_dist(*c.key));
    const uint32_t total = *c.nb_count;
    const uint32_t cnt = total < c.nb_cap ? total : c.nb_cap;
    const int m = c.m, r = c.r;
    double *ch = c.scratch + (int64_t)tid * 3 * (m + 1);
    double *prev = ch + m, *cur = prev + (m + 1);
    double best = INFINITY;
    uint32_t bidx = 0xffffffffu;
    for (uint32_t e = tid; e < cnt; e += blockDim.x) {
        if (!(c.nb_d[e] <= thr)) continue;
        atomicAdd(&s_cert, 1u);
        const uint32_t idx = c.nb_idx[e];
        const float *wv = c.T + idx;
        double sum = 0.0;
        for (int j = 0; j < m; ++j) sum += (double)wv[j];
        const double mu = sum / m;
        double v = 0.0;
        for (int j = 0; j < m; ++j) {
            const double d = (double)wv[j] - mu;
            v += d * d;
        }
        const double sigma = sqrt(v / m);
        const bool flat = sigma <= kSigmaFlat;
        for (int j = 0; j < m; ++j) ch[j] = flat ? 0.0 : ((double)wv[j] - mu) / sigma;
        for (int x = 0; x <= m; ++x) {
            prev[x] = INFINITY;
            cur[x] = INFINITY;
        }
        prev[0] = 0.0;
        double *P = prev, *C = cur;
        for (int i = 1; i <= m; ++i) {
            const int jlo = i - r < 1 ? 1 : i - r, jhi = i + r > m ? m : i + r;
            C[jlo - 1] = INFINITY;
            if (jhi + 1 <= m) C[jhi + 1] = INFINITY;
            const double qi = c.qhat64[i - 1];
            for (int jj = jlo; jj <= jhi; ++jj) {
                const double diff = qi - ch[jj - 1];
                const double a1 = P[jj], a2 = C[jj - 1], a3 = P[jj - 1];
                double mn = a1 < a2 ? a1 : a2;
                mn = mn < a3 ? mn : a3;
                C[jj] = __dadd_rn(__dmul_rn(diff, diff), mn);
            }
            double *t = P;
            P = C;
            C = t;
        }
        const double d = P[m];
        if (d < best || (d == best && idx < bidx)) {
            best = d;
            bidx = idx;
        }
    }
    sd[tid] = best;
    si[tid] = bidx;
    __syncthreads();
    if (tid == 0) {
        double bd = INFINITY;
        uint32_t bi = 0xffffffffu;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            if (sd[t] < bd || (sd[t] == bd && si[t] < bi)) {
                bd = sd[t];
                bi = si[t];
            }
        }
        *c.res_idx = bi == 0xffffffffu ? -1 : (int64_t)bi;
        *c.res_dist = bd;
        *c.res_status = total > c.nb_cap ? DTWS_EOVERFLOW : (bi == 0xffffffffu ? DTWS_EHIP : DTWS_OK);
        if (c.counters) atomicAdd(&c.counters[7], (unsigned long long)s_cert);
    }
}

// ------------------------------------------------------------------ block-parallel certification
// The qualifying near-best candidates (D32 <= threshold of the final best-so-far) are compacted,
// then one block per candidate evaluates eq. (dtw) in FP64 along anti-diagonals a = i + j: all
// cells of one anti-diagonal depend only on the two previous ones, so the block's threads split
// each anti-diagonal and synchronise between anti-diagonals.  Anti-diagonals are kept in a ring
// of three row-indexed buffers of length L = r + 4 in LDS, next to the normalised query and
// candidate (FP64, two-pass statistics as in eq. (Normalization1)).
constexpr int kCertBlocks = 64;
constexpr int kCertThreads = 256;

__global__ __launch_bounds__(256) void k_cert_select(CertArgs c) {
    const float thr = threshold_of(key_dist(*c.key));
    const uint32_t total = *c.nb_count;
    const uint32_t cnt = total < c.nb_cap ? total : c.nb_cap;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        if (c.nb_d[e] <= thr) {
            const uint32_t pos = atomicAdd(c.cert_count, 1u);
            if (pos < c.nb_cap) c.cert_idx[pos] = c.nb_idx[e];
        }
    }
}

__device__ inline double block_sum64(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

__global__ __launch_bounds__(kCertThreads) void k_cert_dtw(CertArgs c) {
    extern __shared__ double sm[];
    __shared__ double red[kCertThreads / 64];
    const int m = c.m, r = c.r, L = r + 4;
    double *qh = sm, *ch = sm + m, *ring = sm + 2 * m;   // ring: 3 x L
    const uint32_t cnt0 = *c.cert_count;
    const uint32_t cnt = cnt0 < c.nb_cap ? cnt0 : c.nb_cap;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int j = tid; j < m; j += nt) qh[j] = c.qhat64[j];
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const uint32_t idx = c.cert_idx[e];
        const float *wv = c.T + idx;
        double s = 0.0;
        for (int j = tid; j < m; j += nt) s += (double)wv[j];
        const double mu = block_sum64(s, red) / m;
        double v = 0.0;
        for (int j = tid; j < m; j += nt) {
            const double dd = (double)wv[j] - mu;
            v += dd * dd;
        }
        const double sigma = sqrt(block_sum64(v, red) / m);
        const bool flat = sigma <= kSigmaFlat;
        for (int j = tid; j < m; j += nt) ch[j] = flat ? 0.0 : ((double)wv[j] - mu) / sigma;
        __syncthreads();
        // anti-diagonal a holds rows i in [lo(a), hi(a)]: |2i - a| <= r, 0 <= i, a - i < m
        for (int a = 0; a <= 2 * (m - 1); ++a) {
            int lo = (a - r + 1) >> 1;          // ceil((a - r) / 2) for a - r >= -1
            if (a - r < 0) lo = -((r - a) >> 1);
            if (lo < a - (m - 1)) lo = a - (m - 1);
            if (lo < 0) lo = 0;
            int hi = (a + r) >> 1;
            if (hi > a) hi = a;
            if (hi > m - 1) hi = m - 1;
            double *cur = ring + (a % 3) * L, *p1 = ring + ((a + 2) % 3) * L, *p2 = ring + ((a + 1) % 3) * L;
            for (int i = lo + tid; i <= hi; i += nt) {
                const int j = a - i;
                const double diff = qh[i] - ch[j];
                double best;
                if (a == 0) {
                    best = 0.0;
                } else {
                    // predecessors; a cell is readable iff it lies in the band and the grid
                    const double up = (i >= 1 && (i - 1) - j <= r && j - (i - 1) <= r) ? p1[(i - 1) % L] : INFINITY;
                    const double left = (j >= 1 && i - (j - 1) <= r && (j - 1) - i <= r) ? p1[i % L] : INFINITY;
                    const double dg = (i >= 1 && j >= 1) ? p2[(i - 1) % L] : INFINITY;
                    best = up < left ? up : left;
                    best = best < dg ? best : dg;
                }
                cur[i % L] = __dadd_rn(__dmul_rn(diff, diff), best);
            }
            __syncthreads();
        }
        if (tid == 0) {
            c.cert_d[e] = ring[((2 * (m - 1)) % 3) * L + (m - 1) % L];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_cert_reduce(CertArgs c) {
    __shared__ double sd[256];
    __shared__ uint32_t si[256];
    const uint32_t cnt0 = *c.cert_count;
    const uint32_t cnt = cnt0 < c.nb_cap ? cnt0 : c.nb_cap;
    double best = INFINITY;
    uint32_t bidx = 0xffffffffu;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const double d = c.cert_d[e];
        const uint32_t idx = c.cert_idx[e];
        if (d < best || (d == best && idx < bidx)) {
            best = d;
            bidx = idx;
        }
    }
    sd[threadIdx.x] = best;
    si[threadIdx.x] = bidx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < (int)blockDim.x; ++t)
            if (sd[t] < best || (sd[t] == best && si[t] < bidx)) {
                best = sd[t];
                bidx = si[t];
            }
        *c.res_idx = bidx == 0xffffffffu ? -1 : (int64_t)bidx;
        *c.res_dist = best;
        const bool overflow = *c.nb_count > c.nb_cap || cnt0 > c.nb_cap;
        *c.res_status = overflow ? DTWS_EOVERFLOW : (bidx == 0xffffffffu ? DTWS_EHIP : DTWS_OK);
        if (c.counters) atomicAdd(&c.counters[7], (unsigned long long)cnt);
    }
}

// ------------------------------------------------------------------ launchers
template <bool SEARCH>
static hipError_t launch_dtw_t(const DtwArgs &a, int64_t max_count, int num_cu, float *wide_rows,
                               int64_t wide_lanes, hipStream_t s) {
    if (max_count <= 0) return hipSuccess;
    const int nc = (a.r + 1 + 7) / 8;   // smallest NC with 8*NC - 1 >= r
    if (nc > kMaxChunks) {
        int64_t lanes = wide_lanes;
        if (lanes > max_count) lanes = max_count;
        const int64_t blocks = (lanes + 63) / 64;
        hipLaunchKernelGGL(k_dtw_wide<SEARCH>, dim3((unsigned)blocks), dim3(64), 0, s, a, wide_rows, lanes);
        return hipGetLastError();
    }
    int64_t blocks = (max_count + 255) / 256;
    // narrow bands (a few registers per lane) run more waves per SIMD to cover their loads' latency
    const int64_t cap = (int64_t)num_cu * (nc <= 3 ? 16 : 4);
    if (blocks > cap) blocks = cap;
    const dim3 g((unsigned)blocks), b(256);
    switch (nc) {
#define DTWS_CASE(N) \
    case N: hipLaunchKernelGGL((k_dtw<N, SEARCH>), g, b, N >= kBoundMinNC && a.Un ? kBoundLdsBytes : 0, s, a); break;
        DTWS_CASE(1) DTWS_CASE(2) DTWS_CASE(3) DTWS_CASE(4) DTWS_CASE(5) DTWS_CASE(6) DTWS_CASE(7)
        DTWS_CASE(8) DTWS_CASE(9) DTWS_CASE(10) DTWS_CASE(11) DTWS_CASE(12) DTWS_CASE(13) DTWS_CASE(14)
#undef DTWS_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dtw(const DtwArgs &a, bool search, int64_t max_count, int num_cu, float *wide_rows,
                      int64_t wide_lanes, hipStream_t s) {
    return search ? launch_dtw_t<true>(a, max_count, num_cu, wide_rows, wide_lanes, s)
                  : launch_dtw_t<false>(a, max_count, num_cu, wide_rows, wide_lanes, s);
}

hipError_t launch_bsf_update(uint64_t *keys, const float *d, const int64_t *idx, int64_t count, int num_cu,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > num_cu * 8) blocks = num_cu * 8;
    hipLaunchKernelGGL(k_bsf_update, dim3((unsigned)blocks), dim3(256), 0, s, keys, d, idx, count);
    return hipGetLastError();
}

hipError_t launch_certify(const CertArgs &c, hipStream_t s) {
    const size_t shm = sizeof(double) * (2 * (size_t)c.m + 3 * (size_t)(c.r + 4));
    if (shm > 60 * 1024 || !c.cert_idx) {
        // very wide bands: one thread per candidate with rows in global scratch
        hipLaunchKernelGGL(k_certify, dim3(1), dim3(256), 0, s, c);
        return hipGetLastError();
    }
    hipError_t e = launch_fill_u32(c.cert_count, 0, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cert_select, dim3(1), dim3(256), 0, s, c);
    if (c.r <= kDiagMaxBand) {
        e = launch_cert_diag_list(c, kCertBlocks, s);   // one wave per candidate along anti-diagonals
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_cert_dtw, dim3(kCertBlocks), dim3(kCertThreads), shm, s, c);
    }
    hipLaunchKernelGGL(k_cert_reduce, dim3(1), dim3(256), 0, s, c);
    return hipGetLastError();
}

}  // namespace dtws
