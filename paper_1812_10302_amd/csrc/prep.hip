// Query preparation, per-window normalisation statistics and the raw-series envelope.
//
//  k_query_prep   eq. (Normalization1) for the query, eq. (envelope) of the normalised query,
//                 and the order in which the LB_Keogh sums visit query positions.
//  k_znorm_stats  mean / population sigma of every length-m window (eq. (Normalization1)),
//                 from FP64 prefix sums of the series anchored at each tile's first point.
//  k_series_env   max / min of the raw series over [k-r, k+r] clipped to the series; mapped
//                 through a candidate's normalisation this envelope contains the candidate's
//                 own envelope (eq. (envelope) applied to the candidate), so LB_Keogh against
//                 it (eq. (LBKeoghEQ)) is a valid, slightly looser bound.
#include "dtws_internal.h"

namespace dtws {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a block of `nthreads` threads (multiple of 64); `red` holds nthreads/64 doubles.
__device__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// Ordering used to sort query positions: larger key first, lower position on ties.
__device__ inline bool before(float ka, int ia, float kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

// Sort key of query position j: the expected query-envelope LB_Keogh term (eq. (LBKeoghEC)) of a
// candidate value c ~ N(0, 1), which is what the points of a z-normalised window look like one at a
// time: E[(c - U)+^2] + E[(L - c)+^2] = (1 + U^2) Q(U) - U phi(U) + (1 + L^2) Q(-L) + L phi(L), with
// Q the standard normal upper tail and phi its density.  Visiting the positions in decreasing
// expected term lets a sum pass the threshold after fewer terms than visiting them by |qhat|
// alone, because a narrow envelope far from zero outweighs a large |qhat| inside a wide one.
__device__ inline float expected_term(float u, float l) {
    const float kInvSqrt2 = 0.70710678f, kInvSqrt2Pi = 0.39894228f;
    const float tu = 0.5f * erfcf(u * kInvSqrt2), tl = 0.5f * erfcf(-l * kInvSqrt2);
    const float pu = kInvSqrt2Pi * expf(-0.5f * u * u), pl = kInvSqrt2Pi * expf(-0.5f * l * l);
    return fmaxf(fmaf(1.0f + u * u, tu, -u * pu), 0.0f) + fmaxf(fmaf(1.0f + l * l, tl, l * pl), 0.0f);
}

}  // namespace

// ------------------------------------------------------------------ query preparation
__device__ void query_prep_body(const float *__restrict__ Q, int m, int r, const QueryBufs &b) {
    __shared__ double red[16];
    __shared__ float qh[kMaxM];
    __shared__ float U[kMaxM], L[kMaxM];
    __shared__ float skey[kMaxM];
    __shared__ int sidx[kMaxM];
    const int tid = threadIdx.x, nt = blockDim.x;

    double s = 0.0;
    for (int j = tid; j < m; j += nt) s += (double)Q[j];
    const double mu = block_sum(s, red) / m;
    double v = 0.0;
    for (int j = tid; j < m; j += nt) {
        const double d = (double)Q[j] - mu;
        v += d * d;
    }
    const double sigma = sqrt(block_sum(v, red) / m);
    const bool flat = sigma <= kSigmaFlat;
    for (int j = tid; j < m; j += nt) {
        const double z = flat ? 0.0 : ((double)Q[j] - mu) / sigma;
        b.qhat64[j] = z;
        qh[j] = (float)z;
    }
    __syncthreads();
    for (int x = tid; x < 2 * kQPad + m; x += nt)
        b.qpad[x] = (x >= kQPad && x < kQPad + m) ? qh[x - kQPad] : kSentinel;
    // envelope of the normalised query, windows clipped to [0, m)
    for (int j = tid; j < m; j += nt) {
        const int a = j - r < 0 ? 0 : j - r, e = j + r > m - 1 ? m - 1 : j + r;
        float u = qh[a], l = qh[a];
        for (int k = a + 1; k <= e; ++k) {
            u = fmaxf(u, qh[k]);
            l = fminf(l, qh[k]);
        }
        U[j] = u;
        L[j] = l;
        b.Unat[j] = u;
        b.Lnat[j] = l;
    }
    __syncthreads();
    // bitonic sort of positions by decreasing expected term (padding keys sort last)
    int P = 1;
    while (P < m) P <<= 1;
    for (int j = tid; j < P; j += nt) {
        skey[j] = j < m ? expected_term(U[j], L[j]) : -1.0f;
        sidx[j] = j;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = tid; t < P; t += nt) {
                const int o = t ^ jj;
                if (o > t) {
                    const bool up = (t & k) == 0;
                    const bool swap = up ? before(skey[o], sidx[o], skey[t], sidx[t])
                                         : before(skey[t], sidx[t], skey[o], sidx[o]);
                    if (swap) {
                        const float tk = skey[t];
                        skey[t] = skey[o];
                        skey[o] = tk;
                        const int ti = sidx[t];
                        sidx[t] = sidx[o];
                        sidx[o] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < m; k += nt) {
        const int j = sidx[k];
        b.order[k] = j;
        b.qsorted[k] = qh[j];
        b.Usorted[k] = U[j];
        b.Lsorted[k] = L[j];
    }
    // Pad to a multiple of 16 with neutral terms so the bound loops run whole blocks of 16: an
    // infinite query envelope adds nothing to the query-envelope bound, and a NaN query value
    // adds nothing to the data-envelope bound (max(NaN, x) = x under IEEE maxNum).
    const int mpad = (m + 15) & ~15;
    for (int k = m + tid; k < mpad; k += nt) {
        b.order[k] = 0;
        b.qsorted[k] = __builtin_nanf("");
        b.Usorted[k] = INFINITY;
        b.Lsorted[k] = -INFINITY;
    }
}

__global__ __launch_bounds__(1024) void k_query_prep(const float *__restrict__ Q, int m, int r, QueryBufs b) {
    query_prep_body(Q, m, r, b);
}

// One block per query of a batch: query k is Qp[qoff[k] .. qoff[k] + m_k).
__global__ __launch_bounds__(1024) void k_query_prep_batch(const float *__restrict__ Qp, const BatchQ *bq,
                                                           QueryBufs base, int64_t qstride, int64_t mstride,
                                                           int64_t m64stride) {
    const int k = blockIdx.x;
    const BatchQ q = bq[k];
    QueryBufs b;
    b.qpad = base.qpad + k * qstride;
    b.qhat64 = base.qhat64 + k * m64stride;
    b.qsorted = base.qsorted + k * mstride;
    b.Usorted = base.Usorted + k * mstride;
    b.Lsorted = base.Lsorted + k * mstride;
    b.Unat = base.Unat + k * mstride;
    b.Lnat = base.Lnat + k * mstride;
    b.order = base.order + k * mstride;
    query_prep_body(Qp + q.qoff, q.m, q.r, b);
}

// ------------------------------------------------------------------ window statistics
constexpr int kStatTile = 1024;   // candidates per block
constexpr int kStatThreads = 256; // 4 consecutive positions per thread

// Exclusive scan of 4 consecutive values per thread across the block; returns the block total.
__device__ inline void block_exscan4(double (&v)[4], double *wsum, double &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double run = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const double x = v[u];
        v[u] = run;
        run += x;
    }
    // inclusive wave scan of the per-thread totals
    double inc = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    double wbase = 0.0;
    total = 0.0;
    for (int w = 0; w < kStatThreads / 64; ++w) {
        if (w < wid) wbase += wsum[w];
        total += wsum[w];
    }
    const double tbase = wbase + inc - run;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] += tbase;
}

template <bool EXPORT>
__global__ __launch_bounds__(kStatThreads) void k_znorm_stats(const float *__restrict__ T, int64_t n, int m,
                                                              int64_t N, double *__restrict__ mu_out,
                                                              double *__restrict__ sg_out, float *__restrict__ mu32,
                                                              float *__restrict__ s32, float *__restrict__ o32) {
    __shared__ double Pa1[kStatTile + 1], Pa2[kStatTile + 1], Pb1[kStatTile], Pb2[kStatTile];
    __shared__ double wsum[8], red[8];
    const int64_t c0 = (int64_t)blockIdx.x * kStatTile;
    if (c0 >= N) return;
    const int tid = threadIdx.x;
    const double a = (double)T[c0];
    double total1, total2;
    // scan A over positions c0 + [0, kStatTile)
    {
        double v1[4], v2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t g = c0 + 4 * tid + u;
            const double d = g < n ? (double)T[g] - a : 0.0;
            v1[u] = d;
            v2[u] = d * d;
        }
        block_exscan4(v1, wsum, total1);
        block_exscan4(v2, wsum, total2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Pa1[4 * tid + u] = v1[u];
            Pa2[4 * tid + u] = v2[u];
        }
        if (tid == 0) {
            Pa1[kStatTile] = total1;
            Pa2[kStatTile] = total2;
        }
    }
    __syncthreads();
    // prefix up to position m (relative to c0)
    double B1, B2;
    if (m <= kStatTile) {
        B1 = Pa1[m];
        B2 = Pa2[m];
    } else {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t y = kStatTile + tid; y < m; y += kStatThreads) {
            const int64_t g = c0 + y;
            const double d = g < n ? (double)T[g] - a : 0.0;
            s1 += d;
            s2 += d * d;
        }
        B1 = Pa1[kStatTile] + block_sum(s1, red);
        B2 = Pa2[kStatTile] + block_sum(s2, red);
    }
    // scan B over positions c0 + m + [0, kStatTile)
    {
        double v1[4], v2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t g = c0 + m + 4 * tid + u;
            const double d = g < n ? (double)T[g] - a : 0.0;
            v1[u] = d;
            v2[u] = d * d;
        }
        block_exscan4(v1, wsum, total1);
        block_exscan4(v2, wsum, total2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Pb1[4 * tid + u] = B1 + v1[u];
            Pb2[4 * tid + u] = B2 + v2[u];
        }
    }
    __syncthreads();
    const int64_t cnt = N - c0 < kStatTile ? N - c0 : kStatTile;
    const double inv_m = 1.0 / m;
    for (int t = tid; t < cnt; t += kStatThreads) {
        const double S1 = Pb1[t] - Pa1[t], S2 = Pb2[t] - Pa2[t];
        const double md = EXPORT ? S1 / m : S1 * inv_m, msq = EXPORT ? S2 / m : S2 * inv_m;
        double var = msq - md * md;
        double mu = a + md;
        // The prefix difference carries an absolute error of about (t + m) * 2^-53 * msq, i.e. a
        // relative error of var of about (1 + 1024/m) * 2^-53 * msq / var.  Short windows and
        // windows with heavy cancellation (near-flat ones) are recomputed two-pass instead.
        if (m <= 64 || !(var > 4e-6 * msq)) {
            const float *w = T + c0 + t;
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
        const int64_t i = c0 + t;
        if (EXPORT) {
            mu_out[i] = mu;
            sg_out[i] = sqrt(var > 0.0 ? var : 0.0);
        } else {
            // the scale is stored in FP32: the FP32 reciprocal square root of the FP64 variance
            // (relative error ~2^-23; var > kSigmaFlat^2 is a normal FP32 number), 0 when flat
            const float m32 = (float)mu;
            const float inv = var > kSigmaFlat * kSigmaFlat ? __builtin_amdgcn_rsqf((float)var) : 0.0f;
            mu32[i] = m32;
            s32[i] = inv;
            o32[i] = (float)(-(mu - (double)m32)) * inv;
        }
    }
}

// ------------------------------------------------------------------ raw series envelope
constexpr int kEnvTile = 2048;
constexpr int kEnvThreads = 256;
constexpr int kEnvMaxPer = (kEnvTile + 2 * (kMaxM - 1) + kEnvThreads - 1) / kEnvThreads;

__global__ __launch_bounds__(kEnvThreads) void k_series_env(const float *__restrict__ T, int64_t n, int r,
                                                            float *__restrict__ U, float *__restrict__ L) {
    extern __shared__ float smem[];
    const int len = kEnvTile + 2 * r;
    float *Mx = smem, *Mn = smem + len;
    const int64_t x0 = (int64_t)blockIdx.x * kEnvTile;
    const int64_t lo = x0 - r;
    const int tid = threadIdx.x;
    for (int y = tid; y < len; y += kEnvThreads) {
        const int64_t g = lo + y;
        const bool in = g >= 0 && g < n;
        const float t = in ? T[g] : 0.0f;
        Mx[y] = in ? t : -INFINITY;
        Mn[y] = in ? t : INFINITY;
    }
    __syncthreads();
    const int w = 2 * r + 1;
    int p = 1;
    while (2 * p <= w) {
        float ra[kEnvMaxPer], rb[kEnvMaxPer];
#pragma unroll
        for (int u = 0; u < kEnvMaxPer; ++u) {
            const int y = tid + u * kEnvThreads;
            if (y < len) {
                const bool has = y + p < len;
                ra[u] = has ? fmaxf(Mx[y], Mx[y + p]) : Mx[y];
                rb[u] = has ? fminf(Mn[y], Mn[y + p]) : Mn[y];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kEnvMaxPer; ++u) {
            const int y = tid + u * kEnvThreads;
            if (y < len) {
                Mx[y] = ra[u];
                Mn[y] = rb[u];
            }
        }
        __syncthreads();
        p *= 2;
    }
    for (int x = tid; x < kEnvTile; x += kEnvThreads) {
        const int64_t g = x0 + x;
        if (g >= n) break;
        U[g] = fmaxf(Mx[x], Mx[x + w - p]);
        L[g] = fminf(Mn[x], Mn[x + w - p]);
    }
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_query_prep(const float *Q, int m, int r, const QueryBufs &b, hipStream_t s) {
    hipLaunchKernelGGL(k_query_prep, dim3(1), dim3(1024), 0, s, Q, m, r, b);
    return hipGetLastError();
}

hipError_t launch_query_prep_batch(const float *Qp, const BatchQ *bq, int nq, const QueryBufs &base,
                                  int64_t qstride, int64_t mstride, int64_t m64stride, hipStream_t s) {
    hipLaunchKernelGGL(k_query_prep_batch, dim3(nq), dim3(1024), 0, s, Qp, bq, base, qstride, mstride, m64stride);
    return hipGetLastError();
}

hipError_t launch_znorm_stats(const float *T, int64_t n, int m, double *mu, double *sg, float *mu32, float *s32,
                              float *o32, hipStream_t s) {
    const int64_t N = n - m + 1;
    const int64_t blocks = (N + kStatTile - 1) / kStatTile;
    if (mu)
        hipLaunchKernelGGL(k_znorm_stats<true>, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, T, n, m, N, mu, sg,
                           mu32, s32, o32);
    else
        hipLaunchKernelGGL(k_znorm_stats<false>, dim3((unsigned)blocks), dim3(kStatThreads), 0, s, T, n, m, N, mu,
                           sg, mu32, s32, o32);
    return hipGetLastError();
}

hipError_t launch_series_env(const float *T, int64_t n, int r, float *U, float *L, hipStream_t s) {
    const int64_t blocks = (n + kEnvTile - 1) / kEnvTile;
    const size_t shm = sizeof(float) * 2 * (kEnvTile + 2 * r);
    hipLaunchKernelGGL(k_series_env, dim3((unsigned)blocks), dim3(kEnvThreads), shm, s, T, n, r, U, L);
    return hipGetLastError();
}

}  // namespace dtws
