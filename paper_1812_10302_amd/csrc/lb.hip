// Cascade of lower bounds (Section 2.2): LB_KimFL, then LB_Keogh of the candidate against the
// query envelope (the paper's "EC", eq. (LBKeoghEC)), then LB_Keogh of the query against the
// data envelope (the paper's "EQ", eq. (LBKeoghEQ)).  A later bound runs only on candidates
// that survived the earlier ones (the cascade principle) and each sum stops as soon as it
// exceeds the threshold (early abandoning).  The query positions are visited in order of
// decreasing |qhat| so that the sums grow fastest first.
//
// Layout: one lane per candidate start, consecutive lanes on consecutive starts, so that for a
// fixed query position j the 64 lanes of a wave read 64 consecutive series points (one
// coalesced 256-byte access); the normalisation (mu, 1/sigma, correction) of each candidate
// comes from the per-window statistics pass.  The candidate value is
//     c_j = fma(T[i+j] - mu32, inv_sigma, corr),  corr = -(mu - mu32) * inv_sigma,
// which keeps the subtraction small even when |mu| is large.
#include "dtws_internal.h"

namespace dtws {



__device__ inline unsigned long long wave_add_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// MODE 0: write all three bound values (no abandoning, no pruning).
// MODE 1: prune against the threshold and append the survivors' starts.
template <int MODE>
__global__ __launch_bounds__(256) void k_lb(LbArgs a) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int m = a.m;
    float thr = INFINITY;
    if (MODE == 1) thr = a.key ? threshold_of(key_dist(__atomic_load_n(a.key, __ATOMIC_RELAXED))) : a.fixed_thr;
    const float q0 = a.qh[0], ql = a.qh[m - 1];
    unsigned long long n_kim = 0, n_kq = 0, n_kd = 0;
    for (int64_t i = a.first + gtid; i < a.last; i += stride) {
        const float mu = a.mu[i], s = a.s[i], o = a.o[i];
        const float *Ti = a.T + i;
        const float c0 = fmaf(Ti[0] - mu, s, o), cl = fmaf(Ti[m - 1] - mu, s, o);
        const float d0 = q0 - c0, dl = ql - cl;
        const float kim = fmaf(d0, d0, dl * dl);
        bool alive = true;
        if (MODE == 1 && kim > thr) {
            alive = false;
            ++n_kim;
        }
        float kq = 0.0f;
        if (alive) {
            for (int k = 0; k < m; ++k) {
                const int j = a.order[k];
                const float c = fmaf(Ti[j] - mu, s, o);
                const float e = fmaxf(fmaxf(c - a.Us[k], a.Ls[k] - c), 0.0f);
                kq = fmaf(e, e, kq);
                if (MODE == 1 && (k & 7) == 7 && kq > thr) break;
            }
            if (MODE == 1 && kq > thr) {
                alive = false;
                ++n_kq;
            }
        }
        float kd = 0.0f;
        if (alive) {
            const float *Ui = a.envU + i, *Li = a.envL + i;
            for (int k = 0; k < m; ++k) {
                const int j = a.order[k];
                const float u = fmaf(Ui[j] - mu, s, o), l = fmaf(Li[j] - mu, s, o);
                const float q = a.qs[k];
                const float e = fmaxf(fmaxf(q - u, l - q), 0.0f);
                kd = fmaf(e, e, kd);
                if (MODE == 1 && (k & 7) == 7 && kd > thr) break;
            }
            if (MODE == 1 && kd > thr) {
                alive = false;
                ++n_kd;
            }
        }
        if (MODE == 0) {
            if (a.out_kim) a.out_kim[i] = kim;
            if (a.out_kq) a.out_kq[i] = kq;
            if (a.out_kd) a.out_kd[i] = kd;
        } else {
            const uint64_t mask = __ballot(alive);
            if (mask) {
                const int lane = threadIdx.x & 63;
                const int leader = __ffsll((unsigned long long)mask) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(a.surv_count, (uint32_t)__popcll(mask));
                base = __shfl(base, leader, 64);
                const uint32_t pos = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                if (alive) a.surv[pos] = (int32_t)i;
            }
        }
    }
    if (MODE == 1 && a.counters) {
        n_kim = wave_add_u64(n_kim);
        n_kq = wave_add_u64(n_kq);
        n_kd = wave_add_u64(n_kd);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&a.counters[1], n_kim);
            atomicAdd(&a.counters[2], n_kq);
            atomicAdd(&a.counters[3], n_kd);
        }
    }
}

hipError_t launch_lb(const LbArgs &a, int mode, int num_cu, hipStream_t s) {
    const int64_t cnt = a.last - a.first;
    if (cnt <= 0) return hipSuccess;
    int64_t blocks = (cnt + 255) / 256;
    const int64_t cap = (int64_t)num_cu * 16;
    if (blocks > cap) blocks = cap;
    if (mode == 0)
        hipLaunchKernelGGL(k_lb<0>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_lb<1>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dtws
