// Cascade of lower bounds (Section 2.2): LB_KimFL, then LB_Keogh of the candidate against the
// query envelope (the paper's "EC", eq. (LBKeoghEC)), then LB_Keogh of the query against the
// data envelope (the paper's "EQ", eq. (LBKeoghEQ)).  A later bound runs only on candidates
// that survived the earlier ones (the cascade principle) and each sum stops as soon as it
// exceeds the threshold (early abandoning).  The query positions are visited in order of
// decreasing expected term (see the query preparation) so that the sums grow fastest first.
//
// Layout: one lane per candidate start, consecutive lanes on consecutive starts, so that for a
// fixed query position j the 64 lanes of a wave read 64 consecutive series points (one
// coalesced 256-byte access); the normalisation of each candidate comes from the per-window
// statistics pass.  The candidate value is
//     c_j = fma(T[i+j] - mu32, inv_sigma, corr),  corr = -(mu - mu32) * inv_sigma,
// which keeps the subtraction small even when |mu| is large.
#include "device.h"

namespace dtws {

namespace {

QView make_view(const LbArgs &a) {
    return QView{a.order, a.Us, a.Ls, a.qs, a.m, (a.m + 15) & ~15};
}

struct StatsArrays {
    static constexpr bool kRuns = false;
    const float *mu, *s, *o;
    __device__ void operator()(int64_t i, float &m, float &sg, float &off) const {
        m = mu[i];
        sg = s[i];
        off = o[i];
    }
};

struct EmitList {
    int32_t *surv;
    uint32_t *count;
    __device__ void operator()(bool alive, int64_t i, float) const {
        const uint64_t mask = __ballot(alive);
        if (mask) {
            const int lane = threadIdx.x & 63;
            const int leader = __ffsll((unsigned long long)mask) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
            base = __shfl(base, leader, 64);
            if (alive) surv[base + (uint32_t)__popcll(mask & lanemask_lt())] = (int32_t)i;
        }
    }
};

}  // namespace

// Stage values: every bound of every candidate in full (no abandoning, no pruning).
__global__ __launch_bounds__(256) void k_lb_values(LbArgs a, QView v) {
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int m = a.m;
    const float q0 = a.qh[0], ql = a.qh[m - 1];
    for (int64_t i = a.first + gtid; i < a.last; i += stride) {
        const float mu = a.mu[i], s = a.s[i], o = a.o[i];
        const float *Ti = a.T + i;
        const float c0 = fmaf(Ti[0] - mu, s, o), cl = fmaf(Ti[m - 1] - mu, s, o);
        const float d0 = q0 - c0, dl = ql - cl;
        const float kim = fmaf(d0, d0, dl * dl);
        const float kq = keogh_q_terms(v, Ti, mu, s, o, 0.0f, 0, v.mpad, false, INFINITY);
        const float kd = keogh_d(v, a.envU + i, a.envL + i, mu, s, o, INFINITY);
        if (a.out_kim) a.out_kim[i] = kim;
        if (a.out_kq) a.out_kq[i] = kq;
        if (a.out_kd) a.out_kd[i] = kd;
        if (a.out_key) a.out_key[i] = ((uint64_t)__float_as_uint(fmaxf(fmaxf(kim, kq), kd)) << 32) | (uint64_t)i;
    }
}

// Pruning: each wave owns groups of 64 consecutive candidates, grid-strided over [first, last).
__global__ __launch_bounds__(256) void k_lb_prune(LbArgs a, QView v) {
    __shared__ WaveQueue q1s[4];
    __shared__ WaveQueue2 q2s[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const float thr = a.key ? threshold_of(load_bsf(a.key)) : a.fixed_thr;
    CascadeCounts cnt;
    StrideSource src{a.first + wave * 64, nwaves * 64, a.last};
    cascade(v, a.T, a.envU, a.envL, thr, a.qh, src, q1s[wid], q2s[wid],
            StatsArrays{a.mu, a.s, a.o}, EmitList{a.surv, a.surv_count}, cnt);
    if (a.counters) {
        const unsigned long long c_kim = cnt.wave_kim(), c_kq = wave_add_u64(cnt.kq),
                                 c_kd = wave_add_u64(cnt.kd);
        if (lane == 0) {
            atomicAdd(&a.counters[1], c_kim);
            atomicAdd(&a.counters[2], c_kq);
            atomicAdd(&a.counters[3], c_kd);
        }
    }
}

// One segment [a0, a1) of the LB-sorted candidate list (keys ascending: (bits(LB) << 32) | start,
// LB >= 0 so its bits order like its value): the leading candidates whose bound lies within the
// pruning slack of the current best-so-far go to surv, their number to *count; the rest of the
// segment (and every later one) is pruned.
__global__ __launch_bounds__(256) void k_lbs_segment(const uint64_t *keys, int64_t a0, int64_t a1,
                                                     const uint64_t *bsf_key, int32_t *surv, uint32_t *count) {
    const float thr = threshold_of(key_dist(*bsf_key));
    const uint64_t lim = ((uint64_t)__float_as_uint(thr) << 32) | 0xFFFFFFFFull;   // keys with LB <= thr
    int64_t lo = a0, hi = a1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] > lim) hi = mid;
        else lo = mid + 1;
    }
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = a0 + gtid; k < lo; k += stride) surv[k - a0] = (int32_t)(keys[k] & 0xFFFFFFFFull);
    if (gtid == 0) *count = (uint32_t)(lo - a0);
}

hipError_t launch_lb_sorted_segment(const uint64_t *keys, int64_t a0, int64_t a1, const uint64_t *bsf_key,
                                    int32_t *surv, uint32_t *count, int num_cu, hipStream_t s) {
    int64_t blocks = (a1 - a0 + 255) / 256;
    if (blocks > num_cu * 4) blocks = num_cu * 4;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_lbs_segment, dim3((unsigned)blocks), dim3(256), 0, s, keys, a0, a1, bsf_key, surv, count);
    return hipGetLastError();
}

hipError_t launch_lb(const LbArgs &a, int mode, int num_cu, hipStream_t s) {
    const int64_t cnt = a.last - a.first;
    if (cnt <= 0) return hipSuccess;
    int64_t blocks = (cnt + 255) / 256;
    const int64_t cap = (int64_t)num_cu * 16;
    if (blocks > cap) blocks = cap;
    const QView v = make_view(a);
    if (mode == 0)
        hipLaunchKernelGGL(k_lb_values, dim3((unsigned)blocks), dim3(256), 0, s, a, v);
    else
        hipLaunchKernelGGL(k_lb_prune, dim3((unsigned)blocks), dim3(256), 0, s, a, v);
    return hipGetLastError();
}

}  // namespace dtws
