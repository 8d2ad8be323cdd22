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

// Query-side arrays never change during a launch: reading them through the constant address
// space lets the compiler use scalar loads for the (wave-uniform) positions.
template <class T>
__device__ __forceinline__ T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Order LDS traffic of one wave (the queues below are private to a wave).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- pruning (MODE 1)
// Each wave owns a stream of groups of 64 consecutive candidates.  Level 0 (coalesced, uniform):
// LB_KimFL and the first K0 terms of the query-envelope bound for all 64 candidates.  Survivors
// are compacted into a wave-private LDS queue; whenever it holds 64 entries, level 1 runs the
// next terms up to K1 on a full batch; its survivors go to a second queue whose full batches run
// the remaining terms with early abandoning, then the data-envelope bound.  Every batch starts
// all its lanes at the same term, so the query-side arrays are read with scalar loads.
constexpr int kQCap = 128;   // power of two, >= 2 * 64
constexpr int kK0 = 16, kK1 = 64;

struct WaveQueue {
    int32_t idx[kQCap];
    float kq[kQCap], mu[kQCap], s[kQCap], o[kQCap];
};


// One block of 16 query-envelope terms starting at k0 (a multiple of 16): all 16 series loads
// are issued before any use, so a wave waits for one memory round trip per block.
__device__ inline float keogh_q_block(const LbArgs &a, const float *Ti, float mu, float s, float o, float kq,
                                      int k0) {
    float t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = Ti[ldc(a.order + k0 + u)];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float c = fmaf(t[u] - mu, s, o);
        const float e = fmaxf(fmaxf(c - ldc(a.Us + k0 + u), ldc(a.Ls + k0 + u) - c), 0.0f);
        kq = fmaf(e, e, kq);
    }
    return kq;
}

__device__ inline float keogh_q_terms(const LbArgs &a, const float *Ti, float mu, float s, float o, float kq, int k0,
                                      int k1, bool early, float thr) {
    for (int k = k0; k < k1; k += 16) {
        kq = keogh_q_block(a, Ti, mu, s, o, kq, k);
        if (early && kq > thr) break;
    }
    return kq;
}

__device__ inline float keogh_d(const LbArgs &a, int64_t i, float mu, float s, float o, float thr) {
    const float *Ui = a.envU + i, *Li = a.envL + i;
    float kd = 0.0f;
    const int mpad = (a.m + 15) & ~15;
    for (int k0 = 0; k0 < mpad; k0 += 16) {
        float u[16], l[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = ldc(a.order + k0 + v);
            u[v] = Ui[j];
            l[v] = Li[j];
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float uu = fmaf(u[v] - mu, s, o), ll = fmaf(l[v] - mu, s, o);
            const float q = ldc(a.qs + k0 + v);
            const float e = fmaxf(fmaxf(q - uu, ll - q), 0.0f);
            kd = fmaf(e, e, kd);
        }
        if (kd > thr) break;
    }
    return kd;
}

__device__ inline void q_push(WaveQueue &q, uint32_t &tail, bool pred, int32_t i, float kq, float mu, float s,
                              float o) {
    const uint64_t mask = __ballot(pred);
    if (pred) {
        const uint32_t p = (tail + (uint32_t)__popcll(mask & lanemask_lt())) & (kQCap - 1);
        q.idx[p] = i;
        q.kq[p] = kq;
        q.mu[p] = mu;
        q.s[p] = s;
        q.o[p] = o;
    }
    tail += (uint32_t)__popcll(mask);
    wave_sync();
}

// Pops up to 64 entries (one per lane); returns whether this lane got one.
__device__ inline bool q_pop(WaveQueue &q, uint32_t &head, uint32_t tail, int32_t &i, float &kq, float &mu,
                             float &s, float &o) {
    const int lane = threadIdx.x & 63;
    const uint32_t avail = tail - head;
    const uint32_t take = avail < 64u ? avail : 64u;
    const bool got = (uint32_t)lane < take;
    const uint32_t p = (head + lane) & (kQCap - 1);
    if (got) {
        i = q.idx[p];
        kq = q.kq[p];
        mu = q.mu[p];
        s = q.s[p];
        o = q.o[p];
    }
    head += take;
    wave_sync();
    return got;
}

__device__ inline void append_survivors(const LbArgs &a, bool alive, int64_t i) {
    const uint64_t mask = __ballot(alive);
    if (mask) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(a.surv_count, (uint32_t)__popcll(mask));
        base = __shfl(base, leader, 64);
        if (alive) a.surv[base + (uint32_t)__popcll(mask & lanemask_lt())] = (int32_t)i;
    }
}

// Stage-value writer (MODE 0): every bound of every candidate in full, one lane per candidate.
__global__ __launch_bounds__(256) void k_lb_values(LbArgs a) {
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
        const float kq = keogh_q_terms(a, Ti, mu, s, o, 0.0f, 0, (m + 15) & ~15, false, INFINITY);
        const float kd = keogh_d(a, i, mu, s, o, INFINITY);
        if (a.out_kim) a.out_kim[i] = kim;
        if (a.out_kq) a.out_kq[i] = kq;
        if (a.out_kd) a.out_kd[i] = kd;
    }
}

__global__ __launch_bounds__(256) void k_lb_prune(LbArgs a) {
    __shared__ WaveQueue queues[4][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    WaveQueue &q1 = queues[wid][0], &q2 = queues[wid][1];
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int m = a.m;
    const int mpad = (m + 15) & ~15;
    const int K0 = mpad < kK0 ? mpad : kK0, K1 = mpad < kK1 ? mpad : kK1;
    const float thr = a.key ? threshold_of(key_dist(__atomic_load_n(a.key, __ATOMIC_RELAXED))) : a.fixed_thr;
    const float q0 = a.qh[0], ql = a.qh[m - 1];
    uint32_t n_kim = 0, n_kq = 0, n_kd = 0;
    uint32_t h1 = 0, t1 = 0, h2 = 0, t2 = 0;
    int64_t g = a.first + wave * 64;
    bool done = false;
    // Wave-uniform scheduler: a full level-2 batch first, then a full level-1 batch, then a new
    // group; so each queue holds fewer than 64 entries whenever a push can reach it.
    for (;;) {
        if (t2 - h2 >= 64u || (done && t2 != h2)) {
            int32_t i = 0;
            float kq = 0.f, mu = 0.f, s = 0.f, o = 0.f;
            const bool got = q_pop(q2, h2, t2, i, kq, mu, s, o);
            bool alive = got;
            if (got) {
                kq = keogh_q_terms(a, a.T + i, mu, s, o, kq, K1, mpad, true, thr);
                if (kq > thr) {
                    alive = false;
                    ++n_kq;
                }
            }
            if (alive) {
                const float kd = keogh_d(a, i, mu, s, o, thr);
                if (kd > thr) {
                    alive = false;
                    ++n_kd;
                }
            }
            append_survivors(a, alive, i);
            continue;
        }
        if (t1 - h1 >= 64u || (done && t1 != h1)) {
            int32_t i = 0;
            float kq = 0.f, mu = 0.f, s = 0.f, o = 0.f;
            const bool got = q_pop(q1, h1, t1, i, kq, mu, s, o);
            bool alive = got;
            if (got && K1 > K0) {
                kq = keogh_q_terms(a, a.T + i, mu, s, o, kq, K0, K1, false, thr);
                if (kq > thr) {
                    alive = false;
                    ++n_kq;
                }
            }
            q_push(q2, t2, alive, i, kq, mu, s, o);
            continue;
        }
        if (done) break;
        if (g >= a.last) {
            done = true;
            continue;
        }
        // level 0: a group of 64 consecutive candidates
        const int64_t i = g + lane;
        const bool valid = i < a.last;
        const int64_t ii = valid ? i : a.first;      // keeps idle lanes' loads in range
        const float mu = a.mu[ii], s = a.s[ii], o = a.o[ii];
        const float *Ti = a.T + ii;
        const float c0 = fmaf(Ti[0] - mu, s, o), cl = fmaf(Ti[m - 1] - mu, s, o);
        const float d0 = q0 - c0, dl = ql - cl;
        const float kim = fmaf(d0, d0, dl * dl);
        bool alive = valid && !(kim > thr);
        if (valid && !alive) ++n_kim;
        float kq = 0.0f;
        if (__ballot(alive)) {
            kq = keogh_q_terms(a, Ti, mu, s, o, 0.0f, 0, K0, false, thr);
            if (alive && kq > thr) {
                alive = false;
                ++n_kq;
            }
        }
        q_push(q1, t1, alive, (int32_t)ii, kq, mu, s, o);
        g += nwaves * 64;
    }

    if (a.counters) {
        const unsigned long long c_kim = wave_add_u64(n_kim), c_kq = wave_add_u64(n_kq), c_kd = wave_add_u64(n_kd);
        if (lane == 0) {
            atomicAdd(&a.counters[1], c_kim);
            atomicAdd(&a.counters[2], c_kq);
            atomicAdd(&a.counters[3], c_kd);
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
        hipLaunchKernelGGL(k_lb_values, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_lb_prune, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dtws
