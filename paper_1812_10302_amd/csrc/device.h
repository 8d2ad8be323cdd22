// Device helpers shared by the plain and the batched search kernels.
#pragma once
#include <utility>

#include "dtws_internal.h"

namespace dtws {

// ---------------------------------------------------------------- wave utilities
__device__ inline unsigned long long wave_add_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline unsigned long long wave_add(unsigned long long v) { return wave_add_u64(v); }

// Number of lanes below this one whose bit is set in mask (the hardware masked bit count).
__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Orders the LDS traffic of one wave (for structures private to a wave).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Query-side arrays never change during a launch: reading them through the constant address
// space lets the compiler use scalar loads for wave-uniform positions.
template <class T>
__device__ __forceinline__ T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// A value the caller knows to be the same in every lane, placed in scalar registers.
__device__ __forceinline__ int64_t uniform(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Best-so-far keys change only through device-scope atomicMin, so a device-scope load sees them
// (served by L2, no trip to memory).
__device__ inline uint64_t load_key(const uint64_t *key) {
    return __hip_atomic_load(key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float load_bsf(const uint64_t *key) { return key_dist(load_key(key)); }
// The distance half of the key alone (its upper 32 bits), as raw bits.
__device__ inline uint32_t load_key_dist_bits(const uint64_t *key) {
    return __hip_atomic_load((const uint32_t *)key + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- bound terms
// Query side of the bounds: positions in visiting order (decreasing expected term), padded with neutral
// terms to a multiple of 16.
struct QView {
    const int32_t *order;
    const float *Us, *Ls, *qs;
    int m, mpad;
};

// One block of 16 query-envelope terms (eq. (LBKeoghEC)) starting at k0, a multiple of 16: all
// 16 series loads are issued before any use, so a wave waits for one memory round trip.
__device__ inline float keogh_q_block(const QView &v, const float *Ti, float mu, float s, float o, float kq,
                                      int k0) {
    float t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = Ti[ldc(v.order + k0 + u)];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float c = fmaf(t[u] - mu, s, o);
        const float e = fmaxf(fmaxf(c - ldc(v.Us + k0 + u), ldc(v.Ls + k0 + u) - c), 0.0f);
        kq = fmaf(e, e, kq);
    }
    return kq;
}

__device__ inline float keogh_q_terms(const QView &v, const float *Ti, float mu, float s, float o, float kq, int k0,
                                      int k1, bool early, float thr) {
    for (int k = k0; k < k1; k += 16) {
        kq = keogh_q_block(v, Ti, mu, s, o, kq, k);
        if (early && kq > thr) break;
    }
    return kq;
}

// The query against the data envelope (eq. (LBKeoghEQ)), early abandoning per 16 terms.
__device__ inline float keogh_d(const QView &v, const float *Ui, const float *Li, float mu, float s, float o,
                                float thr) {
    float kd = 0.0f;
    for (int k0 = 0; k0 < v.mpad; k0 += 16) {
        float u[16], l[16];
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int j = ldc(v.order + k0 + w);
            u[w] = Ui[j];
            l[w] = Li[j];
        }
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const float uu = fmaf(u[w] - mu, s, o), ll = fmaf(l[w] - mu, s, o);
            const float q = ldc(v.qs + k0 + w);
            const float e = fmaxf(fmaxf(q - uu, ll - q), 0.0f);
            kd = fmaf(e, e, kd);
        }
        if (kd > thr) break;
    }
    return kd;
}

// ---------------------------------------------------------------- wave-private queues
constexpr int kQCap = 256;    // level-1 queue: power of two, >= 3 * 64 (a level-0 step pushes two groups)
constexpr int kQCap2 = 128;   // level-2 queue: power of two, >= 2 * 64 (level 1 pushes one batch)
constexpr int kK1 = 64;   // query-envelope terms of level 1

template <int CAP>
struct WaveQueueT {
    static constexpr uint32_t kMask = CAP - 1;
    int32_t idx[CAP];
    float kq[CAP], mu[CAP], s[CAP], o[CAP];
};
using WaveQueue = WaveQueueT<kQCap>;
using WaveQueue2 = WaveQueueT<kQCap2>;

template <class Q>
__device__ inline void q_push(Q &q, uint32_t &tail, bool pred, int32_t i, float kq, float mu, float s, float o) {
    const uint64_t mask = __ballot(pred);
    if (pred) {
        const uint32_t p = (tail + rank_in(mask)) & Q::kMask;
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
template <class Q>
__device__ inline bool q_pop(Q &q, uint32_t &head, uint32_t tail, int32_t &i, float &kq, float &mu, float &s,
                             float &o) {
    const int lane = threadIdx.x & 63;
    const uint32_t avail = tail - head;
    const uint32_t take = avail < 64u ? avail : 64u;
    const bool got = (uint32_t)lane < take;
    const uint32_t p = (head + lane) & Q::kMask;
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

// ---------------------------------------------------------------- cascade over a candidate range
struct CascadeCounts {
    uint32_t kim = 0, kq = 0, kd = 0;   // per lane
    uint32_t kim_w = 0;                 // LB_Kim prunes counted for the whole wave (same in every lane)
    __device__ unsigned long long wave_kim() const { return wave_add_u64(kim) + kim_w; }
};

// Runs the bound cascade (one wave) on groups of 64 consecutive candidates handed out by
// src.next(g, last): the group starts at g, starts at or beyond `last` are idle lanes; next()
// returns false when the source is exhausted.  Level 0 (coalesced, uniform, two groups per step):
// LB_KimFL, plus the first 16 query-envelope terms for a group in which more than half survive
// it.  With Stats::kRuns and m a multiple of 64 the source hands out whole items (src.next_run)
// that level 0 walks as chains of groups m apart, carrying the prefix entries from one group to
// the next, so the window statistics cost one prefix lookup per candidate.  Survivors are compacted into the wave's LDS queue q1; full batches of 64 run the
// query-envelope terms up to K1, 16 at a time with early abandoning (level 1), and their
// survivors go to
// q2, whose full batches run the remaining terms with
// early abandoning and then the data-envelope bound (level 2, if envU is set).  Candidates that
// pass everything go to emit(alive, i, kq), kq the candidate's full query-envelope sum.  A scheduler that is uniform across the wave serves a
// full q2 batch first, then a full q1 batch, then new groups: q2 holds fewer than 64 entries when
// level 1 pushes up to 64 into it, and q1 fewer than 64 when level 0 pushes up to two groups (128)
// into it, which kQCap accommodates; at the end both queues are drained.
//   stats(i, mu, s, o): normalisation parameters of candidate i.  ENV = false compiles the
//   data-envelope bound out (fewer registers when the caller never passes an envelope).
template <bool ENV = true, class Stats, class Emit, class Source>
__device__ __forceinline__ void cascade(const QView &v, const float *T, const float *envU, const float *envL,
                                        float thr, const float *qh, Source &src, WaveQueue &q1, WaveQueue2 &q2,
                                        const Stats &stats, const Emit &emit, CascadeCounts &cnt) {
    const int lane = threadIdx.x & 63;
    const int m = v.m, mpad = v.mpad;
    const float q0 = ldc(qh), ql = ldc(qh + m - 1);
    const int K1 = mpad < kK1 ? mpad : kK1;
    uint32_t h1 = 0, t1 = 0, h2 = 0, t2 = 0;
    bool done = false;
    // chain mode (Stats::kRuns, m a multiple of 64): the current item [cf, clast) is walked as m / 64
    // chains; chain j visits the groups cf + 64 j + t m, t = 0, 1, ..., so the prefix entry at the
    // end of a group's windows is the one at the start of the chain's next group (carried in
    // cnext); two chains advance per step
    const bool chains = Stats::kRuns && (m & 63) == 0;
    int64_t cf = 0, clast = 0, cg = 0;
    int cj = 0, cJ = m >> 6;
    bool citem = false, cfresh = true;
    double2 ccarry[2];
    ccarry[0] = ccarry[1] = make_double2(0.0, 0.0);
    // loads of the chain walk's next step, issued one step ahead (valid while cnext is set)
    bool cnext = false;
    double2 npe[2];
    float nc0[2], ncl[2];
    npe[0] = npe[1] = make_double2(0.0, 0.0);
    nc0[0] = nc0[1] = ncl[0] = ncl[1] = 0.0f;
    for (;;) {
        if (t2 - h2 >= 64u || (done && t2 != h2)) {
            int32_t i = 0;
            float kq = 0.f, mu = 0.f, s = 0.f, o = 0.f;
            const bool got = q_pop(q2, h2, t2, i, kq, mu, s, o);
            bool alive = got;
            if (got) {
                kq = keogh_q_terms(v, T + i, mu, s, o, kq, K1, mpad, true, thr);
                if (kq > thr) {
                    alive = false;
                    ++cnt.kq;
                }
            }
            if (ENV && alive && envU) {
                const float kd = keogh_d(v, envU + i, envL + i, mu, s, o, thr);
                if (kd > thr) {
                    alive = false;
                    ++cnt.kd;
                }
            }
            emit(alive, i, kq);
            continue;
        }
        if (t1 - h1 >= 64u || (done && t1 != h1)) {
            int32_t i = 0;
            float kq = 0.f, mu = 0.f, s = 0.f, o = 0.f;
            const bool got = q_pop(q1, h1, t1, i, kq, mu, s, o);
            bool alive = got;
            if (got) {
                // entries with kq < 0 have no term done yet, the others the first 16; the first
                // block runs for the whole batch when any entry needs it, so the term position
                // stays wave-uniform (scalar loads of the query side)
                if (__ballot(kq < 0.0f)) {
                    const float k16 = keogh_q_block(v, T + i, mu, s, o, 0.0f, 0);
                    if (kq < 0.0f) kq = k16;
                }
                kq = keogh_q_terms(v, T + i, mu, s, o, kq, 16, K1, true, thr);
                if (kq > thr) {
                    alive = false;
                    ++cnt.kq;
                }
            }
            q_push(q2, t2, alive, i, kq, mu, s, o);
            continue;
        }
        if (done) break;
        if constexpr (Stats::kRuns) {
            if (chains) {
                if (!citem) {
                    if (!src.next_run(cf, clast)) {
                        done = true;
                        continue;
                    }
                    cf = uniform(cf);
                    clast = uniform(clast);
                    citem = true;
                    cj = 0;
                    cg = cf;
                    cfresh = true;
                }
                // level-0 steps in a tight loop while q1 has room for two more groups (< 64 entries
                // leaves 192 free slots); back to the scheduler when it fills or the item ends
                do {
                    // chains cj and cj + 1 (if it exists) at the same step t: groups cg and cg + 64
                    cg = uniform(cg);
                    const bool two = cj + 1 < cJ;
                    // the two groups are addressed from scalar bases with 32-bit lane offsets; idle
                    // lanes (past the item end, or no second chain) read the group's first start
                    auto lane_offsets = [&](int64_t g, bool tw, uint32_t (&off)[2], bool (&valid)[2]) {
                        const int64_t span = clast - g;
                        const uint32_t lim = span < 128 ? (uint32_t)span : 128u;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint32_t o = 64u * h + (uint32_t)lane;
                            valid[h] = (h == 0 || tw) && o < lim;
                            off[h] = valid[h] ? o : 0u;
                        }
                    };
                    // stored (even) prefix entries of the window ends and the series points at
                    // the window starts and ends of the step at g (g and m are even), into the
                    // registers of the step loaded ahead
                    auto load_step = [&](int64_t g, bool tw) {
                        uint32_t o[2];
                        bool v[2];
                        lane_offsets(g, tw, o, v);
                        const double2 *PE = stats.pre.PPe + ((g + m) >> 1);
                        const float *Tg = T + g, *TLg = Tg + (m - 1);
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            npe[h] = PE[o[h] >> 1];
                            nc0[h] = Tg[o[h]];
                            ncl[h] = TLg[o[h]];
                        }
                    };
                    uint32_t off[2];
                    bool valid[2];
                    lane_offsets(cg, two, off, valid);
                    if (!cnext) load_step(cg, two);   // an item's first step: nothing was loaded ahead
                    double2 pe[2];
                    float c0v[2], clv[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        pe[h] = npe[h];
                        c0v[h] = nc0[h];
                        clv[h] = ncl[h];
                    }
                    // the next step's loads go out before this step's work, unconditionally (a
                    // load under a branch makes every later wait count it): the chain pair's next
                    // step, else the next pair's first step, else (the item ends) this step again
                    {
                        int64_t gn = cg + m;
                        bool twn = two;
                        cnext = gn < clast;
                        if (!cnext) {
                            const int cjn = cj + (two ? 2 : 1);
                            gn = cf + 64 * cjn;
                            twn = cjn + 1 < cJ;
                            cnext = cjn < cJ && gn < clast;
                            if (!cnext) {
                                gn = cg;
                                twn = two;
                            }
                        }
                        load_step(uniform(gn), twn);
                    }
                    const double2 *P0 = stats.pre.PPe + (cg >> 1);
                    const float *T0 = T + cg;
                    // anchors and totals of the blocks of both groups' starts (scalar loads, issued
                    // together; the entry past the last block exists)
                    double alo[2], ahi[2];
                    double2 tbk[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int64_t b0 = (cg + 64 * h) >> kPBShift;
                        const double *tb = (const double *)(stats.pre.tot + b0);
                        alo[h] = ldc(stats.pre.anc + b0);
                        ahi[h] = ldc(stats.pre.anc + b0 + 1);
                        tbk[h] = make_double2(ldc(tb), ldc(tb + 1));
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        // block of the group's starts and whether its windows end past it: the
                        // same for all 64 lanes (scalar); idle lanes' values are never used
                        const int64_t gs = cg + 64 * h;
                        const int64_t b0 = gs >> kPBShift, e0 = (b0 + 1) << kPBShift;
                        const bool cross = gs + m >= e0;
                        // odd lanes (odd starts and ends) complete their prefix entries with the
                        // point before: the window's last point at the end (already loaded), the
                        // point before the start at a chain start
                        const bool odd = (off[h] & 1u) != 0;
                        const double aend = cross ? ahi[h] : alo[h];
                        double2 pev = pe[h];
                        {
                            const double d = odd ? (double)clv[h] - aend : 0.0;
                            pev.x += d;
                            pev.y = fma(d, d, pev.y);
                        }
                        double2 p0 = ccarry[h];
                        if (cfresh) {
                            p0 = P0[off[h] >> 1];
                            const double d = odd ? (double)T0[off[h] & ~1u] - alo[h] : 0.0;
                            p0.x += d;
                            p0.y = fma(d, d, p0.y);
                        }
                        ccarry[h] = pev;
                        const double a0 = alo[h];
                        double S1, S2;
                        stats.sums_group(cross, (int)(gs + m - e0) + lane, p0, pev, alo[h], ahi[h], tbk[h], S1, S2);
                        float mu = 0.0f, s = 0.0f, o = 0.0f;
                        if (valid[h]) stats.finish(cg + off[h], a0, S1, S2, mu, s, o);
                        const float d0 = q0 - fmaf(c0v[h] - mu, s, o), dl = ql - fmaf(clv[h] - mu, s, o);
                        const bool alive = valid[h] && !(fmaf(d0, d0, dl * dl) > thr);
                        cnt.kim_w += (uint32_t)(__popcll(__ballot(valid[h])) - __popcll(__ballot(alive)));
                        q_push(q1, t1, alive, (int32_t)cg + (int32_t)off[h], -1.0f, mu, s, o);
                    }
                    cfresh = false;
                    cg += m;
                    if (cg >= clast) {
                        cj += two ? 2 : 1;
                        cg = cf + 64 * cj;
                        cfresh = true;
                        if (cj >= cJ || cg >= clast) citem = false;
                    }
                } while (citem && t1 - h1 < 64u);
                continue;
            }
        }
        // two groups per step: the loads of both are in flight together
        int64_t gA, lastA, gB, lastB;
        if (!src.next(gA, lastA)) {
            done = true;
            continue;
        }
        const bool hasB = src.next(gB, lastB);
        if (!hasB) {
            gB = gA;
            lastB = gA;
        }
        const int64_t iA = gA + lane, iB = gB + lane;
        const bool vA = iA < lastA, vB = iB < lastB;
        const int64_t iiA = vA ? iA : gA, iiB = vB ? iB : gA;   // idle lanes reuse a valid start
        float muA, sA, oA, muB, sB, oB;
        stats(iiA, muA, sA, oA);
        stats(iiB, muB, sB, oB);
        const float a0 = T[iiA], al = T[iiA + m - 1], b0 = T[iiB], bl = T[iiB + m - 1];
        const float dA0 = q0 - fmaf(a0 - muA, sA, oA), dAl = ql - fmaf(al - muA, sA, oA);
        const float dB0 = q0 - fmaf(b0 - muB, sB, oB), dBl = ql - fmaf(bl - muB, sB, oB);
        const bool aliveA = vA && !(fmaf(dA0, dA0, dAl * dAl) > thr);
        const bool aliveB = vB && !(fmaf(dB0, dB0, dBl * dBl) > thr);
        if (vA && !aliveA) ++cnt.kim;
        if (vB && !aliveB) ++cnt.kim;
        // a group where LB_Kim pruned little runs the first 16 query-envelope terms right here on
        // coalesced lanes; otherwise its survivors enter the queue with no term done (kq = -1)
        float kqA = -1.0f, kqB = -1.0f;
        bool keepA = aliveA, keepB = aliveB;
        if (__popcll(__ballot(aliveA)) > 32) {
            kqA = keogh_q_block(v, T + iiA, muA, sA, oA, 0.0f, 0);
            if (aliveA && kqA > thr) {
                keepA = false;
                ++cnt.kq;
            }
        }
        if (__popcll(__ballot(aliveB)) > 32) {
            kqB = keogh_q_block(v, T + iiB, muB, sB, oB, 0.0f, 0);
            if (aliveB && kqB > thr) {
                keepB = false;
                ++cnt.kq;
            }
        }
        q_push(q1, t1, keepA, (int32_t)iiA, kqA, muA, sA, oA);
        q_push(q1, t1, keepB, (int32_t)iiB, kqB, muB, sB, oB);
        if (!hasB) done = true;
    }
}

// Group source over [first, last) with a fixed stride (grid-stride loop of the plain kernel).
struct StrideSource {
    int64_t g, step, end;
    __device__ bool next(int64_t &gg, int64_t &last) {
        if (g >= end) return false;
        gg = g;
        last = end;
        g += step;
        return true;
    }
};

// ---------------------------------------------------------------- DTW column machinery

template <int KK>
__device__ __forceinline__ float row_bcast(float v) {
    // DPP row_newbcast:KK -- every lane of a 16-lane row reads lane KK of that row; written as
    // update_dpp(old=0, bound_ctrl) so that the compiler folds it into the consuming v_sub_f32_dpp
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + KK, 0xF, 0xF, true));
}

template <int I, int N, int NC>
__device__ __forceinline__ void cell(float (&a)[N], const float (&q)[NC], float c, float &below) {
    const float diff = row_bcast<(I & 15)>(q[I >> 4]) - c;
    const float mn = fminf(fminf(a[I], a[I + 1]), below);
    const float v = fmaf(diff, diff, mn);
    a[I] = v;
    below = v;
}

template <int NC, int... I>
__device__ __forceinline__ void column_impl(float (&a)[16 * NC + 1], const float (&q)[NC], float c,
                                            std::integer_sequence<int, I...>) {
    float below = INFINITY;
    (cell<I, 16 * NC + 1, NC>(a, q, c, below), ...);
}

template <int NC>
__device__ __forceinline__ void column(float (&a)[16 * NC + 1], const float (&q)[NC], float c) {
    column_impl<NC>(a, q, c, std::make_integer_sequence<int, 16 * NC>{});
}


// Band cells of columns [0, J) of an m x m DP with band r.
__device__ inline unsigned long long band_cells(int m, int r, int J) {
    long long cells = (long long)J * (2 * r + 1);
    const long long lower = J <= r ? (long long)J * r - (long long)J * (J - 1) / 2 : (long long)r * (r + 1) / 2;
    const long long ex = (long long)J - (m - r);
    const long long upper = ex > 0 ? ex * (ex + 1) / 2 : 0;
    return (unsigned long long)(cells - lower - upper);
}

// Per-lane normalisation of the window at `start`: two-pass FP64 mean and sigma.
__device__ inline void lane_stats(const float *w, int m, float &mu, float &s, float &o) {
    double sum = 0.0;
    for (int j = 0; j < m; ++j) sum += (double)w[j];
    const double mu64 = sum / m;
    double v = 0.0;
    for (int j = 0; j < m; ++j) {
        const double d = (double)w[j] - mu64;
        v += d * d;
    }
    const double sigma = sqrt(v / m);
    const double inv = sigma <= kSigmaFlat ? 0.0 : 1.0 / sigma;
    mu = (float)mu64;
    s = (float)inv;
    o = (float)(-(mu64 - (double)mu) * inv);
}



// Lane DTW kernels with bands of at least kBoundMinNC chunks (97 cells and more) may add a bound of
// the columns still to come to their abandoning test.  Every warping path visits every later column
// j, in a cell of a row i with |i - j| <= r, whose cost (q_i - c_j)^2 is at least the LB_Keogh term
// of c_j against the query envelope (eq. (LBKeoghEC)), because L_j <= q_i <= U_j.  So after column
// j the distance is at least the band minimum plus the terms of the columns after j.
constexpr int kBoundMinNC = 7;
constexpr int kBoundBlocks = 64;                                    // suffix entries per lane
constexpr size_t kBoundLdsBytes = sizeof(float) * kBoundBlocks * 256;   // per 256-lane workgroup

// Columns per suffix block for a window of m points: a multiple of 16 (the abandoning test runs
// after every 16th column) with at most kBoundBlocks blocks.
__device__ __forceinline__ int bound_block(int m) { return 16 * ((m + 16 * kBoundBlocks - 1) / (16 * kBoundBlocks)); }

// Suffix sums of the query-envelope LB_Keogh terms of one lane's candidate, block b of G columns:
// sfx[256 b] = the sum of the terms of columns b G .. m-1, for b < ceil(m / G).  sfx points at the
// lane's own entry of a [kBoundBlocks][256] LDS array, so only this lane touches it.  Un, Ln: the
// query envelope in natural order (the same FP32 values the DTW cells use); the candidate value is
// the one the DTW computes, fma(t - mu, s, o).  Each term is the single non-zero one of
// max(c - U, 0) and max(L - c, 0), squared.
__device__ __forceinline__ void bound_suffix(const float *Tp, float mu, float s, float o, const float *Un,
                                             const float *Ln, int m, int G, float *sfx) {
    const int nb = (m + G - 1) / G;
    float acc = 0.0f;
    for (int b = nb - 1; b >= 0; --b) {
        const int j0 = b * G, j1 = j0 + G < m ? j0 + G : m;
        float part = 0.0f;
#pragma unroll 16
        for (int j = j0; j < j1; ++j) {
            const float c = fmaf(Tp[j] - mu, s, o);
            const float e = fmaxf(c - Un[j], 0.0f) + fmaxf(Ln[j] - c, 0.0f);
            part = fmaf(e, e, part);
        }
        acc += part;
        sfx[256 * b] = acc;
    }
}

// Banded DTW of one candidate per lane (register kernel; see dtw.hip).  qpad: the query's sentinel-padded
// normalised values; key: best-so-far key read for abandoning (null: use thr0 only).  Returns the
// distance in D and whether the lane stayed within the threshold; jdead is the number of columns
// completed before abandoning and jrun the number of columns the wave executed.  sfx (or null):
// the lane's suffix bounds from bound_suffix with blocks of G columns, added to the band minimum in
// the abandoning test.
template <int NC>
__device__ __forceinline__ void dtw_lanes(const float *T, int64_t start, float mu, float s, float o,
                                          const float *qpad, int m, int r, bool live, const uint64_t *key,
                                          float thr0, bool &alive, float &D, int &jdead, int &jrun,
                                          const float *sfx = nullptr, int G = 16) {
    constexpr int W = 16 * NC;
    constexpr int R = 8 * NC - 1;
    const int ql = threadIdx.x & 15;
    // the query value of band slot k = 16 cc + ql at column j is q_{j-R+k} = qb[j + 16 cc]: one base
    // pointer and immediate offsets.  NC is the smallest with 8 NC - 1 >= r, so the slots outside the
    // band lie in the first chunk (k < R - r <= 7) and the last (k > R + r >= 16 NC - 9); they take the
    // sentinel.  With one or two chunks a per-chunk offset that points the outside slots at the
    // padding is cheaper (no select on a column of only 16 or 32 cells): measured 6-10% faster there.
    const float *qb = qpad + (kQPad - R + ql);
    const bool inlo = ql >= R - r, inhi = 16 * (NC - 1) + ql <= R + r;
    int qoff[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
        const int kpos = 16 * cc + ql;
        qoff[cc] = (kpos >= R - r && kpos <= R + r) ? kQPad - R + kpos : 0;
    }
    auto qload = [&](float (&q)[NC], int jj) {
        if constexpr (NC <= 2) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) q[cc] = qpad[qoff[cc] + jj];
        } else {
            const float *qj = qb + jj;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) q[cc] = qj[16 * cc];
            q[0] = inlo ? q[0] : kSentinel;
            q[NC - 1] = inhi ? q[NC - 1] : kSentinel;
        }
    };
    float arr[W + 1];
#pragma unroll
    for (int x = 0; x <= W; ++x) arr[x] = INFINITY;
    arr[R] = 0.0f;   // d(-1,-1) of the virtual column before column 0
    float thr = key ? fminf(thr0, threshold_of(load_bsf(key))) : thr0;
    // the best-so-far is re-read every 16 columns; each read is issued 16 columns before its use
    uint32_t kpend = key ? load_key_dist_bits(key) : ~0u;
    alive = live;
    jdead = m;
    const float *Tp = T + start;
    float qcur[NC];
    qload(qcur, 0);
    if constexpr (NC <= 3) {
        // narrow bands: a column is little work (16 NC cells), so one column of work cannot cover
        // the latency of the next column's series load; the series comes in blocks of 16 columns,
        // the next block's loads issued before this block's columns (indices clamped to the window)
        float tb[16], tn[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) tb[u] = Tp[u < m ? u : m - 1];
        int j0 = 0;
        for (; j0 < m; j0 += 16) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int jj = j0 + 16 + u;
                tn[u] = Tp[jj < m ? jj : m - 1];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int jc = j0 + u;
                if (jc < m) {
                    const int jn = jc + 1 < m ? jc + 1 : jc;
                    float qnext[NC];
                    qload(qnext, jn);
                    column<NC>(arr, qcur, fmaf(tb[u] - mu, s, o));
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc) qcur[cc] = qnext[cc];
                }
            }
            if (j0 + 16 <= m) {
                // the check after every 16 columns, as below
                float mn = arr[0];
#pragma unroll
                for (int x = 1; x < W; ++x) mn = fminf(mn, arr[x]);
                if (key) {
                    thr = fminf(thr0, threshold_of(__uint_as_float(kpend)));
                    kpend = load_key_dist_bits(key);
                }
                if (alive && mn > thr) {
                    alive = false;
                    jdead = j0 + 16;
                }
                if (__ballot(alive) == 0) {
                    j0 += 16;
                    break;
                }
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) tb[u] = tn[u];
        }
        jrun = j0 < m ? j0 : m;
        D = arr[R];
        if (alive && !(D <= thr)) alive = key ? false : alive;   // search mode keeps only improvements
        return;
    }
    float tcur = Tp[0];
    int j = 0;
    for (; j < m; ++j) {
        const int jn = j + 1 < m ? j + 1 : j;
        const float tnext = Tp[jn];
        float qnext[NC];
        qload(qnext, jn);
        const float c = fmaf(tcur - mu, s, o);
        column<NC>(arr, qcur, c);
        tcur = tnext;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) qcur[cc] = qnext[cc];
        if ((j & 15) == 15) {
            float mn = arr[0];
#pragma unroll
            for (int x = 1; x < W; ++x) mn = fminf(mn, arr[x]);
            if (key) {
                thr = fminf(thr0, threshold_of(__uint_as_float(kpend)));
                kpend = load_key_dist_bits(key);
            }
            if (sfx) {
                // plus the bound of the columns after j from the first whole block after them
                const int b = (j + G) / G;
                if (b * G < m) mn += sfx[256 * b];
            }
            if (alive && mn > thr) {
                alive = false;
                jdead = j + 1;
            }
            if (__ballot(alive) == 0) {
                ++j;
                break;
            }
        }
    }
    jrun = j;
    D = arr[R];
    if (alive && !(D <= thr)) alive = key ? false : alive;   // search mode keeps only improvements
}

// Normalisation parameters of a candidate from FP64 mean and sigma (eq. (Normalization1)):
// c_j = fma(T[i+j] - mu32, s, o) with s = 1/sigma (0 for a flat window), o = -(mu - mu32) * s.
__device__ inline void norm_params(double mu, double sigma, float &mu32, float &s, float &o) {
    const double inv = sigma <= kSigmaFlat ? 0.0 : 1.0 / sigma;
    mu32 = (float)mu;
    s = (float)inv;
    o = (float)(-(mu - (double)mu32) * inv);
}

}  // namespace dtws
