// Tiled bound cascade of the batched search, for the rounds in which every query of the batch visits
// the same candidates (series order, or one round over all blocks after the learned seeding).
//
// The cascade is the one of Section 2.2 (LB_KimFL, then LB_Keogh against the query envelope, then
// LB_Keogh against the data envelope, each pruning against the query's best-so-far), but the work
// is cut by series tile instead of by query.  One workgroup takes kTileC consecutive candidate
// starts: it stages the tile's series points and the (m - 1)-point halo in LDS once, computes the
// candidates' normalisation once per distinct query length (in queries sorted by length), keeps each
// candidate's normalised first and last points in registers, and then runs every query of that
// length over the tile:
//   level 0  LB_KimFL of the lane's candidates from registers (five VALU operations per query and
//            candidate), survivors compacted into the wave's LDS list;
//   level 1  the first kK1 query-envelope terms of LB_Keogh on full waves of survivors, the series
//            values read from the LDS tile (terms in the query's visiting order, wave-uniform, so the
//            query side comes through scalar loads), abandoning by blocks of 16;
//   level 2  the remaining terms and the data-envelope bound on full waves of level-1 survivors
//            (a ring of 128 entries per wave, drained when a query ends);
// survivors (query, start) go to the batch's survivor list as in the per-query kernel.  The series
// is read from HBM once per round for all queries; the window statistics once per tile and length.
#include "batch_stats.h"

namespace dtws {

constexpr int kTileC = 2048;                                 // candidates per tile
constexpr int kTileWaves = 4;
constexpr int kTileWaveC = kTileC / kTileWaves;              // candidates per wave
constexpr int kTilePerLane = kTileWaveC / 64;                // candidates per lane
constexpr int kTileQ2 = 128;                                 // level-2 ring per wave (power of two)

static_assert(kTilePerLane * 64 * kTileWaves == kTileC, "tile split");

// One block of 16 query-envelope terms from the LDS tile (Tl = the candidate's first point).
__device__ __forceinline__ float keogh_q_lds16(const QView &v, const float *Tl, float mu, float s, float o, float kq,
                                               int k0) {
    float tv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) tv[u] = Tl[ldc(v.order + k0 + u)];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float c = fmaf(tv[u] - mu, s, o);
        const float e = fmaxf(fmaxf(c - ldc(v.Us + k0 + u), ldc(v.Ls + k0 + u) - c), 0.0f);
        kq = fmaf(e, e, kq);
    }
    return kq;
}

// Terms [k0, k1) (multiples of 16) with abandoning when no live lane is within the threshold.
// `terms` counts the terms evaluated for a live lane.
__device__ __forceinline__ float keogh_q_lds(const QView &v, const float *Tl, float mu, float s, float o, float kq,
                                             int k0, int k1, bool live, float thr, uint32_t &terms) {
    for (int k = k0; k < k1; k += 16) {
        kq = keogh_q_lds16(v, Tl, mu, s, o, kq, k);
        terms += live ? 16u : 0u;
        if (__ballot(live && !(kq > thr)) == 0) break;
    }
    return kq;
}

size_t tile_lds_bytes(int max_m) {
    const int tlen = (kTileC + max_m - 1 + 3) & ~3;
    return sizeof(float) * ((size_t)tlen + 3 * kTileC) + sizeof(int32_t) * kTileC +
           (sizeof(int32_t) + sizeof(float)) * kTileWaves * kTileQ2;
}

template <bool PREFIX, bool ENV>
__global__ __launch_bounds__(256) void k_lb_tile(BatchArgs a, TileArgs t) {
    extern __shared__ float lds_t[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tlen = (kTileC + t.halo + 3) & ~3;
    float *Tt = lds_t;
    float *smu = Tt + tlen, *ssg = smu + kTileC, *sof = ssg + kTileC;
    int32_t *q1 = (int32_t *)(sof + kTileC) + wid * kTileWaveC;
    int32_t *q2i = (int32_t *)(sof + kTileC) + kTileC + wid * kTileQ2;
    float *q2k = (float *)((int32_t *)(sof + kTileC) + kTileC + kTileWaves * kTileQ2) + wid * kTileQ2;
    const int64_t t0 = t.c_lo + (int64_t)blockIdx.x * kTileC;
    for (int x = tid; x < kTileC + t.halo; x += blockDim.x) {
        const int64_t y = t0 + x;
        Tt[x] = y < a.n ? a.T[y] : 0.0f;
    }
    CascadeCounts cnt;
    uint32_t terms = 0;   // query-envelope terms evaluated (this lane)
    for (int g = 0; g < t.ngroups; ++g) {
        const int qbeg = t.gfirst[g], qend = t.gfirst[g + 1];
        const BatchQ b0 = a.bq[t.qlist[qbeg]];
        const int m = b0.m;
        const int64_t cend = t.c_hi < b0.N ? t.c_hi : b0.N;
        __syncthreads();   // the tile is staged; the previous length's statistics are no longer read
        if (t0 >= cend) continue;   // the same for the whole workgroup
        // normalisation of the tile's candidates for this length (coalesced)
        for (int k = tid; k < kTileC; k += blockDim.x) {
            const int64_t i = t0 + k;
            float mu = 0.0f, s = 0.0f, o = 0.0f;
            if (i < cend) {
                if (PREFIX) {
                    StatsPrefix{a.T, a.pre, m, 1.0 / m}(i, mu, s, o);
                } else {
                    const int64_t so = b0.stat_slot * a.slot_stride;
                    StatsArr{a.mu + so, a.s + so, a.o + so}(i, mu, s, o);
                }
            }
            smu[k] = mu;
            ssg[k] = s;
            sof[k] = o;
        }
        __syncthreads();
        // the lane's candidates: normalised first and last points
        float c0[kTilePerLane], cl[kTilePerLane];
        uint32_t vmask = 0;
#pragma unroll
        for (int u = 0; u < kTilePerLane; ++u) {
            const int local = wid * kTileWaveC + u * 64 + lane;
            const float mu = smu[local], s = ssg[local], o = sof[local];
            c0[u] = fmaf(Tt[local] - mu, s, o);
            cl[u] = fmaf(Tt[local + m - 1] - mu, s, o);
            if (t0 + local < cend) vmask |= 1u << u;
        }
        for (int qi = qbeg; qi < qend; ++qi) {
            const int q = __builtin_amdgcn_readfirstlane(ldc(t.qlist + qi));
            // a block this query visited in an earlier round (the tile lies inside one block)
            if (t.skip_below > 0 && ldc(a.rank + (int64_t)q * a.maxblocks + t0 / t.block) < t.skip_below) continue;
            const float *qh = a.qpad + (int64_t)q * a.qstride + kQPad;
            const float q0 = ldc(qh), ql = ldc(qh + m - 1);
            const float thr = threshold_of(load_bsf(a.keys + q));
            // level 0: LB_KimFL, survivors into the wave's list in candidate order
            uint32_t n1 = 0;
#pragma unroll
            for (int u = 0; u < kTilePerLane; ++u) {
                const float d0 = q0 - c0[u], dl = ql - cl[u];
                const bool valid = (vmask >> u) & 1u;
                const bool alive = valid && !(fmaf(d0, d0, dl * dl) > thr);
                const uint64_t mk = __ballot(alive);
                if (alive) q1[n1 + rank_in(mk)] = wid * kTileWaveC + u * 64 + lane;
                n1 += (uint32_t)__popcll(mk);
                cnt.kim_w += (uint32_t)(__popcll(__ballot(valid)) - __popcll(mk));
            }
            if (n1 == 0) continue;
            wave_sync();
            const QView v{a.order + q * a.mstride, a.Us + q * a.mstride, a.Ls + q * a.mstride, a.qs + q * a.mstride, m,
                          (m + 15) & ~15};
            const int K1 = v.mpad < kK1 ? v.mpad : kK1;
            const EmitBatch emit{a.surv_q, a.surv_i, a.surv_lb, a.surv_count, a.qcnt, a.overflow, a.surv_cap, q};
            const int eslot = ENV ? a.bq[q].env_slot : 0;
            const float *eU = ENV && a.envU ? a.envU + eslot * a.slot_stride : nullptr;
            const float *eL = ENV && a.envU ? a.envL + eslot * a.slot_stride : nullptr;
            uint32_t h2 = 0, t2 = 0;   // level-2 ring (wave-uniform head and tail)
            // level 2 on up to 64 ring entries: the remaining query-envelope terms, then the data
            // envelope; survivors are emitted
            auto level2 = [&]() {
                const uint32_t avail = t2 - h2, take = avail < 64u ? avail : 64u;
                const bool got = (uint32_t)lane < take;
                const uint32_t p = (h2 + (got ? (uint32_t)lane : 0u)) & (kTileQ2 - 1);
                const int local = q2i[p];
                float kq = q2k[p];
                h2 += take;
                const float mu = smu[local], s = ssg[local], o = sof[local];
                kq = keogh_q_lds(v, Tt + local, mu, s, o, kq, K1, v.mpad, got, thr, terms);
                bool alive = got && !(kq > thr);
                if (got && !alive) ++cnt.kq;
                if (ENV && eU && __ballot(alive)) {
                    const int64_t i = t0 + local;
                    const float kd = keogh_d(v, eU + i, eL + i, mu, s, o, thr);
                    if (alive && kd > thr) {
                        alive = false;
                        ++cnt.kd;
                    }
                }
                emit(alive, t0 + local, kq);
                wave_sync();
            };
            for (uint32_t b = 0; b < n1; b += 64) {
                const bool got = b + (uint32_t)lane < n1;
                const int local = q1[got ? b + lane : b];
                const float mu = smu[local], s = ssg[local], o = sof[local];
                const float kq = keogh_q_lds(v, Tt + local, mu, s, o, 0.0f, 0, K1, got, thr, terms);
                const bool alive = got && !(kq > thr);
                if (got && !alive) ++cnt.kq;
                const uint64_t mk = __ballot(alive);
                if (alive) {
                    const uint32_t p = (t2 + rank_in(mk)) & (kTileQ2 - 1);
                    q2i[p] = local;
                    q2k[p] = kq;
                }
                t2 += (uint32_t)__popcll(mk);
                wave_sync();
                if (t2 - h2 >= 64u) level2();   // the ring holds < 64 before a push of <= 64
            }
            while (t2 != h2) level2();
        }
    }
    if (a.counters) {
        const unsigned long long c_kim = cnt.wave_kim(), c_kq = wave_add_u64(cnt.kq), c_kd = wave_add_u64(cnt.kd),
                                 c_terms = wave_add_u64(terms);
        if (lane == 0) {
            atomicAdd(&a.counters[1], c_kim);
            atomicAdd(&a.counters[2], c_kq);
            atomicAdd(&a.counters[3], c_kd);
            atomicAdd(&a.counters[9], c_terms);
        }
    }
}

hipError_t launch_lb_tile(const BatchArgs &a, const TileArgs &t, bool prefix, int64_t max_N, hipStream_t s) {
    const int64_t hi = t.c_hi < max_N ? t.c_hi : max_N;
    if (hi <= t.c_lo) return hipSuccess;
    const int64_t tiles = (hi - t.c_lo + kTileC - 1) / kTileC;
    const size_t lds = tile_lds_bytes(t.halo + 1);
    const bool env = a.envU != nullptr;
    const dim3 g((unsigned)tiles), b(256);
    if (prefix && env) hipLaunchKernelGGL((k_lb_tile<true, true>), g, b, lds, s, a, t);
    else if (prefix) hipLaunchKernelGGL((k_lb_tile<true, false>), g, b, lds, s, a, t);
    else if (env) hipLaunchKernelGGL((k_lb_tile<false, true>), g, b, lds, s, a, t);
    else hipLaunchKernelGGL((k_lb_tile<false, false>), g, b, lds, s, a, t);
    return hipGetLastError();
}

}  // namespace dtws
