// Batched search: many queries of different lengths and bands against one series.
//
// Work is a device queue of items (query, block of consecutive candidate starts).  Each query's
// blocks are visited in a per-query order (series order, a seeded permutation, or the learned
// model's ranking) and in rounds: the first 64K candidates of every query, then the next 1M,
// the next 16M, then the rest.  A round is one persistent launch of the bound cascade over all
// queries' items (waves pop items from an atomic head); survivors (query, start) are then
// counting-sorted into per-query segments padded to whole waves, grouped by DTW band bucket, and
// one DTW launch per bucket covers every query of that bucket.  The best-so-far of each query
// lives in device memory throughout (the reduction of Algorithm 1 becomes an atomic minimum on
// a packed (distance, index) key) and every later round prunes with the tighter values.
//
// Window statistics for any query length come from one blocked prefix of the series: FP64 sums
// of (t - a_b) and (t - a_b)^2 anchored at the first point a_b of each 4096-point block, so a
// window's sums are a difference of two nearby partial sums (re-anchored when the window crosses
// one block boundary; m <= 2048 < 4096 crosses at most one).  When all queries share one length
// the per-window arrays of the statistics pass are used instead.
#include "batch_stats.h"

namespace dtws {

constexpr int kPrefixThreads = 256;  // 16 points per thread

__device__ inline uint64_t splitmix64_d(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// ------------------------------------------------------------------ blocked prefix
// One workgroup per block of kPB points: each thread scans 16 consecutive points in FP64, the
// workgroup scans the thread totals, and the results leave through LDS in two halves so that the
// stores are coalesced.
__global__ __launch_bounds__(kPrefixThreads) void k_prefix(const float *__restrict__ T, int64_t n, double2 *PPe,
                                                           double *anc, double2 *tot, Decimated dec,
                                                           uint32_t levels) {
    constexpr int kHalf = kPB / 2, kPad = 16 + 1;           // 16 entries per thread, one spare
    __shared__ double2 stage[kPrefixThreads / 2 * kPad];
    __shared__ double ws1[kPrefixThreads / 64], ws2[kPrefixThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t b = blockIdx.x, x0 = b * kPB;
    const double a = (double)T[x0];
    // this thread's 16 points: four 16-byte loads when the block is whole and the series is
    // 16-byte aligned (x0 is a multiple of 4096), else point by point with a bounds test
    float t[16];
    if (x0 + kPB <= n && ((uintptr_t)T & 15u) == 0) {
        const float4 *T4 = (const float4 *)(T + x0) + 4 * tid;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float4 f = T4[w];
            t[4 * w] = f.x;
            t[4 * w + 1] = f.y;
            t[4 * w + 2] = f.z;
            t[4 * w + 3] = f.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t y = x0 + 16 * tid + u;
            t[u] = y < n ? T[y] : 0.0f;
        }
    }
    double v1[16], v2[16];
    double r1 = 0.0, r2 = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int64_t y = x0 + 16 * tid + u;
        const double d = y < n ? (double)t[u] - a : 0.0;
        v1[u] = r1;
        v2[u] = r2;
        r1 += d;
        r2 += d * d;
    }
    double i1 = r1, i2 = r2;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y1 = __shfl_up(i1, off, 64), y2 = __shfl_up(i2, off, 64);
        if (lane >= off) {
            i1 += y1;
            i2 += y2;
        }
    }
    if (lane == 63) {
        ws1[wid] = i1;
        ws2[wid] = i2;
    }
    __syncthreads();
    double b1 = 0.0, b2 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kPrefixThreads / 64; ++w) {
        if (w < wid) {
            b1 += ws1[w];
            b2 += ws2[w];
        }
        t1 += ws1[w];
        t2 += ws2[w];
    }
    b1 += i1 - r1;
    b2 += i2 - r2;
    const int64_t lim = n + 1 - x0;   // entries [x0, n] exist
    for (int h = 0; h < 2; ++h) {
        const int owner = tid - h * (kPrefixThreads / 2);
        if (owner >= 0 && owner < kPrefixThreads / 2) {
#pragma unroll
            for (int u = 0; u < 16; ++u) stage[owner * kPad + u] = make_double2(b1 + v1[u], b2 + v2[u]);
        }
        __syncthreads();
        // even entries only (consecutive threads write consecutive entries)
        for (int e2 = tid; e2 < kHalf / 2; e2 += kPrefixThreads) {
            const int e = 2 * e2;
            const int64_t x = (int64_t)h * kHalf + e;
            if (x < lim) PPe[(x0 + x) >> 1] = stage[(e >> 4) * kPad + (e & 15)];
        }
        // decimated copies: consecutive threads write consecutive entries of each level
        for (int L = kDecFirst; L < kDecLevels; ++L) {
            if (!((levels >> L) & 1u)) continue;
            for (int e = tid; e < (kHalf >> L); e += kPrefixThreads) {
                const int el = e << L;   // block-local position within this half
                const int64_t x = (int64_t)h * kHalf + el;
                if (x < lim) dec.lv[L][(x0 + x) >> L] = stage[(el >> 4) * kPad + (el & 15)];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        anc[b] = a;
        tot[b] = make_double2(t1, t2);
        if (b == (int64_t)gridDim.x - 1) {
            // sentinels: the entry past the last block, and PP[n] when n ends a block
            anc[b + 1] = a;
            tot[b + 1] = make_double2(0.0, 0.0);
            if (x0 + kPB == n) {
                PPe[n >> 1] = make_double2(0.0, 0.0);   // n is even here
                for (int L = kDecFirst; L < kDecLevels; ++L)
                    if (((levels >> L) & 1u) && (n & ((1 << L) - 1)) == 0) dec.lv[L][n >> L] = make_double2(0.0, 0.0);
            }
        }
    }
}

// ------------------------------------------------------------------ work order
__device__ inline uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// mode 0: series order; 1: seeded permutation k -> (A k + C) mod nb.  A starts at a seeded value in
// [1, nb - 1] and steps up to the first value coprime to nb (nb - 1 always is), so the map is a
// bijection of [0, nb) for every block count.
__global__ void k_make_perm(BatchArgs a, int mode, uint64_t seed) {
    const int q = blockIdx.y;
    const BatchQ bq = a.bq[q];
    const int64_t nb = bq.nblocks;
    const uint64_t h = splitmix64_d(seed ^ (0x51ED2701ull * (uint64_t)(q + 1)));
    uint64_t A = 1, C = 0;
    if (mode == 1 && nb > 1) {
        A = 1 + h % (uint64_t)(nb - 1);
        while (gcd_u64(A, (uint64_t)nb) != 1) A = A + 1 < (uint64_t)nb ? A + 1 : 1;
        C = (h >> 8) % (uint64_t)nb;
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = k;
        if (mode == 1 && nb > 1) v = (int64_t)((A * (uint64_t)k + C) % (uint64_t)nb);
        a.perm[(int64_t)q * a.maxblocks + k] = (int32_t)v;
    }
}

// The inverse of every query's block order: rank[q][perm[q][k]] = k.
__global__ void k_perm_rank(BatchArgs a) {
    const int q = blockIdx.y;
    const int64_t nb = a.bq[q].nblocks;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x)
        a.rank[(int64_t)q * a.maxblocks + a.perm[(int64_t)q * a.maxblocks + k]] = (int32_t)k;
}

// Round -1: the best-so-far of every query starts from one seeded random candidate (Algorithm 1).
__global__ void k_seed_random(BatchArgs a, uint64_t seed) {
    for (int q = threadIdx.x; q < a.nq; q += blockDim.x) {
        const int64_t N = a.bq[q].N;
        a.surv_q[q] = q;
        a.surv_i[q] = (int32_t)(splitmix64_d(seed + (uint64_t)q) % (uint64_t)N);
        a.surv_lb[q] = 0.0f;
        a.qcnt[q * kCntStride] = 1;
    }
    if (threadIdx.x == 0) *a.surv_count = (uint32_t)a.nq;
}

// ------------------------------------------------------------------ batched bound cascade
// Work-item source of one wave for one query: consumes the current item group by group, pops the
// next item when it runs out, and stops (keeping the popped item) at the first item of another
// query, so the caller can drain the queues before switching query.  Items of round r are
// (query, rank k, part); part selects one of `parts` equal pieces of the k-th block of the
// query's visiting order.  They go out query-major, or block-major in series order when the
// round's blocks are the same for every query (then the waves on the queries of one block run at
// about the same time and share its data through the caches).  The last round of another order
// also goes block-major in series order over every block, each query skipping the blocks it ranked
// below skip_below (those it visited in the earlier rounds): the rest of every query's blocks, in
// an order the queries share.
struct ItemSource {
    const BatchArgs *a;
    int round, rank_lo, parts;
    uint32_t per_q, total;
    int q;                      // query being processed
    int64_t gnext = 0, gend = 0;  // rest of the current item
    bool pending = false;       // an item of another query was popped
    int pq = -1;
    int64_t pfirst = 0, plast = 0;
    bool natural = false;       // the round holds every block: series order, block-major
    bool subq = false;          // natural: in eight sub-queues, one per XCD
    int skip_below = 0;         // natural: skip a query's blocks of rank below this
    uint32_t sub_done = 0;      // natural: sub-queues found empty

    // pops items until one that exists; false when the round is exhausted
    __device__ bool pop(int &qq, int64_t &first, int64_t &last) {
        const int lane = threadIdx.x & 63;
        for (;;) {
            int k = 0, part = 0;
            if (subq) {
                // series order in eight sub-queues: block b goes to the workgroups with
                // blockIdx.x = b (mod 8), which the hardware places on one XCD, so the queries of a
                // block share that XCD's L2; an empty sub-queue sends the wave to the others
                const uint32_t nranks = (uint32_t)(per_q / (uint32_t)parts);
                const int home = (int)(blockIdx.x & 7u);
                bool got = false;
                for (int j = 0; j < 8 && !got; ++j) {
                    const int x = (home + j) & 7;
                    if (sub_done & (1u << x)) continue;
                    uint32_t c = 0;
                    if (lane == 0) c = atomicAdd(&a->heads[round * 8 + x], 1u);
                    c = __builtin_amdgcn_readfirstlane(c);
                    const uint32_t nbx = nranks > (uint32_t)x ? (nranks - (uint32_t)x + 7u) / 8u : 0u;
                    if (c >= nbx * (uint32_t)parts * (uint32_t)a->nq) {
                        sub_done |= 1u << x;
                        continue;
                    }
                    qq = (int)(c % (uint32_t)a->nq);
                    const uint32_t rest = c / (uint32_t)a->nq;
                    k = rank_lo + (int)(rest / (uint32_t)parts) * 8 + x;
                    part = (int)(rest % (uint32_t)parts);
                    got = true;
                }
                if (!got) return false;
            } else {
                uint32_t idx = 0;
                if (lane == 0) idx = atomicAdd(&a->heads[round * 8], 1u);
                idx = __builtin_amdgcn_readfirstlane(idx);   // wave-uniform: item state stays in SGPRs
                if (idx >= total) return false;
                // series order, block-major (the queries of one block one after another), or query
                // by query in visiting order
                uint32_t rest;
                if (natural) {
                    qq = (int)(idx % (uint32_t)a->nq);
                    rest = idx / (uint32_t)a->nq;
                } else {
                    qq = (int)(idx / per_q);
                    rest = idx % per_q;
                }
                k = rank_lo + (int)(rest / (uint32_t)parts);
                part = (int)(rest % (uint32_t)parts);
            }
            const BatchQ bq = a->bq[qq];
            if (k >= bq.nblocks) continue;
            const int64_t blk = natural ? k : a->perm[(int64_t)qq * a->maxblocks + k];
            if (skip_below > 0 && a->rank[(int64_t)qq * a->maxblocks + blk] < skip_below) continue;
            const int64_t piece = a->block / parts;
            first = blk * a->block + part * piece;
            if (first >= bq.N) continue;
            last = first + piece < bq.N ? first + piece : bq.N;
            return true;
        }
    }

    // the rest of the current item as one run, or the next item of this query
    __device__ bool next_run(int64_t &g, int64_t &last) {
        if (gnext >= gend) {
            int qq;
            int64_t f, l;
            if (!pop(qq, f, l)) return false;
            if (qq != q) {
                pending = true;
                pq = qq;
                pfirst = f;
                plast = l;
                return false;
            }
            gnext = f;
            gend = l;
        }
        g = gnext;
        last = gend;
        gnext = gend;
        return true;
    }

    __device__ bool next(int64_t &g, int64_t &last) {
        if (gnext >= gend) {
            int qq;
            int64_t f, l;
            if (!pop(qq, f, l)) return false;
            if (qq != q) {
                pending = true;
                pq = qq;
                pfirst = f;
                plast = l;
                return false;
            }
            gnext = f;
            gend = l;
        }
        g = gnext;
        last = gend;
        gnext += 64;
        return true;
    }
};

template <bool PREFIX, bool ENV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_lb_batch(BatchArgs a, int round,
                                                                                     int rank_lo, int rank_hi, int parts,
                                                                                     int natural, int skip_below) {
    __shared__ WaveQueue q1s[4];
    __shared__ WaveQueue2 q2s[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    ItemSource src{&a, round, rank_lo, parts, (uint32_t)(rank_hi - rank_lo) * (uint32_t)parts, 0u, -1};
    src.total = src.per_q * (uint32_t)a.nq;
    src.natural = (natural & 1) != 0;
    src.subq = (natural & 2) != 0;
    src.skip_below = skip_below;
    CascadeCounts cnt;
    int q;
    int64_t f, l;
    if (!src.pop(q, f, l)) goto finish;
    for (;;) {
        src.q = q;
        src.gnext = f;
        src.gend = l;
        src.pending = false;
        {
            const BatchQ bq = a.bq[q];
            const QView v{a.order + q * a.mstride, a.Us + q * a.mstride, a.Ls + q * a.mstride,
                          a.qs + q * a.mstride, bq.m, (bq.m + 15) & ~15};
            const float *qh = a.qpad + q * a.qstride + kQPad;
            const float thr = threshold_of(load_bsf(a.keys + q));
            const EmitBatch emit{a.surv_q, a.surv_i, a.surv_lb, a.surv_count, a.qcnt, a.overflow, a.surv_cap, q};
            const float *eU = a.envU ? a.envU + bq.env_slot * a.slot_stride : nullptr;
            const float *eL = a.envU ? a.envL + bq.env_slot * a.slot_stride : nullptr;
            if (PREFIX) {
                cascade<ENV>(v, a.T, eU, eL, thr, qh, src, q1s[wid], q2s[wid],
                        StatsPrefix{a.T, a.pre, bq.m, 1.0 / bq.m}, emit, cnt);
            } else {
                const int64_t so = bq.stat_slot * a.slot_stride;
                cascade<ENV>(v, a.T, eU, eL, thr, qh, src, q1s[wid], q2s[wid],
                        StatsArr{a.mu + so, a.s + so, a.o + so}, emit, cnt);
            }
        }
        if (!src.pending) break;
        q = src.pq;
        f = src.pfirst;
        l = src.plast;
    }
finish:
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

// ------------------------------------------------------------------ survivor segments
// Queries in bucket order; each query's survivors get ceil(count / 64) whole waves, so a DTW
// wave never mixes queries (the query window is broadcast across the wave).  bucket_w[2c] /
// bucket_w[2c+1] are the wave range of bucket c and bucket_j[2c] / bucket_j[2c+1] its range of
// positions in qorder / wstart.
__global__ void k_seg_plan(BatchArgs a) {
    if (threadIdx.x != 0) return;
    int32_t off = 0, j = 0;
    for (int c = 1; c <= kMaxChunks + 1; ++c) {
        a.bucket_w[2 * c] = off;
        a.bucket_j[2 * c] = j;
        for (int q = 0; q < a.nq; ++q) {
            if (a.bq[q].nc != c) continue;
            a.qorder[j] = q;
            a.wstart[j] = off;
            a.seg_off[q] = (int64_t)off * 64;
            a.fill[q * kCntStride] = 0;
            off += (int32_t)((a.qcnt[q * kCntStride] + 63u) / 64u);
            ++j;
        }
        a.bucket_w[2 * c + 1] = off;
        a.bucket_j[2 * c + 1] = j;
    }
    a.wstart[j] = off;
}

__global__ void k_seg_scatter(BatchArgs a) {
    if (*a.overflow) return;
    uint32_t cnt = *a.surv_count;
    if ((int64_t)cnt > a.surv_cap) cnt = (uint32_t)a.surv_cap;
    const int lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < cnt; base += stride) {
        const uint32_t e = base + lane;
        const bool valid = e < cnt;
        const int q = valid ? a.surv_q[e] : -1;
        // one atomic per distinct query among the wave's 64 entries
        uint64_t pending = __ballot(valid);
        uint32_t pos = 0;
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int q0 = __shfl(q, leader, 64);
            const uint64_t peers = __ballot(valid && q == q0);
            uint32_t b0 = 0;
            if (lane == leader) b0 = atomicAdd(&a.fill[q0 * kCntStride], (uint32_t)__popcll(peers));
            b0 = __shfl(b0, leader, 64);
            if (valid && q == q0) pos = b0 + (uint32_t)__popcll(peers & lanemask_lt());
            pending &= ~peers;
        }
        if (valid) {
            a.sorted[a.seg_off[q] + pos] = a.surv_i[e];
            a.sorted_lb[a.seg_off[q] + pos] = a.surv_lb[e];
        }
    }
}

template <class Stats>
__device__ inline void stats_of(const Stats &st, int64_t i, float &mu, float &s, float &o) {
    st(i, mu, s, o);
}

// ------------------------------------------------------------------ batched DTW (register kernel)
template <int NC, bool PREFIX>
__global__ __launch_bounds__(256) void k_dtw_batch(BatchArgs a) {
    constexpr int W = 16 * NC;
    extern __shared__ float bound_lds[];   // [kBoundBlocks][256] when the suffix bound is on
    if (*a.overflow || *a.surv_count <= a.diag_max) return;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t wlo = a.bucket_w[2 * NC], whi = a.bucket_w[2 * NC + 1];
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0, n_lane_cells = 0;
    for (int64_t w = wlo + wave; w < whi; w += nwaves) {
        int32_t wq0;
        const int q = wave_query(a, NC, w, wq0);
        const BatchQ bq = a.bq[q];
        const int64_t local = (w - wq0) * 64 + lane;
        const bool valid = local < (int64_t)a.qcnt[q * kCntStride];
        const int64_t start = valid ? (int64_t)a.sorted[w * 64 + lane] : 0;
        float mu, s, o;
        if (PREFIX) {
            StatsPrefix{a.T, a.pre, bq.m, 1.0 / bq.m}(start, mu, s, o);
        } else {
            const int64_t so = bq.stat_slot * a.slot_stride;
            StatsArr{a.mu + so, a.s + so, a.o + so}(start, mu, s, o);
        }
        const float *sfx = nullptr;
        int G = 16;
        if constexpr (NC >= kBoundMinNC) {
            if (a.Un) {
                const int64_t qo = (int64_t)__builtin_amdgcn_readfirstlane(q) * a.mstride;
                G = bound_block(bq.m);
                bound_suffix(a.T + start, mu, s, o, a.Un + qo, a.Ln + qo, bq.m, G, bound_lds + threadIdx.x);
                sfx = bound_lds + threadIdx.x;
            }
        }
        bool alive;
        float D;
        int jdead, jrun;
        dtw_lanes<NC>(a.T, start, mu, s, o, a.qpad + q * a.qstride, bq.m, bq.r, valid, a.keys + q, INFINITY,
                      alive, D, jdead, jrun, sfx, G);
        n_lane_cells += (unsigned long long)jrun * W;
        if (valid) {
            ++n_started;
            if (jdead < bq.m) ++n_aband;
            n_cells += band_cells(bq.m, bq.r, jdead);
            if (alive) {
                atomicMin((unsigned long long *)(a.keys + q), (unsigned long long)pack_key(D, (uint32_t)start));
                const uint32_t pos = atomicAdd(a.nb_count, 1u);
                if (pos < a.nb_cap) {
                    a.nb_d[pos] = D;
                    a.nb_idx[pos] = (uint32_t)start;
                    a.nb_q[pos] = q;
                }
            }
        }
    }
    if (a.counters) {
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

// The same DTW with refilling rows.  A wave's lanes abandon their candidates at different columns,
// and a wave that holds 64 candidates runs until the last of them ends.  Here a wave owns a chunk
// of up to kRowChunk consecutive waves' worth of survivors and works on it as four independent rows
// of 16 lanes (the query broadcast never leaves a 16-lane row, so the rows need not share the
// column or even the query): whenever every lane of a row has ended its candidate, the row takes
// the chunk's next 16 survivors and starts them at column 0.  All rows start at column 0 and end
// candidates only at the test every 16 columns, so the tests stay aligned across the wave.  A
// candidate that completes its last column (m - 1) between two tests keeps its distance from that
// column; its row runs on (on clamped inputs) until the test.
// The test also adds the query-envelope LB_Keogh terms of the columns still to come: the cascade's
// full sum for the candidate (sorted_lb) minus the terms of the columns done, which the lane adds up
// as it goes (one term per column, on the value the column uses).  The two sums round differently
// by far less than the threshold's slack.  Without the suffix bound (a.Un null) the total is 0 and
// the terms run on the query itself, so the bound adds max(0 - terms, 0) = 0 (no branch in the
// column loop, which would cost registers).
//
// Eviction (a.ev_live > 0).  Neighbouring starts abandon at nearly the same column, but a row still
// runs until its last candidate ends, so most of its idle lanes sit in rows where one to a few
// candidates run on.  At a test, a row with 1..ev_live live candidates and at least two tests to go
// moves them out: band column, running suffix terms and position into entries of a.ev_out, and
// takes the next 16 candidates.  The moved candidates are bucketed by (query, column) and resumed
// by the RESUME instance of this kernel in full rows of 16 that share query and column, so the
// query broadcast still holds.  A candidate's arithmetic does not change when it moves: the same
// values continue from the same column.  When ev_out is full a row keeps its candidates.
constexpr int kRowChunk = 32;

template <int NC, bool PREFIX, bool RESUME>
__global__ __launch_bounds__(256) void k_dtw_batch_rows(BatchArgs a) {
    constexpr int W = 16 * NC;
    constexpr int R = 8 * NC - 1;
    static_assert(W + 1 <= kEvKpre, "eviction entry layout");
    if (*a.overflow || *a.surv_count <= a.diag_max) return;
    const int lane = threadIdx.x & 63, row = lane >> 4, ql = lane & 15;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // work: waves of 64 survivors (4 rows each) of this bucket, or resume rows of 16 entries
    const int64_t wlo = RESUME ? 0 : a.bucket_w[2 * NC];
    const int64_t whi = RESUME ? ((int64_t)*a.ev_rows + 3) / 4 : a.bucket_w[2 * NC + 1];
    const int64_t nrows_total = RESUME ? (int64_t)*a.ev_rows : 4 * (whi - wlo);
    // chunks of up to kRowChunk waves, fewer when the bucket would not give every wave one
    int64_t cw = (whi - wlo) / nwaves;
    cw = cw < 1 ? 1 : (cw > kRowChunk ? kRowChunk : cw);
    const int64_t nchunks = (whi - wlo + cw - 1) / cw;
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0, n_steps = 0, n_evicted = 0;
    const bool bound = a.Un != nullptr;
    const float *Ubase = bound ? a.Un : a.qpad + kQPad, *Lbase = bound ? a.Ln : a.qpad + kQPad;
    const int64_t ustride = bound ? a.mstride : a.qstride;
    for (int64_t ch = wave; ch < nchunks; ch += nwaves) {
        const int64_t w0 = wlo + ch * cw;
        const int64_t w1 = w0 + cw < whi ? w0 + cw : whi;
        // rows of 16 in the chunk (a resume chunk's last wave may hold fewer than 4)
        int64_t nsl = (w1 - w0) * 4;
        if (RESUME && (w0 - wlo) * 4 + nsl > nrows_total) nsl = nrows_total - (w0 - wlo) * 4;
        const int nslots = (int)nsl;
        // per-lane state of the lane's current candidate
        int q = 0, m = 2, r = 0, jl = 0, j0 = 0, jdead = 0;
        bool valid = false, alive = false, live = false;
        float mu = 0.0f, s = 0.0f, o = 0.0f, thr = INFINITY, D = INFINITY, tcur = 0.0f;
        float lbt = 0.0f, kpre = 0.0f, ucur = 0.0f, lcur = 0.0f;   // suffix bound: total, terms done
        const float *Tp = a.T, *qp = a.qpad, *Unp = Ubase, *Lnp = Lbase;
        const uint64_t *key = a.keys;
        uint32_t kpend = ~0u;
        // the query value of band slot 16 cc + ql at column j is qb[j + 16 cc]; the slots outside
        // the band (only in the first and the last chunk, since 8 NC - 8 <= r <= 8 NC - 1) take the
        // sentinel instead, so that their cells cost infinity
        const float *qb = a.qpad;
        bool inlo = false, inhi = false;
        float arr[W + 1], qcur[NC];
#pragma unroll
        for (int x = 0; x <= W; ++x) arr[x] = INFINITY;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) qcur[cc] = 0.0f;
        // this lane's row takes row slot `slot` of the chunk
        auto take = [&](int slot) {
            int64_t start = 0;
            const float *ent = nullptr;
            if (RESUME) {
                const uint32_t e = a.ev_order[((w0 - wlo) * 4 + slot) * 16 + ql];
                valid = e != ~0u;
                // an empty lane copies the row's first entry (rows never start empty) and stays idle
                const uint32_t e0 = a.ev_order[((w0 - wlo) * 4 + slot) * 16];
                ent = a.ev_in + (int64_t)(valid ? e : e0) * kEvStride;
                q = __float_as_int(ent[kEvQ]);
                start = (int64_t)(uint32_t)__float_as_int(ent[kEvStart]);
                j0 = __float_as_int(ent[kEvCol]);
            } else {
                const int64_t wv = w0 + slot / 4;
                int32_t wq0;
                q = wave_query(a, NC, wv, wq0);
                const int64_t off = (int64_t)(slot & 3) * 16 + ql;
                valid = (wv - wq0) * 64 + off < (int64_t)a.qcnt[q * kCntStride];
                start = valid ? (int64_t)a.sorted[wv * 64 + off] : 0;
                j0 = 0;
                lbt = bound && valid ? a.sorted_lb[wv * 64 + off] : 0.0f;
                kpre = 0.0f;
            }
            const BatchQ bq = a.bq[q];
            m = bq.m;
            r = bq.r;
            if (PREFIX) {
                StatsPrefix{a.T, a.pre, m, 1.0 / m}(start, mu, s, o);
            } else {
                const int64_t so = bq.stat_slot * a.slot_stride;
                StatsArr{a.mu + so, a.s + so, a.o + so}(start, mu, s, o);
            }
            qp = a.qpad + q * a.qstride;
            key = a.keys + q;
            Unp = Ubase + q * ustride;
            Lnp = Lbase + q * ustride;
            ucur = Unp[j0];
            lcur = Lnp[j0];
            qb = qp + (kQPad - R + ql);
            inlo = ql >= R - r;
            inhi = 16 * (NC - 1) + ql <= R + r;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) qcur[cc] = qb[j0 + 16 * cc];
            qcur[0] = inlo ? qcur[0] : kSentinel;
            qcur[NC - 1] = inhi ? qcur[NC - 1] : kSentinel;
            if (RESUME) {
                lbt = ent[kEvLbt];
                kpre = ent[kEvKpre];
                const float4 *e4 = (const float4 *)ent;
#pragma unroll
                for (int x = 0; x < W / 4; ++x) {
                    const float4 v = e4[x];
                    arr[4 * x] = v.x;
                    arr[4 * x + 1] = v.y;
                    arr[4 * x + 2] = v.z;
                    arr[4 * x + 3] = v.w;
                }
                arr[W] = ent[W];
            } else {
#pragma unroll
                for (int x = 0; x <= W; ++x) arr[x] = INFINITY;
                arr[R] = 0.0f;
            }
            Tp = a.T + start;
            tcur = Tp[j0];
            thr = threshold_of(load_bsf(key));
            kpend = load_key_dist_bits(key);
            jl = j0;
            jdead = m;
            D = INFINITY;
            alive = valid;
            live = valid;
        };
        if (row < nslots) take(row);
        int next = nslots < 4 ? nslots : 4;
        for (;;) {
            // 16 columns; each lane's column jl (the same across its row)
#pragma unroll 1
            for (int u = 0; u < 16; ++u) {
                const int jn = jl + 1 < m ? jl + 1 : m - 1;
                const float tnext = Tp[jn];
                float qnext[NC];
                const float *qj = qb + jn;
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) qnext[cc] = qj[16 * cc];
                qnext[0] = inlo ? qnext[0] : kSentinel;
                qnext[NC - 1] = inhi ? qnext[NC - 1] : kSentinel;
                const float c = fmaf(tcur - mu, s, o);
                column<NC>(arr, qcur, c);
                {
                    const float unext = Unp[jn], lnext = Lnp[jn];
                    const float e = fmaxf(c - ucur, 0.0f) + fmaxf(lcur - c, 0.0f);
                    kpre = fmaf(e, e, kpre);
                    ucur = unext;
                    lcur = lnext;
                }
                if (jl == m - 1) D = arr[R];
                tcur = tnext;
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) qcur[cc] = qnext[cc];
                ++jl;
            }
            ++n_steps;
            // the test: every path crosses column jl - 1, so its minimum bounds the distance
            float mn = arr[0];
#pragma unroll
            for (int x = 1; x < W; ++x) mn = fminf(mn, arr[x]);
            mn += fmaxf(lbt - kpre, 0.0f);
            thr = fminf(thr, threshold_of(__uint_as_float(kpend)));
            kpend = load_key_dist_bits(key);
            if (alive && jl < m && mn > thr) {
                alive = false;
                jdead = jl;
            }
            if (live && (!alive || jl >= m)) {
                // the candidate ended: abandoned, or complete with distance D
                live = false;
                ++n_started;
                if (jdead < m) ++n_aband;
                n_cells += band_cells(m, r, jdead) - band_cells(m, r, j0);
                if (alive && D <= thr) {
                    const uint32_t start = (uint32_t)(Tp - a.T);
                    atomicMin((unsigned long long *)key, (unsigned long long)pack_key(D, start));
                    const uint32_t pos = atomicAdd(a.nb_count, 1u);
                    if (pos < a.nb_cap) {
                        a.nb_d[pos] = D;
                        a.nb_idx[pos] = start;
                        a.nb_q[pos] = q;
                    }
                }
            }
            if (a.ev_live > 0) {
                // a row with 1..ev_live live candidates and two tests or more to go moves them out;
                // one atomic per wave reserves the entries in this XCD's part of the buffer, and
                // lanes whose entry would fall beyond it keep their candidate
                const uint32_t rl = (uint32_t)((__ballot(live) >> (16 * row)) & 0xFFFFull);
                const int nl = __popc(rl);
                const bool want = live && nl <= a.ev_live && jl + 32 <= m;
                const uint64_t evl = __ballot(want);
                if (evl) {
                    const int x = (int)(blockIdx.x & 7u);
                    const int64_t part = a.ev_cap / 8;
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(a.ev_out_count + x * kCntStride, (uint32_t)__popcll(evl));
                    base = __shfl(base, 0, 64);
                    const uint32_t idx = base + (uint32_t)__popcll(evl & lanemask_lt());
                    if (want && (int64_t)idx < part) {
                        float *ent = a.ev_out + ((int64_t)x * part + idx) * kEvStride;
                        float4 *e4 = (float4 *)ent;
#pragma unroll
                        for (int y = 0; y < W / 4; ++y)
                            e4[y] = make_float4(arr[4 * y], arr[4 * y + 1], arr[4 * y + 2], arr[4 * y + 3]);
                        ent[W] = arr[W];
                        ent[kEvKpre] = kpre;
                        ent[kEvLbt] = lbt;
                        ent[kEvStart] = __int_as_float((int32_t)(uint32_t)(Tp - a.T));
                        ent[kEvQ] = __int_as_float(q);
                        ent[kEvCol] = __int_as_float(jl);
                        a.ev_out_key[(int64_t)x * part + idx] = (uint32_t)(q * a.ev_levels + jl / 16);
                        n_cells += band_cells(m, r, jl) - band_cells(m, r, j0);
                        ++n_evicted;
                        live = false;
                    }
                }
            }
            // rows with no live lane take the chunk's next row slots, in row order
            const uint64_t lm = __ballot(live);
            uint32_t done = 0;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                if (((lm >> (16 * rr)) & 0xFFFFull) == 0) done |= 1u << rr;
            if (done && next < nslots) {
                const int slot = next + __popc(done & ((1u << row) - 1u));
                if (((done >> row) & 1u) && slot < nslots) take(slot);
                next += __popc(done);
            }
            if (__ballot(live) == 0) break;
        }
    }
    if (a.counters) {
        n_started = wave_add(n_started);
        n_aband = wave_add(n_aband);
        n_cells = wave_add(n_cells);
        n_evicted = wave_add(n_evicted);
        if (lane == 0) {
            atomicAdd(&a.counters[4], n_started);
            atomicAdd(&a.counters[5], n_aband);
            atomicAdd(&a.counters[6], n_cells);
            atomicAdd(&a.counters[8], n_steps * 16ull * W * 64ull);
            if (n_evicted) atomicAdd(&a.counters[11], n_evicted);
        }
    }
}

// Bucketing of the evicted entries by (query, column level): counts, then a plan that gives every
// key a run of whole rows (padding lanes ~0u), then the scatter of entry indices into the runs.

template <bool SCATTER>
__global__ void k_ev_bucket(BatchArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * blockDim.x;
    const int64_t part = a.ev_cap / 8;
    for (int x = 0; x < 8; ++x) {
        uint32_t cnt = a.ev_in_count[x * kCntStride];
        if ((int64_t)cnt > part) cnt = (uint32_t)part;
        for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < cnt; base += stride) {
            const uint32_t e = (uint32_t)(x * part) + base + lane;
            const bool valid = base + lane < cnt;
            const int k = valid ? (int)a.ev_in_key[e] : -1;
            // one atomic per distinct key among the wave's 64 entries
            uint64_t pending = __ballot(valid);
            uint32_t pos = 0;
            while (pending) {
                const int leader = __ffsll((unsigned long long)pending) - 1;
                const int k0 = __shfl(k, leader, 64);
                const uint64_t peers = __ballot(valid && k == k0);
                uint32_t b0 = 0;
                if (lane == leader) b0 = atomicAdd(SCATTER ? &a.ev_kfill[k0] : &a.ev_kcnt[k0], (uint32_t)__popcll(peers));
                b0 = __shfl(b0, leader, 64);
                if (valid && k == k0) pos = b0 + (uint32_t)__popcll(peers & lanemask_lt());
                pending &= ~peers;
            }
            if (SCATTER && valid) a.ev_order[a.ev_koff[k] + pos] = e;
        }
    }
}

// One workgroup of 1024: exclusive scan of the keys' counts rounded up to 16.
__global__ __launch_bounds__(1024) void k_ev_plan(BatchArgs a) {
    __shared__ uint32_t part[1024];
    const int nkeys = a.nq * a.ev_levels;
    const int t = threadIdx.x;
    const int per = (nkeys + 1023) / 1024;
    const int k0 = t * per, k1 = k0 + per < nkeys ? k0 + per : nkeys;
    uint32_t sum = 0;
    for (int k = k0; k < k1; ++k) sum += (a.ev_kcnt[k] + 15u) & ~15u;
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t off = part[t] - sum;
    for (int k = k0; k < k1; ++k) {
        const uint32_t c = a.ev_kcnt[k], c16 = (c + 15u) & ~15u;
        a.ev_koff[k] = off;
        a.ev_kfill[k] = 0;
        for (uint32_t x = c; x < c16; ++x) a.ev_order[off + x] = ~0u;
        off += c16;
    }
    if (t == 1023) *a.ev_rows = part[1023] / 16u;
}

// Wide bands (r > 8 * kMaxChunks - 1): one lane per candidate, DP rows in global scratch.
template <bool PREFIX>
__global__ __launch_bounds__(64) void k_dtw_batch_wide(BatchArgs a) {
    constexpr int c = kMaxChunks + 1;
    if (*a.overflow || *a.surv_count <= a.diag_max) return;
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wave = g >> 6, nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t wlo = a.bucket_w[2 * c], whi = a.bucket_w[2 * c + 1];
    unsigned long long n_started = 0, n_aband = 0, n_cells = 0;
    for (int64_t w = wlo + wave; w < whi; w += nwaves) {
        int32_t wq0;
        const int q = wave_query(a, c, w, wq0);
        const BatchQ bq = a.bq[q];
        const int m = bq.m, r = bq.r;
        const int64_t local = (w - wq0) * 64 + lane;
        if (local >= (int64_t)a.qcnt[q * kCntStride]) continue;
        const int64_t start = a.sorted[w * 64 + lane];
        float mu, s, o;
        if (PREFIX) {
            StatsPrefix{a.T, a.pre, m, 1.0 / m}(start, mu, s, o);
        } else {
            const int64_t so = bq.stat_slot * a.slot_stride;
            StatsArr{a.mu + so, a.s + so, a.o + so}(start, mu, s, o);
        }
        const float *qh = a.qpad + q * a.qstride + kQPad;
        float *prev = a.wide_rows + g * 2 * (int64_t)(a.max_m + 1), *cur = prev + (a.max_m + 1);
        const float *Tp = a.T + start;
        float thr = threshold_of(load_bsf(a.keys + q));
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
                const float cc = fmaf(Tp[jj - 1] - mu, s, o);
                const float diff = qi - cc;
                const float v = fmaf(diff, diff, fminf(fminf(prev[jj], cur[jj - 1]), prev[jj - 1]));
                cur[jj] = v;
                rowmin = fminf(rowmin, v);
            }
            float *t = prev;
            prev = cur;
            cur = t;
            if ((i & 15) == 0) thr = threshold_of(load_bsf(a.keys + q));
            if (rowmin > thr) {
                alive = false;
                idead = i;
                break;
            }
        }
        const float D = prev[m];
        ++n_started;
        if (!alive) ++n_aband;
        n_cells += band_cells(m, r, alive ? m : idead);
        if (alive && D <= thr) {
            atomicMin((unsigned long long *)(a.keys + q), (unsigned long long)pack_key(D, (uint32_t)start));
            const uint32_t pos = atomicAdd(a.nb_count, 1u);
            if (pos < a.nb_cap) {
                a.nb_d[pos] = D;
                a.nb_idx[pos] = (uint32_t)start;
                a.nb_q[pos] = q;
            }
        }
    }
    if (a.counters) {
        atomicAdd(&a.counters[4], n_started);
        atomicAdd(&a.counters[5], n_aband);
        atomicAdd(&a.counters[6], n_cells);
        atomicAdd(&a.counters[8], n_cells);
    }
}

// ------------------------------------------------------------------ batched certification
__global__ __launch_bounds__(256) void k_cert_select_batch(BatchArgs a) {
    const uint32_t total = *a.nb_count;
    const uint32_t cnt = total < a.nb_cap ? total : a.nb_cap;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
        const int q = a.nb_q[e];
        if (a.nb_d[e] <= threshold_of(load_bsf(a.keys + q))) {
            const uint32_t pos = atomicAdd(a.cert_count, 1u);
            if (pos < a.nb_cap) {
                a.cert_idx[pos] = a.nb_idx[e];
                a.cert_q[pos] = q;
            }
        }
    }
}

__device__ inline double block_sum_d(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

// One block per qualifying candidate: FP64 DTW along anti-diagonals (cells of one anti-diagonal
// are independent), three anti-diagonals in an LDS ring of row-indexed buffers of length r + 4.
__global__ __launch_bounds__(256) void k_cert_dtw_batch(BatchArgs a) {
    extern __shared__ double sm[];
    __shared__ double red[4];
    const uint32_t cnt0 = *a.cert_count;
    const uint32_t cnt = cnt0 < a.nb_cap ? cnt0 : a.nb_cap;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        const int q = a.cert_q[e];
        const BatchQ bq = a.bq[q];
        const int m = bq.m, r = bq.r, L = r + 4;
        double *qh = sm, *ch = sm + m, *ring = sm + 2 * m;
        const double *qsrc = a.qhat64 + (int64_t)q * a.max_m;
        for (int j = tid; j < m; j += nt) qh[j] = qsrc[j];
        const float *wv = a.T + a.cert_idx[e];
        double s = 0.0;
        for (int j = tid; j < m; j += nt) s += (double)wv[j];
        const double mu = block_sum_d(s, red) / m;
        double v = 0.0;
        for (int j = tid; j < m; j += nt) {
            const double dd = (double)wv[j] - mu;
            v += dd * dd;
        }
        const double sigma = sqrt(block_sum_d(v, red) / m);
        const bool flat = sigma <= kSigmaFlat;
        for (int j = tid; j < m; j += nt) ch[j] = flat ? 0.0 : ((double)wv[j] - mu) / sigma;
        __syncthreads();
        for (int d = 0; d <= 2 * (m - 1); ++d) {
            int lo = (d - r + 1) >> 1;
            if (d - r < 0) lo = -((r - d) >> 1);
            if (lo < d - (m - 1)) lo = d - (m - 1);
            if (lo < 0) lo = 0;
            int hi = (d + r) >> 1;
            if (hi > d) hi = d;
            if (hi > m - 1) hi = m - 1;
            double *cur = ring + (d % 3) * L, *p1 = ring + ((d + 2) % 3) * L, *p2 = ring + ((d + 1) % 3) * L;
            for (int i = lo + tid; i <= hi; i += nt) {
                const int j = d - i;
                const double diff = qh[i] - ch[j];
                double best;
                if (d == 0) {
                    best = 0.0;
                } else {
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
        if (tid == 0) a.cert_d[e] = ring[((2 * (m - 1)) % 3) * L + (m - 1) % L];
        __syncthreads();
    }
}

// One block per query: minimum certified distance, lowest index on ties.
__global__ __launch_bounds__(256) void k_cert_reduce_batch(BatchArgs a) {
    __shared__ double sd[4];
    __shared__ uint32_t si[4];
    const int q = blockIdx.x;
    const uint32_t cnt0 = *a.cert_count;
    const uint32_t cnt = cnt0 < a.nb_cap ? cnt0 : a.nb_cap;
    double best = INFINITY;
    uint32_t bidx = 0xffffffffu;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        if (a.cert_q[e] != q) continue;
        const double d = a.cert_d[e];
        const uint32_t idx = a.cert_idx[e];
        if (d < best || (d == best && idx < bidx)) {
            best = d;
            bidx = idx;
        }
    }
    // (distance, index) minimum over the wave, then over the block's waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double od = __shfl_xor(best, off, 64);
        const uint32_t oi = __shfl_xor(bidx, off, 64);
        if (od < best || (od == best && oi < bidx)) {
            best = od;
            bidx = oi;
        }
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sd[wid] = best;
        si[wid] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < (int)(blockDim.x >> 6); ++t)
            if (sd[t] < best || (sd[t] == best && si[t] < bidx)) {
                best = sd[t];
                bidx = si[t];
            }
        a.res_idx[q] = bidx == 0xffffffffu ? -1 : (int64_t)bidx;
        a.res_dist[q] = best;
        const bool overflow = *a.overflow || *a.nb_count > a.nb_cap ||
                              *a.cert_count > a.nb_cap;
        a.res_status[q] = overflow ? DTWS_EOVERFLOW : (bidx == 0xffffffffu ? DTWS_EHIP : DTWS_OK);
        if (a.counters && q == 0) atomicAdd(&a.counters[7], (unsigned long long)cnt);
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_prefix(const float *T, int64_t n, double2 *PP, double *anc, double2 *tot, hipStream_t s,
                         const Decimated *dec, uint32_t levels) {
    const Decimated d = dec ? *dec : Decimated{};
    if (!dec) levels = 0;
    const int64_t blocks = (n + kPB - 1) / kPB;
    hipLaunchKernelGGL(k_prefix, dim3((unsigned)blocks), dim3(kPrefixThreads), 0, s, T, n, PP, anc, tot, d, levels);
    return hipGetLastError();
}

hipError_t launch_make_perm(const BatchArgs &a, int mode, uint64_t seed, int64_t max_nblocks, hipStream_t s) {
    int64_t bx = (max_nblocks + 255) / 256;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_make_perm, dim3((unsigned)bx, (unsigned)a.nq), dim3(256), 0, s, a, mode, seed);
    return hipGetLastError();
}

hipError_t launch_perm_rank(const BatchArgs &a, int64_t max_nblocks, hipStream_t s) {
    int64_t bx = (max_nblocks + 255) / 256;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_perm_rank, dim3((unsigned)bx, (unsigned)a.nq), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seed_random(const BatchArgs &a, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_seed_random, dim3(1), dim3(256), 0, s, a, seed);
    return hipGetLastError();
}

hipError_t launch_lb_batch(const BatchArgs &a, bool prefix, int round, int rank_lo, int rank_hi, int parts,
                           bool natural, int skip_below, int blocks, hipStream_t s) {
    const bool env = a.envU != nullptr;
    // the XCD sub-queues pay when every wave gets many items (their ends cost a few failed pops)
    const int64_t items = (int64_t)a.nq * (rank_hi - rank_lo) * parts;
    const int mode = natural ? (items >= 64 * 4 * (int64_t)blocks ? 3 : 1) : 0;
    if (prefix && env)
        hipLaunchKernelGGL((k_lb_batch<true, true>), dim3(blocks), dim3(256), 0, s, a, round, rank_lo, rank_hi, parts,
                           mode, skip_below);
    else if (prefix)
        hipLaunchKernelGGL((k_lb_batch<true, false>), dim3(blocks), dim3(256), 0, s, a, round, rank_lo, rank_hi, parts,
                           mode, skip_below);
    else if (env)
        hipLaunchKernelGGL((k_lb_batch<false, true>), dim3(blocks), dim3(256), 0, s, a, round, rank_lo, rank_hi, parts,
                           mode, skip_below);
    else
        hipLaunchKernelGGL((k_lb_batch<false, false>), dim3(blocks), dim3(256), 0, s, a, round, rank_lo, rank_hi, parts,
                           mode, skip_below);
    return hipGetLastError();
}

hipError_t launch_segments(const BatchArgs &a, int num_cu, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_seg_scatter, dim3(num_cu * 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <bool PREFIX>
static hipError_t launch_dtw_bucket_t(const BatchArgs &a, int nc, int blocks, hipStream_t s) {
    const dim3 g(blocks), b(256);
    switch (nc) {
#define DTWS_BCASE(N) \
    case N:                                                                                                    \
        if (N >= 4 && a.rows)                                                                                  \
            hipLaunchKernelGGL((k_dtw_batch_rows<(N >= 4 ? N : 4), PREFIX, false>), g, b, 0, s, a);            \
        else                                                                                                   \
            hipLaunchKernelGGL((k_dtw_batch<N, PREFIX>), g, b, N >= kBoundMinNC && a.Un ? kBoundLdsBytes : 0, s, a); \
        break;
        DTWS_BCASE(1) DTWS_BCASE(2) DTWS_BCASE(3) DTWS_BCASE(4) DTWS_BCASE(5) DTWS_BCASE(6) DTWS_BCASE(7)
        DTWS_BCASE(8) DTWS_BCASE(9) DTWS_BCASE(10) DTWS_BCASE(11) DTWS_BCASE(12) DTWS_BCASE(13) DTWS_BCASE(14)
#undef DTWS_BCASE
        case kMaxChunks + 1: {
            if (a.diag_wide) break;   // the one-wave-per-candidate kernel takes this bucket
            const int64_t wblocks = a.wide_lanes / 64;
            hipLaunchKernelGGL(k_dtw_batch_wide<PREFIX>, dim3((unsigned)wblocks), dim3(64), 0, s, a);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dtw_bucket(const BatchArgs &a, bool prefix, int nc, int blocks, hipStream_t s) {
    return prefix ? launch_dtw_bucket_t<true>(a, nc, blocks, s) : launch_dtw_bucket_t<false>(a, nc, blocks, s);
}

template <bool PREFIX>
static void launch_resume_t(const BatchArgs &a, int nc, int blocks, hipStream_t s) {
    const dim3 g(blocks), b(256);
    switch (nc) {
#define DTWS_RCASE(N) \
    case N: hipLaunchKernelGGL((k_dtw_batch_rows<N, PREFIX, true>), g, b, 0, s, a); break;
        DTWS_RCASE(4) DTWS_RCASE(5) DTWS_RCASE(6) DTWS_RCASE(7) DTWS_RCASE(8) DTWS_RCASE(9) DTWS_RCASE(10)
        DTWS_RCASE(11) DTWS_RCASE(12) DTWS_RCASE(13) DTWS_RCASE(14)
#undef DTWS_RCASE
        default: break;
    }
}

// Resumes the entries of a.ev_in (written by the previous launch for this bucket): buckets them by
// (query, column level) into rows, then runs the rows kernel on them, evicting into a.ev_out when
// a.ev_live > 0.
hipError_t launch_dtw_resume(const BatchArgs &a, bool prefix, int nc, int blocks, int num_cu, hipStream_t s) {
    if (nc < 4 || nc > kMaxChunks) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(a.ev_kcnt, 0, (int64_t)a.nq * a.ev_levels, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ev_bucket<false>, dim3(num_cu * 4), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ev_plan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_ev_bucket<true>, dim3(num_cu * 4), dim3(256), 0, s, a);
    if (a.ev_live > 0) {
        e = launch_fill_u32(a.ev_out_count, 0, 8 * kCntStride, s);
        if (e != hipSuccess) return e;
    }
    if (prefix) launch_resume_t<true>(a, nc, blocks, s);
    else launch_resume_t<false>(a, nc, blocks, s);
    return hipGetLastError();
}

hipError_t launch_cert_batch(const BatchArgs &a, int max_m, int max_r, hipStream_t s) {
    hipLaunchKernelGGL(k_cert_select_batch, dim3(16), dim3(256), 0, s, a);
    if (max_r <= kDiagMaxBand) {
        hipError_t e = launch_cert_diag(a, max_r, 256, s);
        if (e != hipSuccess) return e;
    } else {
        const size_t shm = sizeof(double) * (2 * (size_t)max_m + 3 * (size_t)(max_r + 4));
        hipLaunchKernelGGL(k_cert_dtw_batch, dim3(256), dim3(max_r < 64 ? 64 : 256), shm, s, a);
    }
    hipLaunchKernelGGL(k_cert_reduce_batch, dim3(a.nq), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dtws
