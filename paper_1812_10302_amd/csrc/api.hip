// C ABI of the dtws library: context management, argument checking and the stream-ordered
// search pipeline (query preparation -> window statistics -> data envelope -> best-so-far
// initialisation from one seeded random candidate -> chunks of {bound cascade, DTW of the
// survivors} with the best-so-far kept on the device -> FP64 certification).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "dtws_internal.h"

using namespace dtws;

namespace {

constexpr int kNumCounters = 16;
constexpr int64_t kMinBlock = 2048;   // smallest work-item block (sizes the order arrays)
constexpr int64_t kDefaultBlock = 4096;
constexpr int kDefaultDiagMax = 16384;  // rounds with at most this many survivors: one wave per candidate

// Decimation levels the proposals of a length-m query read (m a multiple of 64, step m/64 a power
// of two from 8 to 32; shorter steps take their grid from the series).
uint32_t dec_level_of(int m) {
    if (m % 64 != 0 || m < 512) return 0u;
    const int ps = m / 64;
    if ((ps & (ps - 1)) != 0 || ps > 32) return 0u;
    return 1u << __builtin_ctz((unsigned)ps);
}

// entries of all decimated levels for a series of max_n points
int64_t dec_total(int64_t max_n) {
    int64_t t = 0;
    for (int L = kDecFirst; L < kDecLevels; ++L) t += (max_n >> L) + 2;
    return t;
}

int diag_max_of(const dtws_ctx *c) { return c->diag_max >= 0 ? c->diag_max : kDefaultDiagMax; }

// capacity of the near-best list in effect (the schedule may lower it)
uint32_t nb_cap_of(const dtws_ctx *c) {
    return c->list_cap > 0 && c->list_cap < kNearBestCap ? (uint32_t)c->list_cap : (uint32_t)kNearBestCap;
}

void set_err(dtws_ctx *c, hipError_t e, const char *what) {
    if (!c) return;
    snprintf(c->lasterr, sizeof(c->lasterr), "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                         \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) {                   \
            set_err((ctx), e_, #expr);            \
            return DTWS_EHIP;                     \
        }                                         \
    } while (0)

// Launch wrapper: in profiling mode, brackets the launch with an event pair of class `cls`.
struct Prof {
    dtws_ctx *c;
    hipStream_t s;
    int slot = -1;
    Prof(dtws_ctx *c_, hipStream_t s_, int cls) : c(c_), s(s_) {
        if (c->profiling && c->ev_used < dtws_ctx::kMaxEvents) {
            slot = c->ev_used++;
            c->ev_class[slot] = cls;
            (void)hipEventRecord(c->ev[2 * slot], s);
        }
    }
    ~Prof() {
        if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], s);
    }
};
#define PROF(cls) Prof prof_guard_##__LINE__(c, s, (cls))

void prof_begin(dtws_ctx *c, uint32_t flags) {
    c->profiling = (flags & DTWS_PROFILE) != 0;
    c->ev_used = 0;
    for (int k = 0; k < DTWS_K_COUNT; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
}

// After the stream has been synchronised: sum the event pairs per class.
void prof_end(dtws_ctx *c) {
    if (!c->profiling) return;
    for (int e = 0; e < c->ev_used; ++e) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[2 * e], c->ev[2 * e + 1]) == hipSuccess) {
            c->prof_ms[c->ev_class[e]] += ms;
            c->prof_n[c->ev_class[e]] += 1;
        }
    }
    c->profiling = false;
}

template <class T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

QueryBufs query_bufs(dtws_ctx *c, int slot) {
    QueryBufs b;
    b.qpad = c->qpad + (int64_t)slot * c->qstride;
    b.qhat64 = c->qhat64 + (int64_t)slot * c->max_m;
    b.qsorted = c->qsorted + (int64_t)slot * c->mstride;
    b.Usorted = c->Usorted + (int64_t)slot * c->mstride;
    b.Lsorted = c->Lsorted + (int64_t)slot * c->mstride;
    b.Unat = c->Unat + (int64_t)slot * c->mstride;
    b.Lnat = c->Lnat + (int64_t)slot * c->mstride;
    b.order = c->order + (int64_t)slot * c->mstride;
    return b;
}

int check_series(dtws_ctx *c, const float *T, int64_t n, int32_t m) {
    if (!c || !T) return DTWS_EINVAL;
    if (m < 2 || m > c->max_m || n < m || n > c->max_n) return DTWS_EINVAL;
    return DTWS_OK;
}

// Kernel arguments of the plain pipeline for one query in result slot `slot`.
struct PlainArgs {
    LbArgs l;
    DtwArgs d;
    CertArgs ce;
};

PlainArgs plain_args(dtws_ctx *c, const float *T, int64_t n, int m, int r, int slot) {
    const QueryBufs b = query_bufs(c, slot);
    uint64_t *key = c->keys + slot;
    PlainArgs p{};
    DtwArgs &d = p.d;
    d.T = T;
    d.m = m;
    d.r = r;
    d.w = 2 * r + 1;
    d.qpad = b.qpad;
    d.n = n;
    d.single = -1;
    d.mu = c->st_mu;
    d.s = c->st_s;
    d.o = c->st_o;
    d.key = key;
    d.nb_d = c->nb_d;
    d.nb_idx = c->nb_idx;
    d.nb_count = c->nb_count;
    d.nb_cap = nb_cap_of(c);
    d.counters = c->counters;
    d.abandon_at = INFINITY;
    if (c->dtw_bound) {
        d.Un = b.Unat;
        d.Ln = b.Lnat;
    }
    // one wave per candidate for small rounds, and always for bands wider than the register kernel
    const bool diag = r <= kDiagMaxBand;
    d.diag_max = !diag ? 0u : (2 * r + 1 > 16 * kMaxChunks ? 0xFFFFFFFFu : (uint32_t)diag_max_of(c));

    LbArgs &l = p.l;
    l.T = T;
    l.m = m;
    l.qh = b.qpad + kQPad;
    l.qs = b.qsorted;
    l.Us = b.Usorted;
    l.Ls = b.Lsorted;
    l.order = b.order;
    l.mu = c->st_mu;
    l.s = c->st_s;
    l.o = c->st_o;
    l.envU = c->envU;
    l.envL = c->envL;
    l.key = key;
    l.surv = c->surv;
    l.surv_count = c->surv_count;
    l.counters = c->counters;

    CertArgs &ce = p.ce;
    ce.T = T;
    ce.m = m;
    ce.r = r;
    ce.qhat64 = b.qhat64;
    ce.key = key;
    ce.nb_d = c->nb_d;
    ce.nb_idx = c->nb_idx;
    ce.nb_count = c->nb_count;
    ce.nb_cap = d.nb_cap;
    ce.scratch = c->cert_rows;
    ce.cert_idx = c->cert_idx;
    ce.cert_count = c->cert_count;
    ce.cert_d = c->cert_d;
    ce.res_idx = c->res_idx + slot;
    ce.res_dist = c->res_dist + slot;
    ce.res_status = c->res_status + slot;
    ce.counters = c->counters;
    return p;
}

// Candidates [a0, a1) of the plain search: the bound cascade against the query's best-so-far, then
// DTW of its survivors (or DTW of every candidate without the bounds).
int plain_chunk(dtws_ctx *c, const PlainArgs &p, int64_t a0, int64_t a1, uint32_t flags, hipStream_t s) {
    if (flags & DTWS_NO_LOWER_BOUNDS) {
        DtwArgs dr = p.d;
        dr.range_first = a0;
        dr.count = a1 - a0;
        PROF(DTWS_K_DTW);
        HIPCHK(c, launch_dtw(dr, true, a1 - a0, c->num_cu, c->gen_rows, c->gen_lanes, s));
        return DTWS_OK;
    }
    { PROF(DTWS_K_OTHER); HIPCHK(c, launch_fill_u32(c->surv_count, 0, 1, s)); }
    LbArgs l = p.l;
    l.first = a0;
    l.last = a1;
    { PROF(DTWS_K_LB); HIPCHK(c, launch_lb(l, 1, c->num_cu, s)); }
    DtwArgs ds = p.d;
    ds.starts32 = c->surv;
    ds.count_dev = c->surv_count;
    ds.count = a1 - a0;
    // both schedules are enqueued; the device-side survivor count picks the one that runs
    { PROF(DTWS_K_DTW); HIPCHK(c, launch_dtw(ds, true, a1 - a0, c->num_cu, c->gen_rows, c->gen_lanes, s)); }
    if (ds.diag_max > 0) {
        PROF(DTWS_K_DTW_WAVE);
        HIPCHK(c, launch_dtw_diag_list(ds, true, c->num_cu * 4, s));
    }
    return DTWS_OK;
}

// The Prepare / Improve scheme of Section 3.3 (Algorithm 1) with the candidates visited in ascending
// order of their bound.  Prepare: every candidate's three bounds in full, independent of the
// best-so-far (eq. (lbMatrix)); a candidate survives the similarity map of eq. (bitmapMatrix) exactly
// when the largest of them lies within the threshold, so only that maximum is kept, fused with the
// start into a 64-bit key, and the keys are sorted.  Improve: segments of the sorted list, growing
// geometrically (64K, 1M, 16M, then the rest), each running DTW on its candidates whose bound is
// still within the best-so-far (the candidate matrix of eq. (candidateMatrix)); once a segment ends
// beyond the threshold every later one is empty.  The sort buffers (16 B per candidate of max_n and
// the sort's temporary storage) are allocated on the first call.
int lb_sorted_improve(dtws_ctx *c, const PlainArgs &p, int64_t N, hipStream_t s) {
    if (!c->lbs_keys) {
        size_t bytes = 0;
        HIPCHK(c, sort_keys_u64(nullptr, bytes, nullptr, nullptr, c->max_n, s));
        if (hipMalloc((void **)&c->lbs_keys, sizeof(uint64_t) * 2 * (size_t)c->max_n) != hipSuccess ||
            hipMalloc(&c->lbs_temp, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            if (c->lbs_keys) (void)hipFree(c->lbs_keys);
            c->lbs_keys = nullptr;
            c->lbs_temp = nullptr;
            return DTWS_ENOMEM;
        }
        c->lbs_temp_bytes = bytes;
    }
    uint64_t *keys = c->lbs_keys, *sorted = c->lbs_keys + c->max_n;
    {
        PROF(DTWS_K_LB);
        LbArgs l = p.l;
        l.first = 0;
        l.last = N;
        l.out_key = keys;
        HIPCHK(c, launch_lb(l, 0, c->num_cu, s));
        size_t bytes = c->lbs_temp_bytes;
        HIPCHK(c, sort_keys_u64(c->lbs_temp, bytes, keys, sorted, N, s));
    }
    int64_t size = 1 << 16;
    for (int64_t a0 = 0; a0 < N;) {
        const int64_t a1 = (N - a0 < size) ? N : a0 + size;
        { PROF(DTWS_K_LB); HIPCHK(c, launch_lb_sorted_segment(sorted, a0, a1, p.d.key, c->surv, c->surv_count, c->num_cu, s)); }
        DtwArgs ds = p.d;
        ds.starts32 = c->surv;
        ds.count_dev = c->surv_count;
        ds.count = a1 - a0;
        { PROF(DTWS_K_DTW); HIPCHK(c, launch_dtw(ds, true, a1 - a0, c->num_cu, c->gen_rows, c->gen_lanes, s)); }
        if (ds.diag_max > 0) {
            PROF(DTWS_K_DTW_WAVE);
            HIPCHK(c, launch_dtw_diag_list(ds, true, c->num_cu * 4, s));
        }
        a0 = a1;
        size *= 16;
    }
    return DTWS_OK;
}

// One query through the plain pipeline, results into the device result slot `slot`.
// Window statistics for m and the data envelope for r must already be in the context.
int run_query(dtws_ctx *c, const float *T, int64_t n, const float *Q, int m, int r, uint32_t flags, uint64_t seed,
              int slot, hipStream_t s) {
    const int64_t N = n - m + 1;
    const QueryBufs b = query_bufs(c, slot);
    const PlainArgs p = plain_args(c, T, n, m, r, slot);
    { PROF(DTWS_K_PREP); HIPCHK(c, launch_query_prep(Q, m, r, b, s)); }
    { PROF(DTWS_K_OTHER); HIPCHK(c, launch_fill_u64(p.d.key, kEmptyKey, 1, s)); }
    { PROF(DTWS_K_OTHER); HIPCHK(c, launch_fill_u32(c->nb_count, 0, 1, s)); }

    // best-so-far from one seeded random candidate (Algorithm 1, before the main loop)
    {
        DtwArgs d0 = p.d;
        d0.single = (int64_t)(splitmix64(seed) % (uint64_t)N);
        PROF(r <= kDiagMaxBand ? DTWS_K_DTW_WAVE : DTWS_K_DTW);
        if (r <= kDiagMaxBand) HIPCHK(c, launch_dtw_diag_list(d0, true, 1, s));
        else HIPCHK(c, launch_dtw(d0, true, 1, c->num_cu, c->gen_rows, c->gen_lanes, s));
    }

    if (flags & DTWS_LB_SORTED) {
        const int rc = lb_sorted_improve(c, p, N, s);
        if (rc != DTWS_OK) return rc;
    } else {
        // chunks grow geometrically so that the best-so-far tightens before the bulk of the series
        int64_t size = 1 << 16;
        for (int64_t a0 = 0; a0 < N;) {
            const int64_t a1 = (N - a0 < size) ? N : a0 + size;
            const int rc = plain_chunk(c, p, a0, a1, flags, s);
            if (rc != DTWS_OK) return rc;
            a0 = a1;
            size *= 16;   // 64K, 1M, then the rest: few launches once the best-so-far is tight
        }
    }
    { PROF(DTWS_K_CERT); HIPCHK(c, launch_certify(p.ce, s)); }
    return DTWS_OK;
}

// The near-best list of a plain search overflowed: more candidates lie within the FP32 slack of
// the final best-so-far than it holds (for example a flat query against a long flat stretch of the
// series, where every window of the stretch is an exact tie).  The key on the device is final, so
// the candidates the certification must see are exactly those with an FP32 distance within the
// slack of it.  The series is searched again in chunks of at most nb_cap candidates under that
// fixed key (a chunk cannot overflow the list), each chunk's near-best list is certified in FP64,
// and the chunk results are reduced in series order, lowest index on ties.  Blocking; the result
// replaces the slot's entry in the host staging arrays.
int recertify_chunked(dtws_ctx *c, const float *T, int64_t n, int m, int r, uint32_t flags, int slot,
                      hipStream_t s) {
    const int64_t N = n - m + 1;
    const PlainArgs p = plain_args(c, T, n, m, r, slot);
    const int64_t S = p.d.nb_cap;
    double best = INFINITY;
    int64_t bidx = -1;
    for (int64_t a0 = 0; a0 < N; a0 += S) {
        const int64_t a1 = N - a0 < S ? N : a0 + S;
        HIPCHK(c, launch_fill_u32(c->nb_count, 0, 1, s));
        const int rc = plain_chunk(c, p, a0, a1, flags, s);
        if (rc != DTWS_OK) return rc;
        HIPCHK(c, launch_certify(p.ce, s));
        int64_t idx = -1;
        double dist = 0.0;
        int32_t st = 0;
        HIPCHK(c, hipMemcpyAsync(&idx, c->res_idx + slot, sizeof(idx), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(&dist, c->res_dist + slot, sizeof(dist), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(&st, c->res_status + slot, sizeof(st), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (st == DTWS_EOVERFLOW) return DTWS_EOVERFLOW;   // cannot happen: a chunk holds <= nb_cap
        if (idx >= 0 && dist < best) {   // chunks in series order: strict < keeps the lowest index
            best = dist;
            bidx = idx;
        }
    }
    c->h_idx[slot] = bidx;
    c->h_dist[slot] = best;
    c->h_status[slot] = bidx >= 0 ? DTWS_OK : DTWS_EHIP;
    return DTWS_OK;
}

// Fills the context's counters of the last call from the host copy of the device counters.
void parse_counters(dtws_ctx *c, int64_t candidates) {
    const unsigned long long *h = c->h_counters;
    c->last.candidates = candidates;
    c->last.pruned_kim = (int64_t)h[1];
    c->last.pruned_keogh_q = (int64_t)h[2];
    c->last.pruned_keogh_d = (int64_t)h[3];
    c->last.dtw_started = (int64_t)h[4];
    c->last.dtw_abandoned = (int64_t)h[5];
    c->last.dtw_cells = (int64_t)h[6];
    c->last.certified = (int64_t)h[7];
    c->last.dtw_lane_cells = (int64_t)h[8];
    c->last.lb_terms = (int64_t)h[9];
    c->last.dtw_wave_cells = (int64_t)h[10];
    c->last.dtw_evicted = (int64_t)h[11];
    c->last.fallbacks = 0;
}

// Copies the result block (results and counters) to the host and parses the counters.
int fetch_counters(dtws_ctx *c, int64_t candidates, hipStream_t s) {
    HIPCHK(c, hipMemcpyAsync(c->h_res_block, c->res_block, c->res_bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    parse_counters(c, candidates);
    return DTWS_OK;
}

// Copies only the counters to the host and parses them (the result staging is left alone).
int fetch_counters_only(dtws_ctx *c, int64_t candidates, hipStream_t s) {
    HIPCHK(c, hipMemcpyAsync(c->h_counters, c->counters, sizeof(unsigned long long) * kNumCounters,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    parse_counters(c, candidates);
    return DTWS_OK;
}

// Batched pipeline (see batch.hip): all queries in rounds over a device work queue.
struct BatchPlan {
    bool same_m = true;     // per-window statistics slots (few distinct lengths) instead of the prefix
    int nm = 0, nr = 0;     // distinct lengths / bands held in slots (nr = 0: one envelope, largest band)
    int slot_m[8] = {0}, slot_r[8] = {0};
    int max_m = 0, max_r = 0;
    int64_t max_nb = 0, cand = 0, block = 0;
    int64_t score_rows = 0;   // proposals of the learned order (kScoreSamples per block)
    uint32_t dec_levels = 0;  // decimated prefix copies the proposals read
    bool bucket_used[kMaxChunks + 2] = {false};
    int ngroups = 0;          // distinct lengths (tiled cascade: queries grouped by length)
    int64_t max_N = 0;        // largest candidate count of a query
};

BatchPlan plan_batch(dtws_ctx *c, int64_t n, const int64_t *qoff, const int32_t *mh, const int32_t *rh, int nq,
                     bool learned) {
    BatchPlan p;
    // the learned order scores the blocks the model was trained on
    p.block = learned ? learned_block(c) : (c->block > 0 ? c->block : kDefaultBlock);
    for (int k = 0; k < nq; ++k) {
        BatchQ &b = c->h_bq[k];
        b.qoff = qoff[k];
        b.m = mh[k];
        b.r = rh[k] > mh[k] - 1 ? mh[k] - 1 : rh[k];
        b.N = n - b.m + 1;
        b.nblocks = (int32_t)((b.N + p.block - 1) / p.block);
        const int nc = (b.r + 8) / 8;
        b.nc = nc > kMaxChunks ? kMaxChunks + 1 : nc;
        p.bucket_used[b.nc] = true;
        p.max_m = b.m > p.max_m ? b.m : p.max_m;
        p.max_r = b.r > p.max_r ? b.r : p.max_r;
        p.max_nb = b.nblocks > p.max_nb ? b.nblocks : p.max_nb;
        p.cand += b.N;
        // rows of the learned order; the pinned copy is refreshed on every call because a graph
        // replay reads it
        c->h_row_off[k] = p.score_rows;
        p.score_rows += (int64_t)b.nblocks * kScoreSamples;
        p.dec_levels |= dec_level_of(b.m);
    }
    c->h_row_off[nq] = p.score_rows;
    // queries grouped by length for the tiled cascade: h_tile_q[0 .. ngroups] = first position of
    // each group in the list, the list (sorted by length, then index) from h_tile_q[max_q + 1]
    {
        int32_t *gfirst = c->h_tile_q, *qlist = c->h_tile_q + c->max_q + 1;
        for (int k = 0; k < nq; ++k) qlist[k] = k;
        std::stable_sort(qlist, qlist + nq, [&](int32_t x, int32_t y) { return c->h_bq[x].m < c->h_bq[y].m; });
        p.ngroups = 0;
        for (int k = 0; k < nq; ++k)
            if (k == 0 || c->h_bq[qlist[k]].m != c->h_bq[qlist[k - 1]].m) gfirst[p.ngroups++] = k;
        gfirst[p.ngroups] = nq;
        for (int k = 0; k < nq; ++k) p.max_N = c->h_bq[k].N > p.max_N ? c->h_bq[k].N : p.max_N;
    }
    // slots for distinct lengths and bands, in order of first appearance
    bool m_fit = true, r_fit = true;
    for (int k = 0; k < nq; ++k) {
        BatchQ &b = c->h_bq[k];
        int sm = -1, sr = -1;
        for (int t = 0; t < p.nm; ++t)
            if (p.slot_m[t] == b.m) sm = t;
        if (sm < 0 && m_fit) {
            if (p.nm < c->nslots) {
                p.slot_m[p.nm] = b.m;
                sm = p.nm++;
            } else {
                m_fit = false;
            }
        }
        for (int t = 0; t < p.nr; ++t)
            if (p.slot_r[t] == b.r) sr = t;
        if (sr < 0 && r_fit) {
            if (p.nr < c->nslots) {
                p.slot_r[p.nr] = b.r;
                sr = p.nr++;
            } else {
                r_fit = false;
            }
        }
        b.stat_slot = sm < 0 ? 0 : sm;
        b.env_slot = sr < 0 ? 0 : sr;
    }
    p.same_m = m_fit && !c->stats_prefix;
    if (!r_fit) {
        // too many distinct bands: one envelope for the largest band, valid (looser) for all
        p.nr = 1;
        p.slot_r[0] = p.max_r;
        for (int k = 0; k < nq; ++k) c->h_bq[k].env_slot = 0;
    }
    return p;
}

// Enqueues the whole batched search on stream s without any host synchronisation, so the same
// sequence can be captured into a graph.  Results land in the pinned host staging buffers.
int enqueue_batch(dtws_ctx *c, const BatchPlan &p, const float *T, int64_t n, const float *Qp, int nq,
                  uint32_t flags, uint64_t seed, hipStream_t s) {
    const bool same_m = p.same_m;
    const int max_m = p.max_m, max_r = p.max_r;
    const int64_t B = p.block, max_nb = p.max_nb;
    BatchArgs a{};
    a.T = T;
    a.n = n;
    a.nq = nq;
    a.block = B;
    a.max_m = c->max_m;
    a.bq = c->bq;
    a.qpad = c->qpad;
    a.qstride = c->qstride;
    a.qhat64 = c->qhat64;
    a.order = c->order;
    a.Us = c->Usorted;
    a.Ls = c->Lsorted;
    a.Un = c->dtw_bound ? c->Unat : nullptr;
    a.rows = c->dtw_rows;
    a.Ln = c->dtw_bound ? c->Lnat : nullptr;
    a.qs = c->qsorted;
    a.mstride = c->mstride;
    a.keys = c->keys;
    if (same_m) {
        a.mu = c->st_mu;
        a.s = c->st_s;
        a.o = c->st_o;
    } else {
        a.pre = Prefix{c->PP, c->anc, c->tot, T};
    }
    a.envU = c->data_envelope ? c->envU : nullptr;
    a.envL = c->data_envelope ? c->envL : nullptr;
    a.slot_stride = c->max_n;
    a.perm = c->perm;
    a.rank = c->rank;
    a.maxblocks = c->maxblocks;
    a.heads = c->heads;
    a.surv_q = c->surv_q;
    a.surv_i = c->surv_i;
    a.surv_lb = c->surv_lb;
    a.sorted_lb = c->sorted_lb;
    a.surv_count = c->surv_count;
    a.qcnt = c->qcnt;
    a.overflow = c->overflow;
    a.surv_cap = c->list_cap > 0 && c->list_cap < c->bsurv_cap ? c->list_cap : c->bsurv_cap;
    a.nb_cap = nb_cap_of(c);
    a.sorted = c->sorted;
    a.qorder = c->qorder;
    a.wstart = c->wstart;
    a.seg_off = c->seg_off;
    a.fill = c->fill;
    a.bucket_w = c->bucket_w;
    a.bucket_j = c->bucket_j;
    a.nb_d = c->nb_d;
    a.nb_idx = c->nb_idx;
    a.nb_q = c->nb_q;
    a.nb_count = c->nb_count;
    a.cert_idx = c->cert_idx;
    a.cert_q = c->cert_q;
    a.cert_count = c->cert_count;
    a.cert_d = c->cert_d;
    a.res_idx = c->res_idx;
    a.res_dist = c->res_dist;
    a.res_status = c->res_status;
    a.counters = c->counters;
    a.wide_rows = c->gen_rows;
    a.wide_lanes = c->gen_lanes;
    a.ev_live = c->dtw_rows ? c->dtw_evict : 0;
    a.ev_out = c->ev_buf[0];
    a.ev_out_key = c->ev_keybuf[0];
    a.ev_in_key = nullptr;
    a.ev_out_count = c->ev_count;
    a.ev_in = nullptr;
    a.ev_in_count = nullptr;
    a.ev_cap = c->ev_cap;
    a.ev_order = c->ev_order;
    a.ev_rows = c->ev_count + 16 * kCntStride;
    a.ev_levels = c->ev_levels;
    a.ev_kcnt = c->ev_keys;
    a.ev_koff = c->ev_keys + (int64_t)c->max_q * c->ev_levels;
    a.ev_kfill = c->ev_keys + 2 * (int64_t)c->max_q * c->ev_levels;
    a.diag_max = p.max_r <= kDiagMaxBand ? (uint32_t)diag_max_of(c) : 0u;
    a.diag_wide = p.max_r <= kDiagMaxBand;

    QueryBufs base{};
    base.qpad = c->qpad;
    base.qhat64 = c->qhat64;
    base.qsorted = c->qsorted;
    base.Usorted = c->Usorted;
    base.Lsorted = c->Lsorted;
    base.Unat = c->Unat;
    base.Lnat = c->Lnat;
    base.order = c->order;

    // the learned order and its PAA control score the same proposals; only the scorer differs
    const bool paa_only = (flags & DTWS_ORDER_MASK) == DTWS_ORDER_PAA;
    const bool learned = (flags & DTWS_ORDER_MASK) == DTWS_ORDER_LEARNED || paa_only;
    HIPCHK(c, hipMemcpyAsync(c->bq, c->h_bq, sizeof(BatchQ) * nq, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->tile_q, c->h_tile_q, sizeof(int32_t) * (c->max_q + 1 + nq), hipMemcpyHostToDevice, s));
    {
        PROF(DTWS_K_OTHER);
        HIPCHK(c, launch_reset_batch(c->keys, nq, c->counters, kNumCounters, c->heads, 64, c->nb_count, c->cert_count,
                                     c->overflow, s));
    }
    {
        PROF(DTWS_K_PREP);
        HIPCHK(c, launch_query_prep_batch(Qp, c->bq, nq, base, c->qstride, c->mstride, c->max_m, s));
    }
    if (same_m) {
        for (int t = 0; t < p.nm; ++t) {
            PROF(DTWS_K_STATS);
            const int64_t so = (int64_t)t * c->max_n;
            HIPCHK(c, launch_znorm_stats(T, n, p.slot_m[t], nullptr, nullptr, c->st_mu + so, c->st_s + so,
                                         c->st_o + so, s));
        }
    } else {
        PROF(DTWS_K_STATS);
        HIPCHK(c, launch_prefix(T, n, c->PP, c->anc, c->tot, s, &c->dec, learned ? p.dec_levels : 0u));
    }
    for (int t = 0; t < p.nr && c->data_envelope; ++t) {
        PROF(DTWS_K_ENV);
        const int64_t so = (int64_t)t * c->max_n;
        HIPCHK(c, launch_series_env(T, n, p.slot_r[t], c->envU + so, c->envL + so, s));
    }
    ScoreArgs sa{};
    if (learned) {
        // visiting order from the ordering network: blocks by ascending predicted distance of their
        // proposals (the blocked prefix gives every window's PAA)
        PROF(DTWS_K_SCORE);
        if (same_m) HIPCHK(c, launch_prefix(T, n, c->PP, c->anc, c->tot, s, &c->dec, p.dec_levels));
        sa.K = kScoreSamples;
        sa.qpaa = c->qpaa;
        sa.score = c->score;
        sa.sstart = c->sstart;
        sa.bstart = c->bstart;
        sa.row_off = c->row_off;
        sa.pre = Prefix{c->PP, c->anc, c->tot, T};
        sa.dec = c->dec;
        sa.dec_levels = p.dec_levels;
        sa.kinds = 0;
        for (int k = 0; k < nq; ++k) sa.kinds |= c->h_bq[k].m % 64 == 0 ? 1u : 2u;
        sa.total_rows = p.score_rows;
        HIPCHK(c, hipMemcpyAsync(c->row_off, c->h_row_off, sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, s));
        HIPCHK(c, mlp_order_blocks(c->mlp, a, sa, paa_only, s));
    } else {
        PROF(DTWS_K_OTHER);
        HIPCHK(c, launch_make_perm(a, (flags & DTWS_ORDER_MASK) == DTWS_ORDER_RANDOM ? 1 : 0, seed ^ 0xA5A5ull,
                                   max_nb, s));
    }
    if ((flags & DTWS_ORDER_MASK) != DTWS_ORDER_NATURAL && c->rounds > 1) {
        // the last round visits the rest of every query's blocks in series order (see below)
        PROF(DTWS_K_OTHER);
        HIPCHK(c, launch_perm_rank(a, max_nb, s));
    }
    const int dtw_blocks = c->num_cu * (c->dtw_blocks_per_cu > 0 ? c->dtw_blocks_per_cu : 4);
    const int lb_blocks = c->num_cu * (c->lb_blocks_per_cu > 0 ? c->lb_blocks_per_cu : 8);
    // known_count: the round's survivor count when the host knows it (-1 otherwise); a count the
    // one-wave-per-candidate kernel takes whole needs neither the segments nor the lane kernels
    auto dtw_round = [&](int64_t known_count) -> int {
        const bool diag_only = known_count >= 0 && known_count <= (int64_t)a.diag_max;
        if (!diag_only) {
            { PROF(DTWS_K_OTHER); HIPCHK(c, launch_segments(a, c->num_cu, s)); }
            for (int nc = 1; nc <= kMaxChunks + 1; ++nc) {
                if (!p.bucket_used[nc]) continue;
                PROF(DTWS_K_DTW);
                const bool evict = a.ev_live > 0 && nc >= 4 && nc <= kMaxChunks;
                if (evict) HIPCHK(c, launch_fill_u32(c->ev_count, 0, 8 * kCntStride, s));
                HIPCHK(c, launch_dtw_bucket(a, !same_m, nc, dtw_blocks, s));
                // evicted candidates resume in full rows; each resume launch but the last may evict
                // again, into the other buffer
                for (int d = 1; evict && d <= kEvDepth; ++d) {
                    BatchArgs ar = a;
                    ar.ev_in = c->ev_buf[(d - 1) & 1];
                    ar.ev_in_key = c->ev_keybuf[(d - 1) & 1];
                    ar.ev_out_key = c->ev_keybuf[d & 1];
                    ar.ev_in_count = c->ev_count + ((d - 1) & 1) * 8 * kCntStride;
                    ar.ev_out = c->ev_buf[d & 1];
                    ar.ev_out_count = c->ev_count + (d & 1) * 8 * kCntStride;
                    ar.ev_live = d < kEvDepth ? a.ev_live : 0;
                    HIPCHK(c, launch_dtw_resume(ar, !same_m, nc, dtw_blocks, c->num_cu, s));
                }
            }
        }
        if (a.diag_max > 0 || a.diag_wide) {
            PROF(DTWS_K_DTW_WAVE);
            HIPCHK(c, launch_dtw_diag(a, !same_m, p.max_r, c->num_cu * 4, s));
        }
        return DTWS_OK;
    };
    // round -1: the best-so-far starts from one random candidate per query (Algorithm 1), or from
    // the proposals of the best-scored blocks under the learned order
    {
        PROF(DTWS_K_OTHER);
        if (learned) HIPCHK(c, launch_seed_learned(a, sa, s));
        else HIPCHK(c, launch_seed_random(a, seed, s));
    }
    int rc = dtw_round(learned ? (int64_t)nq * kSeedCands : (int64_t)nq);
    if (rc != DTWS_OK) return rc;
    // rounds over the work queue (candidates per query, cumulative): 64K, 1M, 16M, then the rest;
    // with fewer rounds (schedule) 1M then the rest, or everything at once
    const int64_t k64 = int64_t(1) << 16, k1m = int64_t(1) << 20, k16m = int64_t(1) << 24, all = INT64_MAX / 2;
    const int nrounds = c->rounds == 1 ? 1 : (c->rounds == 2 ? 2 : 4);
    const int64_t t4[4] = {k64, k64 + k1m, k64 + k1m + k16m, all}, t2[2] = {k1m, all}, t1[1] = {all};
    const int64_t *targets = nrounds == 4 ? t4 : (nrounds == 2 ? t2 : t1);
    int64_t rank_lo = 0;
    for (int round = 0; round < nrounds && rank_lo < max_nb; ++round) {
        int64_t rank_hi = (targets[round] + B - 1) / B;
        if (rank_hi > max_nb) rank_hi = max_nb;
        {
            PROF(DTWS_K_OTHER);
            HIPCHK(c, launch_fill_u32(c->surv_count, 0, 1, s));
            HIPCHK(c, launch_fill_u32(c->qcnt, 0, (int64_t)nq * kCntStride, s));
        }
        {
            PROF(DTWS_K_LB);
            // small rounds: split each block so that many waves share them
            const int64_t size = (rank_hi - rank_lo) * B;
            int parts = size <= k64 ? 16 : (size <= 2 * k1m ? 4 : 1);
            while (parts > 1 && B / parts < 256) parts /= 2;
            // series order, block-major, whenever the round's blocks are the same for every query:
            // a round that holds them all, or any round of the series order.  The last round of
            // another order goes the same way over every block, each query skipping the blocks it
            // visited in the earlier rounds (ranks below rank_lo).
            const bool series = (flags & DTWS_ORDER_MASK) == DTWS_ORDER_NATURAL;
            const bool rest = !series && rank_lo > 0 && rank_hi >= max_nb;
            const bool natural = (rank_lo == 0 && rank_hi >= max_nb) || series || rest;
            const int skip_below = rest ? (int)rank_lo : 0;
            const int64_t item_lo = rest ? 0 : rank_lo;
            if (natural && c->lb_tile) {
                // every query visits the same candidates: series tiles shared by all queries
                TileArgs t{};
                t.gfirst = c->tile_q;
                t.qlist = c->tile_q + c->max_q + 1;
                t.ngroups = p.ngroups;
                t.c_lo = item_lo * B;
                t.c_hi = rank_hi * B;
                t.halo = max_m - 1;
                t.skip_below = skip_below;
                t.block = B;
                HIPCHK(c, launch_lb_tile(a, t, !same_m, p.max_N, s));
            } else {
                HIPCHK(c, launch_lb_batch(a, !same_m, round, (int)item_lo, (int)rank_hi, parts, natural, skip_below,
                                          lb_blocks, s));
            }
        }
        rc = dtw_round(-1);
        if (rc != DTWS_OK) return rc;
        rank_lo = rank_hi;
    }
    { PROF(DTWS_K_CERT); HIPCHK(c, launch_cert_batch(a, max_m, max_r, s)); }
    HIPCHK(c, hipMemcpyAsync(c->h_res_block, c->res_block, c->res_bytes, hipMemcpyDeviceToHost, s));
    return DTWS_OK;
}

int run_batch(dtws_ctx *c, const float *T, int64_t n, const float *Qp, const int64_t *qoff, const int32_t *mh,
              const int32_t *rh, int nq, uint32_t flags, uint64_t seed, hipStream_t s, dtws_match *out) {
    const BatchPlan p = plan_batch(c, n, qoff, mh, rh, nq, (flags & DTWS_ORDER_MASK) >= DTWS_ORDER_LEARNED);
    const size_t cert_shm = sizeof(double) * (2 * (size_t)p.max_m + 3 * (size_t)(p.max_r + 4));
    if ((flags & (DTWS_NO_LOWER_BOUNDS | DTWS_LB_SORTED)) || cert_shm > 60 * 1024) {
        // outside the batched pipeline's envelope: every query through the plain path
        dtws_counters sum{};
        int worst = DTWS_OK;
        for (int k = 0; k < nq; ++k) {
            const int rc = dtws_search(c, T, n, Qp + qoff[k], mh[k], rh[k], flags & ~(DTWS_ORDER_MASK | DTWS_NO_GRAPH),
                                       seed + k, s, &out[k]);
            if (rc != DTWS_OK && rc != DTWS_EOVERFLOW) return rc;
            if (rc != DTWS_OK) worst = rc;
            const int64_t *src = (const int64_t *)&c->last;
            int64_t *dst = (int64_t *)&sum;
            for (size_t f = 0; f < sizeof(dtws_counters) / sizeof(int64_t); ++f) dst[f] += src[f];
        }
        c->last = sum;
        return worst;
    }
    const bool use_graph = !(flags & (DTWS_PROFILE | DTWS_NO_GRAPH));
    if (!use_graph) {
        prof_begin(c, flags);
        int rc = enqueue_batch(c, p, T, n, Qp, nq, flags, seed, s);
        if (rc != DTWS_OK) return rc;
        HIPCHK(c, hipStreamSynchronize(s));
        prof_end(c);
    } else {
        // The graph is rebuilt when anything it bakes in changes: pointers, sizes, flags, seed, the
        // per-query parameters and the tuning knobs.
        std::vector<int64_t> sig = {(int64_t)(uintptr_t)T, n, (int64_t)(uintptr_t)Qp, nq, (int64_t)flags,
                                    (int64_t)seed, p.block, c->lb_blocks_per_cu, c->dtw_blocks_per_cu, c->diag_max,
                                    c->stats_prefix, c->data_envelope, c->rounds, c->lb_tile, c->list_cap,
                                    c->dtw_bound, c->dtw_rows, c->dtw_evict};
        for (int k = 0; k < nq; ++k) {
            sig.push_back(qoff[k]);
            sig.push_back(mh[k]);
            sig.push_back(rh[k]);
        }
        if (!c->graph_exec || sig != c->graph_sig) {
            if (c->graph_exec) {
                (void)hipGraphExecDestroy(c->graph_exec);
                c->graph_exec = nullptr;
            }
            c->profiling = false;
            HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue_batch(c, p, T, n, Qp, nq, flags, seed, c->gstream);
            hipGraph_t g = nullptr;
            const hipError_t ee = hipStreamEndCapture(c->gstream, &g);
            if (rc != DTWS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ee != hipSuccess) {
                set_err(c, ee, "hipStreamEndCapture");
                return DTWS_EHIP;
            }
            const hipError_t ie = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                c->graph_exec = nullptr;
                set_err(c, ie, "hipGraphInstantiate");
                return DTWS_EHIP;
            }
            c->graph_sig = sig;
        }
        // order the graph after the caller's stream, run it, wait for it
        HIPCHK(c, hipEventRecord(c->gevent, s));
        HIPCHK(c, hipStreamWaitEvent(c->gstream, c->gevent, 0));
        HIPCHK(c, hipGraphLaunch(c->graph_exec, c->gstream));
        HIPCHK(c, hipStreamSynchronize(c->gstream));
        c->graph_launches++;
    }
    parse_counters(c, p.cand);
    int worst = DTWS_OK;
    for (int k = 0; k < nq; ++k) {
        out[k].index = c->h_idx[k];
        out[k].distance = c->h_dist[k];
        out[k].status = c->h_status[k];
        out[k].reserved = 0;
    }
    for (int k = 0; k < nq; ++k) {
        if (out[k].status == DTWS_EOVERFLOW) {
            // survivor or near-best list overflowed: redo this query through the plain path (its
            // kernels add to the profile of the batch; the counters keep the batch's and count the
            // fallback in `fallbacks`)
            dtws_counters keep = c->last;
            double keep_ms[DTWS_K_COUNT];
            int64_t keep_n[DTWS_K_COUNT];
            for (int j = 0; j < DTWS_K_COUNT; ++j) {
                keep_ms[j] = c->prof_ms[j];
                keep_n[j] = c->prof_n[j];
            }
            const int r2 = dtws_search(c, T, n, Qp + qoff[k], mh[k], rh[k], flags & DTWS_PROFILE, seed + k, s,
                                       &out[k]);
            for (int j = 0; j < DTWS_K_COUNT; ++j) {
                c->prof_ms[j] += keep_ms[j];
                c->prof_n[j] += keep_n[j];
            }
            c->last = keep;
            c->last.fallbacks += 1;
            if (r2 != DTWS_OK) worst = r2;
        } else if (out[k].status != DTWS_OK) {
            worst = out[k].status;
        }
    }
    return worst;
}

}  // namespace

namespace dtws {

QueryBufs query_bufs_of(dtws_ctx *c, int slot) { return query_bufs(c, slot); }

void set_hip_error(dtws_ctx *c, hipError_t e, const char *what) { set_err(c, e, what); }

// Work-item block of the learned order: the block the model was trained with, else the schedule's.
int64_t learned_block(const dtws_ctx *c) {
    if (c->model_block > 0) return c->model_block;
    return c->block > 0 ? c->block : kDefaultBlock;
}

int64_t propose_rows(const dtws_ctx *c, int64_t n, int m) {
    const int64_t B = learned_block(c);
    const int64_t N = n - m + 1, nb = (N + B - 1) / B;
    return nb * kScoreSamples;
}

// Proposals of the normalised query in slot 0 (query preparation already enqueued) over T: starts
// and feature rows.  Uses the context's prefix and staging entries h_bq[0] / h_row_off[0..1]: the
// caller synchronises before those change.
int enqueue_propose(dtws_ctx *c, const float *T, int64_t n, int m, int64_t *starts, float *X, hipStream_t s) {
    const int64_t B = learned_block(c);
    const int64_t N = n - m + 1, nb = (N + B - 1) / B, rows = nb * kScoreSamples;
    HIPCHK(c, launch_prefix(T, n, c->PP, c->anc, c->tot, s, &c->dec, dec_level_of(m)));
    BatchQ &bq = c->h_bq[0];
    bq = BatchQ{};
    bq.m = m;
    bq.N = N;
    bq.nblocks = (int32_t)nb;
    c->h_row_off[0] = 0;
    c->h_row_off[1] = rows;
    HIPCHK(c, hipMemcpyAsync(c->bq, c->h_bq, sizeof(BatchQ), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->row_off, c->h_row_off, sizeof(int64_t) * 2, hipMemcpyHostToDevice, s));
    BatchArgs a{};
    a.T = T;
    a.n = n;
    a.nq = 1;
    a.block = B;
    a.max_m = c->max_m;
    a.bq = c->bq;
    a.qhat64 = c->qhat64;
    ScoreArgs sa{};
    sa.K = kScoreSamples;
    sa.total_rows = rows;
    sa.qpaa = c->qpaa;
    sa.sstart = c->sstart;
    sa.row_off = c->row_off;
    sa.pre = Prefix{c->PP, c->anc, c->tot, T};
    sa.dec = c->dec;
    sa.dec_levels = dec_level_of(m);
    sa.kinds = m % 64 == 0 ? 1u : 2u;
    HIPCHK(c, launch_propose(a, sa, X, starts, s));
    return DTWS_OK;
}

}  // namespace dtws

// ============================================================================ C ABI
extern "C" {

DTWS_API const char *dtws_strerror(int code) {
    switch (code) {
        case DTWS_OK: return "ok";
        case DTWS_EINVAL: return "invalid argument";
        case DTWS_ENOMEM: return "out of device memory";
        case DTWS_ENODEV: return "no HIP device";
        case DTWS_EHIP: return "HIP runtime error";
        case DTWS_EOVERFLOW: return "internal list overflow";
        case DTWS_ENOMODEL: return "no learned model loaded";
        default: return "unknown error";
    }
}

DTWS_API const char *dtws_last_error(dtws_ctx *ctx) { return ctx ? ctx->lasterr : ""; }

DTWS_API int dtws_device_count(void) {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess) return 0;
    return cnt < 0 ? 0 : cnt;
}

DTWS_API void dtws_destroy(dtws_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    void *dev[] = {c->qpad, c->qhat64, c->qsorted, c->Usorted, c->Lsorted, c->Unat, c->Lnat, c->order, c->keys, c->st_mu,
                   c->st_s, c->st_o, c->envU, c->envL, c->surv, c->surv_count, c->nb_d, c->nb_idx,
                   c->nb_count, c->cert_rows, c->cert_idx, c->cert_count, c->cert_d, c->res_block, c->gen_rows, c->bq, c->PP, c->PPd, c->anc, c->tot,
                   c->perm, c->rank, c->heads, c->surv_q, c->surv_i, c->surv_lb, c->sorted, c->sorted_lb, c->qcnt, c->fill, c->overflow,
                   c->ev_buf[0], c->ev_buf[1], c->ev_keybuf[0], c->ev_keybuf[1], c->ev_count, c->ev_order, c->ev_keys,
                   c->qorder, c->wstart, c->bucket_w, c->bucket_j, c->seg_off, c->nb_q, c->cert_q,
                   c->mlp.theta, c->mlp.grad, c->mlp.adam_m, c->mlp.adam_v, c->mlp.W1T, c->mlp.W2T, c->mlp.W2b,
                   c->mlp.Xb, c->mlp.XbT, c->mlp.H1b, c->mlp.H1T, c->mlp.dA2b, c->mlp.dA2T, c->mlp.dA1T,
                   c->mlp.C1, c->mlp.C2, c->mlp.y, c->mlp.dy, c->mlp.loss, c->mlp.Xf, c->mlp.part, c->qpaa,
                   c->score, c->sstart, c->bstart, c->row_off, c->tile_q, c->lbs_keys, c->lbs_temp};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->gevent) (void)hipEventDestroy(c->gevent);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->ev) {
        for (int e = 0; e < 2 * dtws_ctx::kMaxEvents; ++e)
            if (c->ev[e]) (void)hipEventDestroy(c->ev[e]);
        delete[] c->ev;
    }
    delete[] c->ev_class;
    void *host[] = {c->h_res_block, c->h_bq, c->h_row_off, c->h_tile_q};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    delete c;
}

DTWS_API int dtws_create(int device, int64_t max_n, int32_t max_m, int32_t max_queries, dtws_ctx **out) {
    if (!out) return DTWS_EINVAL;
    *out = nullptr;
    if (max_n < 2 || max_n >= (int64_t(1) << 31) || max_m < 2 || max_m > kMaxM || max_queries < 1 ||
        max_queries > 65536)
        return DTWS_EINVAL;
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0 || device < 0 || device >= cnt) return DTWS_ENODEV;
    if (hipSetDevice(device) != hipSuccess) return DTWS_ENODEV;
    dtws_ctx *c = new (std::nothrow) dtws_ctx;
    if (!c) return DTWS_ENOMEM;
    c->device = device;
    c->max_n = max_n;
    c->max_m = max_m;
    c->max_q = max_queries;
    if (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->num_cu <= 0)
        c->num_cu = 256;
    c->qstride = 2 * kQPad + max_m;
    c->surv_cap = max_n;                  // a chunk of any size can keep every survivor
    {
        // statistics (12 B) + envelope (8 B) slots of max_n points for distinct lengths / bands of
        // a batch, up to four, within about 24 GB
        const int64_t fit = (int64_t)(24e9 / (20.0 * (double)max_n));
        c->nslots = fit < 1 ? 1 : (fit > 4 ? 4 : (int)fit);
        if (c->nslots > max_queries) c->nslots = max_queries;
    }
    c->mstride = ((int64_t)max_m + 15) / 16 * 16;
    c->gen_lanes = 8192;
    const int64_t Q = max_queries;
    bool ok = dalloc(&c->qpad, Q * c->qstride) == hipSuccess && dalloc(&c->qhat64, Q * max_m) == hipSuccess &&
              dalloc(&c->qsorted, Q * c->mstride) == hipSuccess && dalloc(&c->Usorted, Q * c->mstride) == hipSuccess &&
              dalloc(&c->Lsorted, Q * c->mstride) == hipSuccess && dalloc(&c->order, Q * c->mstride) == hipSuccess &&
              dalloc(&c->Unat, Q * c->mstride) == hipSuccess && dalloc(&c->Lnat, Q * c->mstride) == hipSuccess &&
              dalloc(&c->keys, Q) == hipSuccess && dalloc(&c->st_mu, c->nslots * max_n) == hipSuccess &&
              dalloc(&c->st_s, c->nslots * max_n) == hipSuccess && dalloc(&c->st_o, c->nslots * max_n) == hipSuccess &&
              dalloc(&c->envU, c->nslots * max_n) == hipSuccess && dalloc(&c->envL, c->nslots * max_n) == hipSuccess &&
              dalloc(&c->surv, c->surv_cap) == hipSuccess && dalloc(&c->surv_count, 1) == hipSuccess &&
              dalloc(&c->nb_d, kNearBestCap) == hipSuccess && dalloc(&c->nb_idx, kNearBestCap) == hipSuccess &&
              dalloc(&c->nb_count, 1) == hipSuccess &&
              dalloc(&c->cert_rows, (size_t)256 * 3 * (max_m + 1)) == hipSuccess &&
              dalloc(&c->cert_idx, kNearBestCap) == hipSuccess && dalloc(&c->cert_count, 1) == hipSuccess &&
              dalloc(&c->cert_d, kNearBestCap) == hipSuccess &&
              dalloc(&c->gen_rows, (size_t)c->gen_lanes * 2 * (max_m + 1)) == hipSuccess;
    if (ok) {
        // results: index (Q x int64), distance (Q x double), status (Q x int32, padded to 8 B), counters
        const size_t st_bytes = (sizeof(int32_t) * (size_t)Q + 7) & ~(size_t)7;
        c->res_bytes = (sizeof(int64_t) + sizeof(double)) * (size_t)Q + st_bytes + sizeof(unsigned long long) * kNumCounters;
        ok = hipMalloc((void **)&c->res_block, c->res_bytes) == hipSuccess &&
             hipHostMalloc((void **)&c->h_res_block, c->res_bytes, 0) == hipSuccess;
        if (ok) {
            auto carve = [&](uint8_t *b, int64_t *&idx, double *&dist, int32_t *&st, unsigned long long *&cnt) {
                idx = (int64_t *)b;
                dist = (double *)(b + sizeof(int64_t) * (size_t)Q);
                st = (int32_t *)(b + (sizeof(int64_t) + sizeof(double)) * (size_t)Q);
                cnt = (unsigned long long *)(b + (sizeof(int64_t) + sizeof(double)) * (size_t)Q + st_bytes);
            };
            carve(c->res_block, c->res_idx, c->res_dist, c->res_status, c->counters);
            carve(c->h_res_block, c->h_idx, c->h_dist, c->h_status, c->h_counters);
        }
    }
    if (ok) {
        c->maxblocks = (max_n + kMinBlock - 1) / kMinBlock + 1;
        // batched survivor list (20 B per entry with the sorted copy and the bounds): up to 2^30
        // entries (21.5 GB) on a device of at least 128 GiB, else 2^28; a round that overflows it
        // is redone by the plain search, so this only decides how often that happens
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) total_b = 0;
        const int64_t lim = total_b >= (size_t(128) << 30) ? (int64_t(1) << 30) : (int64_t(1) << 28);
        int64_t cap = Q * max_n < lim ? Q * max_n : lim;
        if (cap < Q * kSeedCands) cap = Q * kSeedCands;   // round -1 of the learned order
        c->bsurv_cap = cap;
        const int64_t nblk = max_n / 4096 + 2;
        ok = dalloc(&c->bq, Q) == hipSuccess && hipHostMalloc((void **)&c->h_bq, sizeof(BatchQ) * Q, 0) == hipSuccess &&
             dalloc(&c->PP, max_n + 1) == hipSuccess && dalloc(&c->PPd, dec_total(max_n)) == hipSuccess &&
             dalloc(&c->anc, nblk) == hipSuccess &&
             dalloc(&c->tot, nblk) == hipSuccess && dalloc(&c->perm, Q * c->maxblocks) == hipSuccess &&
             dalloc(&c->rank, Q * c->maxblocks) == hipSuccess &&
             dalloc(&c->heads, 64) == hipSuccess && dalloc(&c->surv_q, cap) == hipSuccess &&
             dalloc(&c->surv_i, cap) == hipSuccess && dalloc(&c->sorted, cap + 64 * Q) == hipSuccess &&
             dalloc(&c->surv_lb, cap) == hipSuccess && dalloc(&c->sorted_lb, cap + 64 * Q) == hipSuccess &&
             dalloc(&c->qcnt, Q * kCntStride) == hipSuccess && dalloc(&c->fill, Q * kCntStride) == hipSuccess &&
             dalloc(&c->overflow, 1) == hipSuccess && dalloc(&c->qorder, Q + 1) == hipSuccess &&
             dalloc(&c->wstart, Q + 1) == hipSuccess && dalloc(&c->bucket_w, 2 * (kMaxChunks + 2)) == hipSuccess &&
             dalloc(&c->bucket_j, 2 * (kMaxChunks + 2)) == hipSuccess && dalloc(&c->seg_off, Q) == hipSuccess &&
             dalloc(&c->nb_q, kNearBestCap) == hipSuccess && dalloc(&c->cert_q, kNearBestCap) == hipSuccess &&
             dalloc(&c->tile_q, 2 * Q + 2) == hipSuccess &&
             hipHostMalloc((void **)&c->h_tile_q, sizeof(int32_t) * (2 * Q + 2), 0) == hipSuccess;
        // eviction entries of the rows DTW kernel (928 B each, two buffers, each in eight parts, one
        // per XCD): 2^25 on a device of at least 256 GiB (62 GB in all), 2^24 from 128 GiB, else 2^20;
        // a lane finding its part full keeps its candidate
        c->ev_cap = total_b >= (size_t(256) << 30)   ? (int64_t(1) << 25)
                    : total_b >= (size_t(128) << 30) ? (int64_t(1) << 24)
                                                     : (int64_t(1) << 20);
        if (c->ev_cap > cap) c->ev_cap = cap < 4096 ? 4096 : cap;
        c->ev_cap &= ~int64_t(7);
        c->ev_levels = (int)(max_m / 16 + 1);
        const int64_t nkeys = Q * c->ev_levels;
        ok = ok && dalloc(&c->ev_buf[0], c->ev_cap * kEvStride) == hipSuccess &&
             dalloc(&c->ev_buf[1], c->ev_cap * kEvStride) == hipSuccess && dalloc(&c->ev_count, 16 * kCntStride + 1) == hipSuccess &&
             dalloc(&c->ev_keybuf[0], c->ev_cap) == hipSuccess && dalloc(&c->ev_keybuf[1], c->ev_cap) == hipSuccess &&
             dalloc(&c->ev_order, c->ev_cap + 16 * nkeys) == hipSuccess && dalloc(&c->ev_keys, 3 * nkeys) == hipSuccess;
        if (ok) {
            int64_t off = 0;
            for (int L = kDecFirst; L < kDecLevels; ++L) {
                c->dec.lv[L] = c->PPd + off;
                off += (max_n >> L) + 2;
            }
        }
    }
    if (ok) {
        MlpBufs &b = c->mlp;
        b.num_cu = c->num_cu;
        const int64_t R = kMlpChunk;
        ok = dalloc(&b.theta, kModelParams) == hipSuccess && dalloc(&b.grad, kModelParams) == hipSuccess &&
             dalloc(&b.adam_m, kModelParams) == hipSuccess && dalloc(&b.adam_v, kModelParams) == hipSuccess &&
             dalloc(&b.W1T, 256 * 32) == hipSuccess && dalloc(&b.W2T, 256 * 256) == hipSuccess &&
             dalloc(&b.W2b, 256 * 256) == hipSuccess && dalloc(&b.Xb, R * 32) == hipSuccess &&
             dalloc(&b.XbT, R * 32) == hipSuccess && dalloc(&b.H1b, R * 256) == hipSuccess &&
             dalloc(&b.H1T, R * 256) == hipSuccess && dalloc(&b.dA2b, R * 256) == hipSuccess &&
             dalloc(&b.dA2T, R * 256) == hipSuccess && dalloc(&b.dA1T, R * 256) == hipSuccess &&
             dalloc(&b.C1, R * 256) == hipSuccess && dalloc(&b.C2, R * 256) == hipSuccess &&
             dalloc(&b.y, R) == hipSuccess && dalloc(&b.dy, R) == hipSuccess && dalloc(&b.loss, 1) == hipSuccess &&
             dalloc(&b.Xf, R * 32) == hipSuccess && dalloc(&b.part, (int64_t)kColsumGroups * 4 * 256) == hipSuccess &&
             dalloc(&c->qpaa, Q * 16) == hipSuccess && dalloc(&c->sstart, R) == hipSuccess &&
             dalloc(&c->score, Q * c->maxblocks) == hipSuccess && dalloc(&c->bstart, Q * c->maxblocks) == hipSuccess &&
             dalloc(&c->row_off, Q + 1) == hipSuccess &&
             hipHostMalloc((void **)&c->h_row_off, sizeof(int64_t) * (Q + 1), 0) == hipSuccess;
    }
    if (ok) {
        c->ev = new (std::nothrow) hipEvent_t[2 * dtws_ctx::kMaxEvents]();
        c->ev_class = new (std::nothrow) int[dtws_ctx::kMaxEvents]();
        ok = c->ev && c->ev_class;
        for (int e = 0; ok && e < 2 * dtws_ctx::kMaxEvents; ++e) ok = hipEventCreate(&c->ev[e]) == hipSuccess;
    }
    if (ok) ok = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&c->gevent, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dtws_destroy(c);
        return DTWS_ENOMEM;
    }
    *out = c;
    return DTWS_OK;
}

DTWS_API int dtws_get_profile(dtws_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return DTWS_EINVAL;
    for (int k = 0; k < DTWS_K_COUNT; ++k) {
        ms[k] = c->prof_ms[k];
        launches[k] = c->prof_n[k];
    }
    return DTWS_OK;
}

DTWS_API int dtws_get_counters(dtws_ctx *c, dtws_counters *out) {
    if (!c || !out) return DTWS_EINVAL;
    *out = c->last;
    return DTWS_OK;
}

DTWS_API int dtws_search(dtws_ctx *c, const float *T, int64_t n, const float *Q, int32_t m, int32_t r,
                         uint32_t flags, uint64_t seed, void *stream, dtws_match *out) {
    if (check_series(c, T, n, m) != DTWS_OK || !Q || !out || r < 0) return DTWS_EINVAL;
    if (flags & ~(DTWS_ORDER_MASK | DTWS_NO_LOWER_BOUNDS | DTWS_PROFILE | DTWS_NO_GRAPH | DTWS_LB_SORTED))
        return DTWS_EINVAL;
    if ((flags & DTWS_LB_SORTED) && (flags & DTWS_NO_LOWER_BOUNDS)) return DTWS_EINVAL;
    if ((flags & DTWS_ORDER_MASK) == DTWS_ORDER_LEARNED) return DTWS_ENOMODEL;
    if ((flags & DTWS_ORDER_MASK) == DTWS_ORDER_PAA) return DTWS_EINVAL;   // batched calls only
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (r > m - 1) r = m - 1;
    prof_begin(c, flags);
    { PROF(DTWS_K_OTHER); HIPCHK(c, launch_fill_u64((uint64_t *)c->counters, 0, kNumCounters, s)); }
    { PROF(DTWS_K_STATS); HIPCHK(c, launch_znorm_stats(T, n, m, nullptr, nullptr, c->st_mu, c->st_s, c->st_o, s)); }
    if (!(flags & DTWS_NO_LOWER_BOUNDS)) {
        PROF(DTWS_K_ENV);
        HIPCHK(c, launch_series_env(T, n, r, c->envU, c->envL, s));
    }
    int rc = run_query(c, T, n, Q, m, r, flags, seed, 0, s);
    if (rc != DTWS_OK) return rc;
    rc = fetch_counters(c, n - m + 1, s);
    if (rc != DTWS_OK) return rc;
    prof_end(c);
    if (c->h_status[0] == DTWS_EOVERFLOW) {
        rc = recertify_chunked(c, T, n, m, r, flags, 0, s);
        if (rc != DTWS_OK) return rc;
        rc = fetch_counters_only(c, n - m + 1, s);   // the counters include the second scan
        if (rc != DTWS_OK) return rc;
    }
    out->index = c->h_idx[0];
    out->distance = c->h_dist[0];
    out->status = c->h_status[0];
    out->reserved = 0;
    return out->status == DTWS_OK ? DTWS_OK : out->status;
}

DTWS_API int dtws_search_batch(dtws_ctx *c, const float *T, int64_t n, const float *Qp, const int64_t *qoff,
                               const int32_t *mh, const int32_t *rh, int32_t nq, uint32_t flags, uint64_t seed,
                               void *stream, dtws_match *out) {
    if (!c || !T || !Qp || !qoff || !mh || !rh || !out || nq < 1 || nq > c->max_q) return DTWS_EINVAL;
    if (flags & ~(DTWS_ORDER_MASK | DTWS_NO_LOWER_BOUNDS | DTWS_PROFILE | DTWS_NO_GRAPH | DTWS_LB_SORTED))
        return DTWS_EINVAL;
    if ((flags & DTWS_ORDER_MASK) == DTWS_ORDER_LEARNED && !c->has_model) return DTWS_ENOMODEL;
    for (int k = 0; k < nq; ++k)
        if (check_series(c, T, n, mh[k]) != DTWS_OK || rh[k] < 0 || qoff[k] < 0) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    return run_batch(c, T, n, Qp, qoff, mh, rh, nq, flags, seed, s, out);
}

DTWS_API int dtws_model_init(dtws_ctx *c, uint64_t seed) {
    if (!c) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, mlp_init(c->mlp, seed, nullptr));
    HIPCHK(c, hipStreamSynchronize(nullptr));
    c->has_model = true;
    c->model_step = 0;
    c->model_block = 0;
    return DTWS_OK;
}

DTWS_API int dtws_model_get(dtws_ctx *c, float *params, int64_t count) {
    if (!c || !params || count != kModelParams) return DTWS_EINVAL;
    if (!c->has_model) return DTWS_ENOMODEL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpy(params, c->mlp.theta, sizeof(float) * kModelParams, hipMemcpyDeviceToHost));
    return DTWS_OK;
}

DTWS_API int dtws_model_set(dtws_ctx *c, const float *params, int64_t count) {
    if (!c || !params || count != kModelParams) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpy(c->mlp.theta, params, sizeof(float) * kModelParams, hipMemcpyHostToDevice));
    HIPCHK(c, launch_fill_u32((uint32_t *)c->mlp.adam_m, 0, kModelParams, nullptr));
    HIPCHK(c, launch_fill_u32((uint32_t *)c->mlp.adam_v, 0, kModelParams, nullptr));
    HIPCHK(c, mlp_refresh(c->mlp, nullptr));
    HIPCHK(c, hipStreamSynchronize(nullptr));
    c->has_model = true;
    c->model_step = 0;
    c->model_block = 0;
    return DTWS_OK;
}

DTWS_API int dtws_model_forward(dtws_ctx *c, const float *X, int64_t rows, float *y, void *stream) {
    if (!c || !X || !y || rows < 0 || ((uintptr_t)X & 15u) != 0) return DTWS_EINVAL;   // rows are read as float4
    if (!c->has_model) return DTWS_ENOMODEL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    for (int64_t r0 = 0; r0 < rows; r0 += kMlpChunk) {
        const int64_t R = rows - r0 < kMlpChunk ? rows - r0 : kMlpChunk;
        HIPCHK(c, mlp_forward(c->mlp, X + r0 * 32, R, y + r0, false, s));
    }
    return DTWS_OK;
}

DTWS_API int dtws_model_grad(dtws_ctx *c, const float *X, const float *t, int64_t rows, float *grad, float *loss,
                             void *stream) {
    if (!c || !X || !t || !grad || rows < 1 || rows > kMaxTrainRows) return DTWS_EINVAL;
    if (!c->has_model) return DTWS_ENOMODEL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, mlp_backward(c->mlp, X, t, rows, s));
    HIPCHK(c, hipMemcpyAsync(grad, c->mlp.grad, sizeof(float) * kModelParams, hipMemcpyDeviceToDevice, s));
    if (loss) {
        HIPCHK(c, hipMemcpyAsync(loss, c->mlp.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return DTWS_OK;
}

DTWS_API int dtws_model_train_step(dtws_ctx *c, const float *X, const float *t, int64_t rows, float lr, float *loss,
                                   void *stream) {
    if (!c || !X || !t || rows < 1 || rows > kMaxTrainRows || !(lr > 0.0f)) return DTWS_EINVAL;
    if (!c->has_model) return DTWS_ENOMODEL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, mlp_backward(c->mlp, X, t, rows, s));
    HIPCHK(c, mlp_adam(c->mlp, ++c->model_step, lr, s));
    if (loss) {
        HIPCHK(c, hipMemcpyAsync(loss, c->mlp.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return DTWS_OK;
}

DTWS_API int dtws_paa(dtws_ctx *c, const float *T, int64_t n, int32_t m, const int64_t *starts, int64_t count,
                      float *out, void *stream) {
    if (!c || !T || !starts || !out || count < 0 || m < 2 || m > c->max_m || n < m) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_paa(T, n, m, starts, count, out, (hipStream_t)stream));
    return DTWS_OK;
}

DTWS_API int dtws_propose(dtws_ctx *c, const float *T, int64_t n, const float *Q, int32_t m, int64_t *starts,
                         float *X, int64_t max_rows, int64_t *rows_out, void *stream) {
    if (check_series(c, T, n, m) != DTWS_OK || !rows_out) return DTWS_EINVAL;
    const int64_t rows = propose_rows(c, n, m);
    *rows_out = rows;
    if (!starts && !X) return DTWS_OK;
    if (!Q || !starts || !X || max_rows < rows) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, launch_query_prep(Q, m, 0, query_bufs(c, 0), s));
    const int rc = enqueue_propose(c, T, n, m, starts, X, s);
    if (rc != DTWS_OK) return rc;
    // the staging entries are read by the copies above before the call returns
    HIPCHK(c, hipStreamSynchronize(s));
    return DTWS_OK;
}

DTWS_API int dtws_znorm_stats(dtws_ctx *c, const float *T, int64_t n, int32_t m, double *mu, double *sigma,
                              void *stream) {
    if (check_series(c, T, n, m) != DTWS_OK || !mu || !sigma) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_znorm_stats(T, n, m, mu, sigma, nullptr, nullptr, nullptr, (hipStream_t)stream));
    return DTWS_OK;
}

DTWS_API int dtws_lb_cascade(dtws_ctx *c, const float *T, int64_t n, const float *Q, int32_t m, int32_t r,
                             float threshold, float *kim, float *kq, float *kd, int32_t *surv, int64_t *n_surv,
                             void *stream) {
    if (check_series(c, T, n, m) != DTWS_OK || !Q || r < 0) return DTWS_EINVAL;
    if (surv && !n_surv) return DTWS_EINVAL;
    if (!kim && !kq && !kd && !surv) return DTWS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (r > m - 1) r = m - 1;
    const QueryBufs b = query_bufs(c, 0);
    HIPCHK(c, launch_query_prep(Q, m, r, b, s));
    HIPCHK(c, launch_znorm_stats(T, n, m, nullptr, nullptr, c->st_mu, c->st_s, c->st_o, s));
    HIPCHK(c, launch_series_env(T, n, r, c->envU, c->envL, s));
    LbArgs l{};
    l.T = T;
    l.first = 0;
    l.last = n - m + 1;
    l.m = m;
    l.qh = b.qpad + kQPad;
    l.qs = b.qsorted;
    l.Us = b.Usorted;
    l.Ls = b.Lsorted;
    l.order = b.order;
    l.mu = c->st_mu;
    l.s = c->st_s;
    l.o = c->st_o;
    l.envU = c->envU;
    l.envL = c->envL;
    l.fixed_thr = threshold;
    l.out_kim = kim;
    l.out_kq = kq;
    l.out_kd = kd;
    if (kim || kq || kd) HIPCHK(c, launch_lb(l, 0, c->num_cu, s));
    if (surv) {
        HIPCHK(c, launch_fill_u32(c->surv_count, 0, 1, s));
        l.surv = surv;
        l.surv_count = c->surv_count;
        HIPCHK(c, launch_lb(l, 1, c->num_cu, s));
        uint32_t cnt = 0;
        HIPCHK(c, hipMemcpyAsync(&cnt, c->surv_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        *n_surv = cnt;
    }
    return DTWS_OK;
}

DTWS_API int dtws_dtw_band(dtws_ctx *c, const float *T, int64_t n, const float *Q, int32_t m, int32_t r,
                           const int64_t *starts, int64_t count, float abandon_at, float *dist, void *stream) {
    if (check_series(c, T, n, m) != DTWS_OK || !Q || r < 0 || !starts || !dist || count < 0) return DTWS_EINVAL;
    if (count == 0) return DTWS_OK;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (r > m - 1) r = m - 1;
    const QueryBufs b = query_bufs(c, 0);
    HIPCHK(c, launch_query_prep(Q, m, r, b, s));
    DtwArgs d{};
    d.T = T;
    d.m = m;
    d.r = r;
    d.w = 2 * r + 1;
    d.qpad = b.qpad;
    d.starts64 = starts;
    d.count = count;
    d.n = n;
    d.single = -1;
    d.abandon_at = abandon_at;
    d.nb_cap = nb_cap_of(c);
    d.dist_out = dist;
    const bool wave = r <= kDiagMaxBand &&
                      (c->band_lanes == 64 ||
                       (c->band_lanes == 0 && (2 * r + 1 > 16 * kMaxChunks || count <= diag_max_of(c))));
    if (wave) {
        const int64_t blocks = (count + 1) / 2;
        HIPCHK(c, launch_dtw_diag_list(d, false, (int)(blocks < c->num_cu * 8 ? blocks : c->num_cu * 8), s));
    } else if (2 * r + 1 > 16 * kMaxChunks) {
        HIPCHK(c, launch_dtw(d, false, count, c->num_cu, c->gen_rows, c->gen_lanes, s));
    } else {
        // one lane per candidate, as in the search: the windows' normalisation first (one coalesced
        // wave per start, into the context's statistics arrays), in pieces of at most max_n starts
        for (int64_t k0 = 0; k0 < count; k0 += c->max_n) {
            const int64_t cnt = count - k0 < c->max_n ? count - k0 : c->max_n;
            HIPCHK(c, launch_start_stats(T, n, m, starts + k0, cnt, c->st_mu, c->st_s, c->st_o, c->num_cu, s));
            DtwArgs dk = d;
            dk.starts64 = starts + k0;
            dk.count = cnt;
            dk.dist_out = dist + k0;
            dk.mu = c->st_mu;
            dk.s = c->st_s;
            dk.o = c->st_o;
            dk.stats_by_k = true;
            HIPCHK(c, launch_dtw(dk, false, cnt, c->num_cu, c->gen_rows, c->gen_lanes, s));
        }
    }
    return DTWS_OK;
}

DTWS_API int dtws_bsf_update(dtws_ctx *c, uint64_t *keys, const float *d, const int64_t *idx, int64_t count,
                             void *stream) {
    if (!c || !keys || !d || !idx || count < 0) return DTWS_EINVAL;
    if (count == 0) return DTWS_OK;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_bsf_update(keys, d, idx, count, c->num_cu, (hipStream_t)stream));
    return DTWS_OK;
}

}  // extern "C"
