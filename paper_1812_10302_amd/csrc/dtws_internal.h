// Internal declarations of the dtws library (not installed; include/dtws.h is the interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/dtws.h"

namespace dtws {

// Row sentinel: a normalised query value this far out makes (q - c)^2 overflow to +inf in FP32,
// so band cells whose row lies outside [0, m) (or above the band) cost +inf without branches.
constexpr float kSentinel = 1e20f;
// Padding of the sentinel-padded query on each side (elements); >= the largest band.
constexpr int kQPad = 4096 + 64;
constexpr int kMaxM = 2048;
// Pruning slack: a bound or partial DTW computed in FP32 is compared with
// bsf * (1 + kEpsRel) + kEpsAbs so that FP32 rounding can never discard the FP64 best.
constexpr float kEpsRel = 1.0f / 1024.0f;
constexpr float kEpsAbs = 1e-6f;
constexpr double kSigmaFlat = 1e-8;
// Largest band (2r+1) handled by the register-resident DTW kernel (16-cell chunks).
constexpr int kMaxChunks = 14;
constexpr int kNearBestCap = 1 << 20;

__host__ __device__ inline float threshold_of(float bsf) {
    return bsf * (1.0f + kEpsRel) + kEpsAbs;   // +inf stays +inf
}

__device__ inline uint64_t pack_key(float d, uint32_t idx) {
    return (uint64_t(__float_as_uint(d)) << 32) | uint64_t(idx);
}
__device__ inline float key_dist(uint64_t k) { return __uint_as_float(uint32_t(k >> 32)); }

// Per-query device buffers, all inside the context's arrays.
struct QueryBufs {
    float *qpad;      // [2*kQPad + m] sentinel-padded normalised query (FP32)
    double *qhat64;   // [m] normalised query (FP64)
    float *qsorted;   // [m] normalised query in the LB visiting order
    float *Usorted;   // [m] query envelope (upper) in the LB visiting order
    float *Lsorted;   // [m] query envelope (lower) in the LB visiting order
    float *Unat;      // [m] query envelope (upper) in natural order
    float *Lnat;      // [m] query envelope (lower) in natural order
    int32_t *order;   // [m] LB visiting order: positions by decreasing expected LB_Keogh term
};


constexpr int kPBShift = 12;
constexpr int kPB = 1 << kPBShift;       // blocked prefix: block length (points)

// Blocked prefix of the series: blocks of kPB points, anchor anc[b] = T[b * kPB]; for x in block b,
// PP[x] = (sum, sum of squares) of (T[y] - anc[b]) over [b * kPB, x) and tot[b] the same over the
// whole block.  Only the even entries are stored, PPe[k] = PP[2 k]: an odd entry is the even one
// before it plus the single point between them (an odd x never starts a block, so that point has
// x's anchor).  One entry past the last block (anchor repeated, zero sums) and PP[n] exist, so
// readers may touch them without a test.
struct Prefix {
    const double2 *PPe;
    const double *anc;
    const double2 *tot;
    const float *T;   // the series the prefix was built from
    __device__ double2 at(int64_t x) const {
        double2 e = PPe[x >> 1];
        if (x & 1) {
            const double d = (double)T[x - 1] - anc[x >> kPBShift];
            e.x += d;
            e.y = fma(d, d, e.y);
        }
        return e;
    }
};

// Decimated copies of the prefix for the proposals of the learned order: lv[L][k] = PP[k << L],
// L = 3..5 (every 8th .. 32nd entry; shorter steps read the series), written by the prefix pass
// for the levels it is asked for.
constexpr int kDecFirst = 3, kDecLevels = 6;
struct Decimated {
    double2 *lv[kDecLevels];
};

// Per-query parameters of a batch (device array, one entry per query).
struct BatchQ {
    int64_t qoff;      // first element of the query in the packed query array
    int64_t N;         // candidates n - m + 1
    int32_t m, r;      // length and band (r clamped to m - 1)
    int32_t nc;        // DTW bucket: register chunks (1..kMaxChunks), kMaxChunks + 1 = wide band
    int32_t nblocks;   // work items: ceil(N / block)
    int32_t stat_slot; // per-window statistics slot (distinct lengths), when not using the prefix
    int32_t env_slot;  // data-envelope slot (distinct bands, or the batch's largest band)
};

// ---------------------------------------------------------------- kernel arguments
struct LbArgs {
    const float *T;
    int64_t first, last;   // candidate range [first, last)
    int m;
    const float *qh;       // normalised query, natural order (qpad + kQPad)
    const float *qs, *Us, *Ls;
    const int32_t *order;
    const float *mu, *s, *o;
    const float *envU, *envL;
    const uint64_t *key;   // best-so-far key (threshold source) or null
    float fixed_thr;       // threshold when key is null
    float *out_kim, *out_kq, *out_kd;
    uint64_t *out_key;     // stage values: (bits(max of the three bounds) << 32) | start, or null
    int32_t *surv;
    uint32_t *surv_count;
    unsigned long long *counters;
};

struct DtwArgs {
    const float *T;
    int m, r, w;                 // r clamped to m-1, w = 2r+1
    const float *qpad;           // sentinel-padded normalised query
    const int32_t *starts32;     // candidate starts (search mode) ...
    const int64_t *starts64;     // ... or explicit starts (stage entry point), else range_first + k
    int64_t range_first;
    int64_t n;                   // series length: explicit starts outside [0, n-m] are rejected (NaN out)
    const uint32_t *count_dev;   // device-side count of starts32 (search mode) or null
    int64_t count;               // host count, or capacity bound when count_dev is set
    int64_t single;              // >= 0: evaluate only this start
    const float *mu, *s, *o;     // per-window normalisation, or null to compute per lane
    bool stats_by_k;             // mu/s/o are indexed by the list position k, not by the start
    const float *Un, *Ln;        // natural-order query envelope for the suffix bound, or null (off)
    float abandon_at;            // threshold of the stage entry point
    uint32_t diag_max;           // search rounds of at most this many survivors: one wave per candidate
    uint32_t nb_cap;             // capacity of the near-best list (entries beyond it are dropped and
                                 // the certification reports an overflow)
    float *dist_out;             // stage entry point output
    uint64_t *key;               // search mode: best-so-far key
    float *nb_d;
    uint32_t *nb_idx, *nb_count;
    unsigned long long *counters;
};

struct CertArgs {
    const float *T;
    int m, r;
    const double *qhat64;
    const uint64_t *key;
    const float *nb_d;
    const uint32_t *nb_idx, *nb_count;
    double *scratch;    // [256 * 3 * (m + 1)] (wide-band fallback)
    uint32_t *cert_idx; // [1024] compacted qualifying candidates
    uint32_t *cert_count;
    double *cert_d;     // [1024] their FP64 distances
    uint32_t nb_cap;    // capacity of the near-best and certification lists
    int64_t *res_idx;
    double *res_dist;
    int32_t *res_status;
    unsigned long long *counters;
};

// Per-query counters updated by atomics from every wave (survivors per query, segment fill) sit one
// 128-byte cache line apart, so that the atomics of different queries do not serialise on a line.
constexpr int kCntStride = 32;

// Eviction from the refilling-rows DTW kernel: a row whose live candidates have dropped to a few
// moves them, band column and all, into an entry of kEvStride floats (the column, then the meta
// words below), and takes new candidates; the moved ones are bucketed by (query, column) and
// resumed in full rows.  kEvLevels bounds the column levels (columns / 16) of a query.
constexpr int kEvStride = 232;                 // 16 * kMaxChunks + 1 column values, padded, + 5 meta
constexpr int kEvKpre = 227, kEvLbt = 228, kEvStart = 229, kEvQ = 230, kEvCol = 231;
constexpr int kEvDepth = 3;                    // resume launches per bucket (the last one evicts nothing)

struct BatchArgs {
    const float *T;
    int64_t n;
    int nq;
    int64_t block;             // candidates per work item
    int max_m;
    const BatchQ *bq;
    const float *qpad;         // per query, stride qstride
    int64_t qstride;
    const double *qhat64;      // per query, stride max_m
    const int32_t *order;      // per query, stride mstride (16-padded visiting order)
    const float *Us, *Ls, *qs;
    const float *Un, *Ln;      // per query, stride mstride: envelope in natural order
    int64_t mstride;
    int rows;                  // lane DTW of 4+ chunks: refilling rows (k_dtw_batch_rows)
    uint64_t *keys;            // best-so-far per query
    // window statistics: per-window arrays (all queries share m) or the blocked prefix
    const float *mu, *s, *o;
    Prefix pre;
    const float *envU, *envL;  // data envelopes (slot per distinct band), or null
    int64_t slot_stride;       // elements per statistics / envelope slot
    // work queue
    int32_t *perm;             // per query: block visiting order, stride maxblocks
    int32_t *rank;             // its inverse: rank of each block in the query's order
    int64_t maxblocks;
    uint32_t *heads;           // per round
    // survivors of the bound cascade, then sorted into per-query wave segments
    int32_t *surv_q, *surv_i;
    float *surv_lb;            // each survivor's query-envelope LB_Keogh sum (0 where none was taken)
    uint32_t *surv_count, *qcnt, *overflow;   // qcnt and fill: one 128-byte line per query (kCntStride)
    int64_t surv_cap;
    int32_t *sorted;
    float *sorted_lb;          // surv_lb in the order of `sorted`
    int32_t *qorder, *wstart;
    int64_t *seg_off;
    uint32_t *fill;
    int32_t *bucket_w, *bucket_j;
    // near-best list and certification
    float *nb_d;
    uint32_t *nb_idx;
    int32_t *nb_q;
    uint32_t *nb_count;
    uint32_t *cert_idx;
    int32_t *cert_q;
    uint32_t *cert_count;
    double *cert_d;
    int64_t *res_idx;
    double *res_dist;
    int32_t *res_status;
    unsigned long long *counters;
    float *wide_rows;
    int64_t wide_lanes;
    uint32_t diag_max;         // rounds with at most this many survivors use one wave per candidate
    uint32_t nb_cap;           // capacity of the near-best and certification lists
    bool diag_wide;            // bands 112..255 always use one wave per candidate
    // eviction (k_dtw_batch_rows): rows with 1..ev_live live candidates move them to ev_out
    int ev_live;               // 0: off
    float *ev_out;             // entries of kEvStride floats, in 8 parts of ev_cap / 8 (one per XCD)
    uint32_t *ev_out_count;    // the parts' counts, kCntStride apart
    uint32_t *ev_out_key;      // each entry's bucket key: query * ev_levels + column / 16
    const float *ev_in;        // entries being resumed (resume launches)
    const uint32_t *ev_in_key;
    const uint32_t *ev_in_count;
    int64_t ev_cap;            // entries per buffer
    uint32_t *ev_order;        // resume rows: 16 entry indices per row, ~0u = empty lane
    uint32_t *ev_rows;         // number of resume rows
    uint32_t *ev_kcnt, *ev_koff, *ev_kfill;   // per (query, column level): count, offset, fill
    int ev_levels;             // column levels per query (max_m / 16 + 1)
};

// Tiled bound cascade (tile.hip): the queries of a batch grouped by length.
struct TileArgs {
    const int32_t *gfirst;   // [ngroups + 1]: group g's queries are qlist[gfirst[g] .. gfirst[g + 1])
    const int32_t *qlist;    // query indices sorted by length
    int ngroups;
    int64_t c_lo, c_hi;      // candidate starts of the round, the same for every query
    int halo;                // largest query length of the batch - 1
    int skip_below;          // > 0: a query skips the tiles of blocks it ranked below this (visited)
    int64_t block;           // candidates per block (for skip_below)
};

// ---------------------------------------------------------------- ordering network
constexpr int64_t kModelParams = 32 * 256 + 256 + 256 * 256 + 256 + 256 + 1;
constexpr int64_t kOffW1 = 0, kOffb1 = 32 * 256, kOffW2 = kOffb1 + 256, kOffb2 = kOffW2 + 256 * 256,
                  kOffw3 = kOffb2 + 256, kOffb3 = kOffw3 + 256;
constexpr int64_t kMlpChunk = 1 << 18;   // rows per forward pass (workspace size)
constexpr int kScoreSamples = 4;         // proposals scored per block (one per quarter block)
constexpr int kSeedBlocks = 16;          // best-scored blocks per query whose proposals seed the best-so-far
constexpr int kSeedOffsets = 16;         // starts evaluated around each of them: proposal - 8 .. proposal + 7
constexpr int kSeedCands = kSeedBlocks * kSeedOffsets;
constexpr int kColsumGroups = 128;       // row groups of the bias-gradient reduction
constexpr int64_t kMaxTrainRows = 1 << 16;  // rows per gradient / training step

struct MlpBufs {
    float *theta, *grad, *adam_m, *adam_v;   // FP32 master parameters, gradient, Adam moments
    uint16_t *W1T, *W2T, *W2b;               // bfloat16 weight copies
    uint16_t *Xb, *XbT, *H1b, *H1T, *dA2b, *dA2T, *dA1T;
    float *C1, *C2, *y, *dy, *loss, *Xf;
    float *part;                             // kColsumGroups x 4 x 256 partial column sums
    int num_cu;                              // compute units of the device (width of the fused forward)
};

// Scoring of a batch: row (q, blk, j) = row_off[q] + blk * K + j is the proposal of quarter j
// of block blk of query q; score and bstart are indexed by row_off[q] / K + blk.
struct ScoreArgs {
    int K;
    int64_t total_rows;
    float *qpaa, *score;
    int32_t *sstart;           // start of each row of the current chunk (-1: empty quarter)
    int32_t *bstart;           // start of the best-scored proposal of each block
    const int64_t *row_off;    // per query, nq + 1 entries
    Prefix pre;                // blocked prefix of the series
    Decimated dec;             // its decimated copies
    uint32_t dec_levels;       // bit L set: dec.lv[L] holds the current series
    uint32_t kinds;            // bit 0: some query length is a multiple of 64, bit 1: some is not
};

// ---------------------------------------------------------------- launchers (stream-ordered)
hipError_t launch_query_prep(const float *Q, int m, int r, const QueryBufs &b, hipStream_t s);
hipError_t launch_query_prep_batch(const float *Qp, const BatchQ *bq, int nq, const QueryBufs &base,
                                  int64_t qstride, int64_t mstride, int64_t m64stride, hipStream_t s);
hipError_t launch_znorm_stats(const float *T, int64_t n, int m, double *mu, double *sg, float *mu32, float *s32,
                              float *o32, hipStream_t s);
hipError_t launch_series_env(const float *T, int64_t n, int r, float *U, float *L, hipStream_t s);
hipError_t launch_lb(const LbArgs &a, int mode, int num_cu, hipStream_t s);
hipError_t launch_lb_sorted_segment(const uint64_t *keys, int64_t a0, int64_t a1, const uint64_t *bsf_key,
                                    int32_t *surv, uint32_t *count, int num_cu, hipStream_t s);
hipError_t sort_keys_u64(void *temp, size_t &temp_bytes, const uint64_t *in, uint64_t *out, int64_t count,
                         hipStream_t s);
hipError_t launch_dtw(const DtwArgs &a, bool search, int64_t max_count, int num_cu, float *wide_rows,
                      int64_t wide_lanes, hipStream_t s);
hipError_t launch_bsf_update(uint64_t *keys, const float *d, const int64_t *idx, int64_t count, int num_cu,
                             hipStream_t s);
hipError_t launch_certify(const CertArgs &c, hipStream_t s);
hipError_t launch_prefix(const float *T, int64_t n, double2 *PP, double *anc, double2 *tot, hipStream_t s,
                         const Decimated *dec = nullptr, uint32_t levels = 0);
hipError_t launch_make_perm(const BatchArgs &a, int mode, uint64_t seed, int64_t max_nblocks, hipStream_t s);
hipError_t launch_perm_rank(const BatchArgs &a, int64_t max_nblocks, hipStream_t s);
hipError_t launch_seed_random(const BatchArgs &a, uint64_t seed, hipStream_t s);
hipError_t launch_lb_batch(const BatchArgs &a, bool prefix, int round, int rank_lo, int rank_hi, int parts,
                           bool natural, int skip_below, int blocks, hipStream_t s);
hipError_t launch_segments(const BatchArgs &a, int num_cu, hipStream_t s);
hipError_t launch_lb_tile(const BatchArgs &a, const TileArgs &t, bool prefix, int64_t max_N, hipStream_t s);
size_t tile_lds_bytes(int max_m);
hipError_t launch_dtw_bucket(const BatchArgs &a, bool prefix, int nc, int blocks, hipStream_t s);
hipError_t launch_dtw_resume(const BatchArgs &a, bool prefix, int nc, int blocks, int num_cu, hipStream_t s);
hipError_t launch_cert_batch(const BatchArgs &a, int max_m, int max_r, hipStream_t s);
hipError_t mlp_init(const MlpBufs &b, uint64_t seed, hipStream_t s);
hipError_t mlp_refresh(const MlpBufs &b, hipStream_t s);
hipError_t mlp_forward(const MlpBufs &b, const float *X, int64_t R, float *y, bool train, hipStream_t s);
hipError_t mlp_backward(const MlpBufs &b, const float *X, const float *t, int64_t R, hipStream_t s);
hipError_t mlp_adam(const MlpBufs &b, int step, float lr, hipStream_t s);
hipError_t mlp_order_blocks(const MlpBufs &b, const BatchArgs &a, const ScoreArgs &sa, bool paa_only, hipStream_t s);
hipError_t launch_seed_learned(const BatchArgs &a, const ScoreArgs &sa, hipStream_t s);
hipError_t launch_propose(const BatchArgs &a, const ScoreArgs &sa, float *X, int64_t *starts, hipStream_t s);
constexpr int kDiagMaxBand = 1023;       // widest band of the one-wave-per-candidate kernels
constexpr int kDiagMaxBandNarrow = 255;  // widest band of their narrow instances (smaller pads)
size_t diag_lds_bytes(int max_m, bool fp64, int max_r);
hipError_t launch_dtw_diag(const BatchArgs &a, bool prefix, int max_r, int blocks, hipStream_t s);
hipError_t launch_cert_diag(const BatchArgs &a, int max_r, int blocks, hipStream_t s);
hipError_t launch_dtw_diag_list(const DtwArgs &a, bool search, int blocks, hipStream_t s);
hipError_t launch_cert_diag_list(const CertArgs &c, int blocks, hipStream_t s);
hipError_t launch_start_stats(const float *T, int64_t n, int m, const int64_t *starts, int64_t count, float *mu,
                              float *sg, float *off, int num_cu, hipStream_t s);
hipError_t launch_paa(const float *T, int64_t n, int m, const int64_t *starts, int64_t count, float *out,
                      hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_reset_batch(uint64_t *keys, int nq, unsigned long long *counters, int ncounters, uint32_t *heads,
                              int nheads, uint32_t *nb_count, uint32_t *cert_count, uint32_t *overflow, hipStream_t s);
// key of an empty best-so-far: distance +inf, index 0xFFFFFFFF
constexpr uint64_t kEmptyKey = (uint64_t(0x7F800000u) << 32) | 0xFFFFFFFFull;

}  // namespace dtws

// Host helpers shared by the C ABI's translation units (defined in api.hip).
namespace dtws {
int64_t learned_block(const dtws_ctx *c);
int64_t propose_rows(const dtws_ctx *c, int64_t n, int m);
int enqueue_propose(dtws_ctx *c, const float *T, int64_t n, int m, int64_t *starts, float *X, hipStream_t s);
QueryBufs query_bufs_of(dtws_ctx *c, int slot);
void set_hip_error(dtws_ctx *c, hipError_t e, const char *what);
}  // namespace dtws

// Opaque context (declared in dtws.h).
struct dtws_ctx {
    int device = 0;
    int num_cu = 0;
    int64_t max_n = 0;
    int32_t max_m = 0, max_q = 0;
    // per-query buffers, stride qstride floats / max_m elements
    int64_t qstride = 0;
    int64_t mstride = 0;                  // per-query stride of the 16-padded sorted arrays
    float *qpad = nullptr;
    double *qhat64 = nullptr;
    float *qsorted = nullptr, *Usorted = nullptr, *Lsorted = nullptr;
    float *Unat = nullptr, *Lnat = nullptr;   // query envelope in natural order, stride mstride
    int32_t *order = nullptr;
    uint64_t *keys = nullptr;             // best-so-far key per query
    // series-sized scratch
    float *st_mu = nullptr, *st_s = nullptr, *st_o = nullptr;   // per-candidate normalisation
    float *envU = nullptr, *envL = nullptr;                     // raw series envelope(s)
    int nslots = 1;                       // statistics / envelope slots of max_n elements each
    int32_t *surv = nullptr;              // survivor starts
    int64_t surv_cap = 0;
    uint32_t *surv_count = nullptr;
    // near-best list
    float *nb_d = nullptr;
    uint32_t *nb_idx = nullptr;
    uint32_t *nb_count = nullptr;
    // certification scratch and results
    double *cert_rows = nullptr;          // [256 * 2 * (max_m + 1)]
    uint32_t *cert_idx = nullptr;         // [1024] compacted qualifying candidates
    uint32_t *cert_count = nullptr;
    double *cert_d = nullptr;             // [1024]
    int64_t *res_idx = nullptr;           // device [max_q]
    double *res_dist = nullptr;           // device [max_q]
    int32_t *res_status = nullptr;        // device [max_q]
    unsigned long long *counters = nullptr;  // device [8]
    float *gen_rows = nullptr;            // scratch for the wide-band DTW kernel
    int64_t gen_lanes = 0;
    // batched search
    dtws::BatchQ *bq = nullptr, *h_bq = nullptr;   // device / pinned host, max_q entries
    double2 *PP = nullptr;                   // blocked prefix, max_n + 1 entries
    double2 *PPd = nullptr;                  // its decimated copies (see Decimated)
    dtws::Decimated dec{};
    double *anc = nullptr;
    double2 *tot = nullptr;
    int32_t *perm = nullptr, *rank = nullptr;
    int64_t maxblocks = 0;
    uint32_t *heads = nullptr;
    int32_t *surv_q = nullptr, *surv_i = nullptr, *sorted = nullptr;
    float *surv_lb = nullptr, *sorted_lb = nullptr;
    int64_t bsurv_cap = 0;
    uint32_t *qcnt = nullptr, *fill = nullptr, *overflow = nullptr;
    int32_t *qorder = nullptr, *wstart = nullptr, *bucket_w = nullptr, *bucket_j = nullptr;
    int64_t *seg_off = nullptr;
    int32_t *nb_q = nullptr, *cert_q = nullptr;
    // graph of the last batched call, its signature, and the stream it runs on
    hipStream_t gstream = nullptr;
    hipEvent_t gevent = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> graph_sig;
    int64_t graph_launches = 0;
    // tuning knobs (0 = default): candidates per work item, launch widths per compute unit
    int64_t block = 0;
    int lb_blocks_per_cu = 0, dtw_blocks_per_cu = 0;
    int diag_max = -1;   // survivors per round below which DTW runs one wave per candidate (-1: default)
    int band_lanes = 0;  // dtws_dtw_band: 0 = automatic, 1 = one lane per candidate, 64 = one wave per candidate
    int stats_prefix = 0;   // batched: 1 = window statistics always from the blocked prefix
    int data_envelope = 1;  // batched: 0 = skip the data-envelope bound
    int rounds = 4;         // batched: rounds over the work queue (4, 2 or 1)
    int list_cap = 0;       // capacity of the near-best and batched survivor lists (0 = full size)
    int lb_tile = 1;        // batched: tiled multi-query cascade for rounds over the same candidates
    int dtw_bound = 1;      // search DTW on one lane per candidate: suffix bound in the abandoning test
    int dtw_rows = 1;       // batched lane DTW (bands of 4+ chunks): rows of 16 lanes refill from a chunk
    int dtw_evict = 4;      // rows kernel: move a row's live candidates out when at most this many remain
    float *ev_buf[2] = {nullptr, nullptr};   // eviction entries, ev_cap each
    uint32_t *ev_keybuf[2] = {nullptr, nullptr};   // their bucket keys
    uint32_t *ev_count = nullptr;            // per buffer 8 part counts (kCntStride apart), then resume rows
    int64_t ev_cap = 0;
    uint32_t *ev_order = nullptr;            // ev_cap + 16 per key
    uint32_t *ev_keys = nullptr;             // 3 x max_q x ev_levels: count, offset, fill
    int ev_levels = 0;
    uint64_t *lbs_keys = nullptr;   // LB-sorted order: 2 x max_n keys and the sort's temporary storage,
    void *lbs_temp = nullptr;       // allocated on first use
    size_t lbs_temp_bytes = 0;
    int32_t *tile_q = nullptr, *h_tile_q = nullptr;   // device / pinned: groups by length, then queries
    // ordering network
    dtws::MlpBufs mlp{};
    bool has_model = false;
    int model_step = 0;
    int64_t model_block = 0;   // work-item block the model was trained with (0: none recorded)
    float *qpaa = nullptr, *score = nullptr;
    int32_t *sstart = nullptr, *bstart = nullptr;
    int64_t *row_off = nullptr, *h_row_off = nullptr;
    // pinned host staging
    int64_t *h_idx = nullptr;
    double *h_dist = nullptr;
    int32_t *h_status = nullptr;
    // the result arrays and the counters in one device and one pinned host block, fetched by one copy
    uint8_t *res_block = nullptr, *h_res_block = nullptr;
    size_t res_bytes = 0;
    unsigned long long *h_counters = nullptr;
    dtws_counters last{};
    // profiling (DTWS_PROFILE): event pairs around launches, class per pair
    static constexpr int kMaxEvents = 8192;
    hipEvent_t *ev = nullptr;             // 2 * kMaxEvents events
    int *ev_class = nullptr;
    int ev_used = 0;
    bool profiling = false;
    double prof_ms[DTWS_K_COUNT] = {0};
    int64_t prof_n[DTWS_K_COUNT] = {0};
    char lasterr[256] = {0};
};
