/*
 * dtws.h -- exact best-match subsequence search under banded, z-normalised,
 * squared Dynamic Time Warping on one AMD Instinct MI355X (gfx950).
 *
 * The problem (Kraeva & Zymbler, arXiv:1812.10302, Section 2.1, best-match
 * definition, and Algorithm 1 "PhiBestMatch(in T, Q, r; out bsf, bestmatch)"):
 * given a series T of n points, a query Q of m points and a Sakoe-Chiba band
 * of r points, find the start i in [0, n-m] that minimises
 *     DTW_r( znorm(Q), znorm(T[i .. i+m-1]) )
 * where DTW is the recurrence of eq. (dtw) with cells |a-b| > r excluded, the
 * distance is squared (the square root is dropped, Section 2.2, eq. (Euclidean)
 * and the remark after it) and znorm is eq. (Normalization1) with the
 * population sigma.  Ties resolve to the lowest start index.  A window whose
 * sigma is <= 1e-8 normalises to all zeros.  r >= m-1 means unconstrained DTW.
 *
 * Conventions for every call below:
 *  - Pointers named *_dev are DEVICE pointers on the context's device (for
 *    example torch.Tensor.data_ptr() of a CUDA/HIP tensor), contiguous, owned
 *    by the caller, never retained after the call returns.  Pointers named
 *    *_host are host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Kernels are enqueued on it; calls documented as "blocking" synchronise
 *    it before returning, the others return as soon as the work is enqueued.
 *  - The context owns every scratch buffer; they are allocated by
 *    dtws_create and sized by its limits.  Nothing is allocated per call
 *    except where a call's comment says so.
 *  - Return value: DTWS_OK or a negative error code.  Argument errors are
 *    detected before any device work is enqueued.  After DTWS_EHIP,
 *    dtws_last_error() returns the HIP error text.  No C++ exception ever
 *    crosses this interface.
 *  - A context may be used by one host thread at a time; calls that share a
 *    context must not overlap.
 */
#ifndef DTWS_H
#define DTWS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DTWS_API __attribute__((visibility("default")))

typedef struct dtws_ctx dtws_ctx;

enum dtws_status {
    DTWS_OK = 0,
    DTWS_EINVAL = -1,    /* bad argument (null pointer, m < 2, m > n, r < 0, over a limit) */
    DTWS_ENOMEM = -2,    /* device allocation failed in dtws_create                       */
    DTWS_ENODEV = -3,    /* no HIP device, or the device ordinal does not exist           */
    DTWS_EHIP = -4,      /* a HIP runtime call failed; see dtws_last_error                */
    DTWS_EOVERFLOW = -5, /* an internal list overflowed; the result would not be certain  */
    DTWS_ENOMODEL = -6   /* learned ordering asked for but no model is loaded/trained     */
};

/* Search flags (bit set). */
#define DTWS_ORDER_NATURAL 0u        /* blocks in series order (plain search)                     */
#define DTWS_ORDER_RANDOM 1u         /* blocks in a seeded random permutation                     */
#define DTWS_ORDER_LEARNED 2u        /* blocks by ascending score of the learned model            */
#define DTWS_ORDER_PAA 3u            /* blocks by ascending PAA distance of the same proposals the
                                        learned model scores (no network): the learned order's
                                        control, batched calls only                                */
#define DTWS_ORDER_MASK 3u
#define DTWS_NO_LOWER_BOUNDS 4u      /* skip the bound cascade: DTW (with abandoning) on all      */
#define DTWS_PROFILE 8u              /* time every kernel with HIP events on the call's stream
                                        (adds an event pair per launch); see dtws_get_profile     */

#define DTWS_NO_GRAPH 16u            /* batched calls: enqueue eagerly instead of replaying a graph */
#define DTWS_LB_SORTED 32u           /* the Prepare / Improve scheme of Section 3.3 (Algorithm 1):
                                        every candidate's three bounds computed once, independent of
                                        the best-so-far (eq. (lbMatrix)), their maximum sorted, and
                                        the candidates visited in ascending order of it, in segments
                                        that each run DTW on the candidates whose bound is still
                                        within the best-so-far (eqs. (bitmapMatrix), (candidateMatrix)).
                                        A non-learned ordering; same results.  Batched calls run it
                                        query by query.  Allocates 16 B per point of max_n on first use */

/* Kernel classes reported by dtws_get_profile. */
enum dtws_kernel_class {
    DTWS_K_PREP = 0,    /* query normalisation, envelope, visiting order        */
    DTWS_K_STATS = 1,   /* per-window mean / sigma                               */
    DTWS_K_ENV = 2,     /* raw-series envelope                                   */
    DTWS_K_LB = 3,      /* lower-bound cascade                                   */
    DTWS_K_DTW = 4,     /* banded DTW, one lane per candidate (with the best-so-far
                           update)                                               */
    DTWS_K_CERT = 5,    /* FP64 certification                                    */
    DTWS_K_OTHER = 6,   /* fills and bookkeeping                                 */
    DTWS_K_SCORE = 7,   /* learned ordering: features, network, block order      */
    DTWS_K_DTW_WAVE = 8,   /* banded DTW, one wave per candidate (with the update)  */
    DTWS_K_COUNT = 9
};

/* Result of one search: 0-based start and its squared z-normalised DTW
 * distance, certified in FP64.  status is DTWS_OK or an error code. */
typedef struct {
    int64_t index;
    double distance;
    int32_t status;
    int32_t reserved;
} dtws_match;

/* Counters of the last search call on a context (summed over its queries). */
typedef struct {
    int64_t candidates;        /* starts considered                                     */
    int64_t pruned_kim;        /* discarded by LB_KimFL                                 */
    int64_t pruned_keogh_q;    /* discarded by LB_Keogh against the query envelope      */
    int64_t pruned_keogh_d;    /* discarded by LB_Keogh against the data envelope       */
    int64_t dtw_started;       /* candidates whose DTW was started                      */
    int64_t dtw_abandoned;     /* ... and abandoned early                               */
    int64_t dtw_cells;         /* band cells evaluated by DTW (including abandoned)     */
    int64_t certified;         /* near-best candidates re-evaluated in FP64             */
    int64_t dtw_lane_cells;    /* lane-cells issued by the DTW kernels: band bucket x
                                  columns x 64 lanes per wave step, idle lanes included */
    int64_t lb_terms;          /* query-envelope LB_Keogh terms evaluated by the tiled
                                  batched cascade (0 for the other cascade kernels)     */
    int64_t fallbacks;         /* batched queries redone by the plain search after a
                                  list overflowed (their work is not in the counters)   */
    int64_t dtw_wave_cells;    /* the part of dtw_cells evaluated by the one-wave-per-
                                  candidate DTW kernels                                 */
    int64_t dtw_evicted;       /* candidates moved out of a DTW row to resume in another
                                  (schedule field dtw_evict; one candidate may move up
                                  to twice)                                             */
} dtws_counters;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` able to search series of up to
 * max_n points (max_n < 2^31) with queries of up to max_m points (2 <= max_m
 * <= 2048) and batches of up to max_queries queries.  Allocates all device
 * scratch: roughly 24 bytes per series point, small per-query buffers, and the
 * batched survivor list of 20 bytes per entry for min(max_queries * max_n, L)
 * entries, L = 2^30 on a device of at least 128 GiB, else 2^28, and two
 * buffers of 928 bytes per entry for the DTW rows' moved candidates (schedule
 * field dtw_evict), each of min(that list, E) entries (at least 4096), E = 2^25
 * on a device of at least 256 GiB (62 GB in all), 2^24 from 128 GiB, else 2^20.
 * Returns DTWS_ENODEV when no HIP device is present. */
DTWS_API int dtws_create(int device, int64_t max_n, int32_t max_m, int32_t max_queries, dtws_ctx **out);

/* Release the context and all its device memory.  NULL is accepted. */
DTWS_API void dtws_destroy(dtws_ctx *ctx);

/* Static text for an error code. */
DTWS_API const char *dtws_strerror(int code);

/* Text of the last HIP error seen on this context ("" if none). */
DTWS_API const char *dtws_last_error(dtws_ctx *ctx);

/* Number of HIP devices visible (0 when there is none). */
DTWS_API int dtws_device_count(void);

/* Counters of the last dtws_search / dtws_search_batch call. */
DTWS_API int dtws_get_counters(dtws_ctx *ctx, dtws_counters *out_host);

/* Per-kernel-class time of the last search call made with DTWS_PROFILE:
 * ms_host[k] = summed HIP-event time of class k's launches, launches_host[k] =
 * their number (arrays of DTWS_K_COUNT entries).  Zero when the last call
 * was not profiled. */
DTWS_API int dtws_get_profile(dtws_ctx *ctx, double *ms_host, int64_t *launches_host);

/* ------------------------------------------------------------------ search */

/* Best match of one query (Section 2.1 best-match definition; Algorithm 1
 * with the whole series as one fragment, Section 3.1, i.e. one node).
 *   T_dev[n] float32 series, Q_dev[m] float32 query, band r (clamped to m-1),
 *   flags: DTWS_ORDER_* and DTWS_NO_LOWER_BOUNDS, seed: picks the random
 *   candidate whose DTW initialises the best-so-far (Algorithm 1, the random
 *   subsequence) and the random order.  The result never depends on it.
 * Every candidate whose FP32 distance lies within the pruning slack of the
 * final best-so-far is certified in FP64.  When they outnumber the near-best
 * list (for example many exact ties: a flat query against a long flat stretch)
 * the series is scanned again in list-sized chunks under the final
 * best-so-far, so the result stays the lowest-index FP64 minimum.
 * Blocking: the result is written to *out_host when the call returns. */
DTWS_API int dtws_search(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_dev, int32_t m,
                         int32_t r, uint32_t flags, uint64_t seed, void *stream, dtws_match *out_host);

/* Best matches of nq queries of possibly different lengths and bands against
 * one series, all queries in one persistent launch with a device work queue.
 *   Q_packed_dev: the queries back to back; q_offsets_host[k] is query k's
 *   first element in it; m_host[k], r_host[k] its length and band.
 *   out_host[nq] receives one result per query.
 * Blocking.  Results are identical to nq calls of dtws_search. */
DTWS_API int dtws_search_batch(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_packed_dev,
                               const int64_t *q_offsets_host, const int32_t *m_host, const int32_t *r_host,
                               int32_t nq, uint32_t flags, uint64_t seed, void *stream, dtws_match *out_host);

/* ------------------------------------------------ stage-level entry points */

/* Per-window mean and population standard deviation of every length-m window
 * of T (eq. (Normalization1)); mu_dev[i], sigma_dev[i] for i in [0, n-m],
 * FP64.  Computed from FP64 sums anchored within tiles of the series. */
DTWS_API int dtws_znorm_stats(dtws_ctx *ctx, const float *T_dev, int64_t n, int32_t m, double *mu_dev,
                              double *sigma_dev, void *stream);

/* Lower bounds of every candidate i in [0, n-m] against query Q (Section 2.2):
 *   lb_kim_dev[i]     LB_KimFL, squared first-pair plus last-pair difference;
 *   lb_keogh_q_dev[i] sum of squared excursions of the normalised candidate
 *                     outside the query envelope (eq. (envelope), clipped);
 *   lb_keogh_d_dev[i] sum of squared excursions of the normalised query
 *                     outside the data envelope: max/min of the raw series
 *                     over [k-r, k+r] clipped to [0, n), mapped through the
 *                     candidate's normalisation (contains the candidate's own
 *                     envelope, hence a valid, looser bound).
 * Any of the three outputs may be NULL.  FP32.  When survivors_dev is not
 * NULL, also writes the starts with all three bounds <= threshold (in no
 * particular order) and their number to *n_survivors_host (blocking then). */
DTWS_API int dtws_lb_cascade(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_dev, int32_t m,
                             int32_t r, float threshold, float *lb_kim_dev, float *lb_keogh_q_dev,
                             float *lb_keogh_d_dev, int32_t *survivors_dev, int64_t *n_survivors_host,
                             void *stream);

/* Banded DTW (eq. (dtw) with the band) of the normalised query against the
 * normalised candidates at starts_dev[count] (each in [0, n-m]), FP32
 * arithmetic: dist_dev[k] receives the distance, or +inf if the evaluation
 * proved it exceeds abandon_at (pass +inf for exact values, no abandoning). */
DTWS_API int dtws_dtw_band(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_dev, int32_t m,
                           int32_t r, const int64_t *starts_dev, int64_t count, float abandon_at,
                           float *dist_dev, void *stream);

/* dtws_dtw_band for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no context, no
 * allocation.  The prepared query (about 105 KB) lives in a static device array of
 * this library, one per GPU, looked up on the first call on that GPU and held until
 * the process ends.  Runs on the current HIP device; arguments and results as
 * dtws_dtw_band.  Schedule: one wave per candidate when count <= 16384 or
 * 2r+1 > 224, else one lane per candidate normalising its window in the lane.
 * The query preparation rewrites all of the array that the DTW reads, so no
 * state carries over between calls.  Limits: m <= 2048 and
 * r <= 1023 after clamping r to m-1 (DTWS_EINVAL beyond them).  Every call on a GPU
 * shares that GPU's array: calls on one stream are ordered, calls that overlap on
 * one GPU (several streams or host threads) race. */
DTWS_API int dtws_dtw_band_noalloc(const float *T_dev, int64_t n, const float *Q_dev, int32_t m, int32_t r,
                                   const int64_t *starts_dev, int64_t count, float abandon_at, float *dist_dev,
                                   void *stream);

/* Best-so-far update (eq. (bsf)): for each k, atomically lowers keys_dev[0]
 * to min(keys_dev[0], (bits(d_dev[k]) << 32) | idx_dev[k]).  Keys order by
 * distance, then by index, so the minimum is the lowest-index best.
 * d_dev must be non-negative (or +inf), idx_dev in [0, 2^32). */
DTWS_API int dtws_bsf_update(dtws_ctx *ctx, uint64_t *keys_dev, const float *d_dev, const int64_t *idx_dev,
                             int64_t count, void *stream);

/* ---------------------------------------------------------------- schedule
 * How the work is cut and launched; no field changes a result.  dtws_set_schedule
 * takes 0 in block / lb_blocks_per_cu / dtw_blocks_per_cu and -1 in diag_max
 * for the defaults; dtws_get_schedule reports the values in effect. */
typedef struct {
    int64_t block;             /* candidates per work item of the batched search:
                                  2048, 4096 (default), 8192 or 16384 */
    int32_t lb_blocks_per_cu;  /* bound-cascade workgroups per compute unit, 1..64 (8) */
    int32_t dtw_blocks_per_cu; /* one-lane-per-candidate DTW workgroups per compute
                                  unit, 1..64 (4) */
    int32_t diag_max;          /* a DTW round with at most this many candidates runs one
                                  wave per candidate along anti-diagonals instead of one
                                  lane per candidate (bands r <= 1023; 0 = never; 16384).
                                  Bands 112 <= r <= 1023 always run one wave per candidate;
                                  wider bands run one lane per candidate with its rows in
                                  global memory */
    int32_t band_lanes;        /* dtws_dtw_band: 0 = automatic (default: one wave per
                                  candidate for r <= 1023 when count <= diag_max or r >= 112,
                                  else one lane), 1 = one lane per candidate, 64 = one wave
                                  per candidate (r <= 1023) */
    int32_t stats_prefix;      /* batched search, window statistics: 0 = per-length arrays
                                  when the batch has few distinct lengths (default), 1 =
                                  always from the blocked prefix of the series */
    int32_t data_envelope;     /* batched search: 1 = the cascade's data-envelope bound
                                  (default), 0 = skip it (no envelope pass) */
    int32_t rounds;            /* batched search: bound-cascade / DTW rounds over the work
                                  queue, per query 64K, 1M, 16M candidates then the rest (4,
                                  default), 1M then the rest (2), or all at once (1) */
    int32_t list_cap;          /* capacity of the near-best list and of the batched survivor
                                  list: 0 = full size (default), else 64 .. 2^20 entries.  A list
                                  that overflows is recovered (see dtws_search), so this only
                                  changes speed; small values exist to exercise that path */
    int32_t lb_tile;           /* batched search: 1 = the rounds in which every query visits the
                                  same candidates (series order, or a single round) run the tiled
                                  cascade, one LDS-staged series tile shared by all queries
                                  (default); 0 = per-query work items */
    int32_t dtw_bound;         /* search DTW on one lane per candidate, bands of 97 to 223 cells:
                                  1 = every 16 columns the abandoning test adds the LB_Keogh
                                  terms of the columns still to come (query envelope, computed
                                  per candidate before its DTW; default), 0 = the band minimum
                                  alone */
    int32_t dtw_rows;          /* batched search DTW on one lane per candidate, bands of 49 cells
                                  and more: 1 = each wave works through a chunk of survivors as
                                  four rows of 16 lanes, a row taking the next 16 candidates as
                                  soon as all of its own have ended (default); 0 = a wave takes
                                  64 candidates and runs until the last of them ends */
    int32_t dtw_evict;         /* with dtw_rows = 1, bands of 49 to 223 cells: 1..15 = at a test, a
                                  row with at most this many live candidates (and two tests or
                                  more to go) moves them out, band column and all, and takes new
                                  ones; moved candidates resume later in full rows of 16 that
                                  share query and column, up to three times (default 4); 0 = off.
                                  The matches do not depend on it */
} dtws_schedule;

DTWS_API int dtws_get_schedule(dtws_ctx *ctx, dtws_schedule *out_host);
/* DTWS_EINVAL (nothing changed) when a field is outside the ranges above. */
DTWS_API int dtws_set_schedule(dtws_ctx *ctx, const dtws_schedule *s_host);

/* Autotuner: runs dtws_search_batch on the given batch (arguments as there;
 * DTWS_PROFILE is ignored) under candidate schedules, by coordinate descent over
 * diag_max, block, lb_blocks_per_cu, dtw_blocks_per_cu, stats_prefix,
 * data_envelope, rounds, lb_tile, dtw_bound, dtw_rows and dtw_evict starting from the
 * current schedule, then once more over data_envelope, rounds and lb_tile; each
 * candidate is called once untimed (graph capture) and then `reps` times
 * (1..100) timed on the host clock.  All candidates must return identical
 * matches (DTWS_EHIP otherwise, schedule unchanged).  Installs the fastest, writes
 * it to *best_host and its mean time per call (ms) to *best_ms_host.  Blocking. */
DTWS_API int dtws_autotune_batch(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_packed_dev,
                                 const int64_t *q_offsets_host, const int32_t *m_host, const int32_t *r_host,
                                 int32_t nq, uint32_t flags, uint64_t seed, void *stream, int32_t reps,
                                 dtws_schedule *best_host, double *best_ms_host);

/* ------------------------------------------------- learned block ordering
 * Not part of the paper's method: a network scores blocks of candidates so that
 * DTWS_ORDER_LEARNED visits the most promising blocks first; the bounds and the
 * exact DTW still decide, so results equal those of the natural order.
 * Model: y = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 + log(d(x) / 16 + 1e-4),
 * x = (16-segment PAA of the normalised query, 16-segment PAA of the normalised
 * candidate), segment t of a length-m window = positions [floor(t m / 16),
 * floor((t+1) m / 16)), d(x) = sum_t (x_t - x_{t+16})^2 (FP32) the squared PAA
 * distance: the network learns a correction to the logarithm of the PAA distance,
 * trained on y* = log(DTW / m + 1e-4) (dtws_model_train below, or the caller's own recipe through
 * dtws_model_train_step).  Products in bfloat16 on the matrix cores
 * with FP32 accumulation; FP32 master parameters; Adam (beta 0.9 / 0.999,
 * eps 1e-8).  Parameters: one flat FP32 vector of DTWS_MODEL_PARAMS values in
 * the order W1 (32 x 256, row = input), b1 (256), W2 (256 x 256, row = layer-1
 * unit), b2 (256), w3 (256), b3 (1). */
#define DTWS_MODEL_PARAMS 74497
#define DTWS_MODEL_MAX_ROWS 65536   /* rows per dtws_model_grad / dtws_model_train_step */

/* He-normal initialisation of the hidden layers from a seed (counter-based; deterministic), zero
 * biases and a zero output layer (w3, b3): the initial model orders exactly by its PAA-distance
 * term. */
DTWS_API int dtws_model_init(dtws_ctx *ctx, uint64_t seed);

/* Copy the FP32 parameters out of / into the context (count = DTWS_MODEL_PARAMS).
 * Setting resets the Adam state.  Blocking. */
DTWS_API int dtws_model_get(dtws_ctx *ctx, float *params_host, int64_t count);
DTWS_API int dtws_model_set(dtws_ctx *ctx, const float *params_host, int64_t count);

/* Predictions y_dev[rows] for feature rows X_dev[rows][32] (FP32, row-major; X_dev
 * 16-byte aligned, as every torch or hipMalloc allocation is: DTWS_EINVAL otherwise). */
DTWS_API int dtws_model_forward(dtws_ctx *ctx, const float *X_dev, int64_t rows, float *y_dev, void *stream);

/* Gradient of the mean squared error against targets t_dev[rows] (rows <=
 * DTWS_MODEL_MAX_ROWS) into grad_dev[DTWS_MODEL_PARAMS]; the loss to *loss_host
 * when not NULL (blocking then). */
DTWS_API int dtws_model_grad(dtws_ctx *ctx, const float *X_dev, const float *t_dev, int64_t rows, float *grad_dev,
                             float *loss_host, void *stream);

/* One Adam step with learning rate lr on a batch of rows (<= DTWS_MODEL_MAX_ROWS). */
DTWS_API int dtws_model_train_step(dtws_ctx *ctx, const float *X_dev, const float *t_dev, int64_t rows, float lr,
                                   float *loss_host, void *stream);

/* Training recipe of dtws_model_train.  Queries are drawn from the training series, shape by shape
 * (query length m[k], band r[k] of the labels, k < shapes): of every four queries three are cuts of
 * the series at a seeded start plus Gaussian noise of standard deviation noise_std x (0.5, 1, 2) in
 * turn, one an independent random walk.  A query's candidates are its proposals over the whole
 * series (the rows the learned order scores, for the context's current block), random_per_query
 * uniform starts, and for a cut query near_per_query starts within +-m/4 of its source and
 * near_per_query within +-2 proposal strides of it.  Each pair's label is its exact banded DTW
 * distance d from this library's DTW kernels; the target is log(d / m + 1e-4).  Every epoch visits
 * the pairs in a seeded order, batch rows per Adam step (a last partial batch is skipped), with the
 * learning rate falling linearly from lr to lr_final over the epochs. */
#define DTWS_TRAIN_MAX_SHAPES 8
typedef struct {
    int32_t shapes;                      /* 1 .. DTWS_TRAIN_MAX_SHAPES                         */
    int32_t m[DTWS_TRAIN_MAX_SHAPES];    /* query lengths (2 .. max_m, < n)                    */
    int32_t r[DTWS_TRAIN_MAX_SHAPES];    /* bands (>= 0; clamped to m - 1)                     */
    int32_t queries_per_shape;           /* >= 1                                               */
    int32_t random_per_query;            /* >= 0                                               */
    int32_t near_per_query;              /* >= 0                                               */
    int32_t epochs;                      /* >= 0 (0: build the pairs only)                     */
    int32_t batch;                       /* rows per Adam step, 64 .. DTWS_MODEL_MAX_ROWS      */
    int32_t init;                        /* 1: fresh initialisation from seed; 0: continue     */
    float lr, lr_final;                  /* > 0                                                */
    float noise_std;                     /* >= 0                                               */
    int32_t reserved;                    /* 0                                                  */
    uint64_t seed;
} dtws_train_cfg;

/* Trains the ordering network on pairs drawn from the training series Ttrain_dev[n] (device,
 * n <= max_n) as described above; everything runs on the device in this library's kernels.  The
 * model records the context's current work-item block: the learned order then uses that block,
 * whatever the schedule says, so training and search see the same proposals (set the block with
 * dtws_set_schedule before training).  loss_curve_host[epochs] (may be NULL) receives each epoch's
 * mean batch loss, *pairs_host (may be NULL) the number of pairs.  Allocates its pair buffers
 * (about 132 bytes per pair) for the duration of the call.  Blocking.  DTWS_EINVAL for a recipe
 * outside the ranges above or fewer pairs than one batch; DTWS_ENOMODEL for init = 0 without a
 * model. */
DTWS_API int dtws_model_train(dtws_ctx *ctx, const float *Ttrain_dev, int64_t n, const dtws_train_cfg *cfg,
                              void *stream, float *loss_curve_host, int64_t *pairs_host);

/* Serialised model: a 64-byte header (magic "DTWSMLP1", the parameter count, the work-item block it
 * was trained with, the FNV-1a 64-bit hash of the parameters) followed by the FP32 parameters.
 * dtws_model_save with buf_host NULL writes the size needed to *bytes_inout; otherwise *bytes_inout
 * must be at least that size and receives it.  dtws_model_load checks size, magic, count and hash
 * (DTWS_EINVAL on any mismatch, nothing changed) and resets the Adam state. */
DTWS_API int dtws_model_save(dtws_ctx *ctx, void *buf_host, size_t *bytes_inout);
DTWS_API int dtws_model_load(dtws_ctx *ctx, const void *buf_host, size_t bytes);

/* Proposals that the learned order scores (DTWS_ORDER_LEARNED).  The candidates
 * 0 .. n-m are cut into quarter blocks of block/4 starts (block: the one the model
 * was trained with, else the schedule's); the
 * proposal of a quarter is its start whose 16-segment PAA is nearest (squared
 * Euclidean, FP32, lowest start on ties) to the query's, among every ps-th start
 * of the quarter, ps = max(1, m/64) for m >= 128 and 1 below.  Row k (quarter k)
 * gets starts_dev[k] (-1 for a quarter past the last candidate) and X_dev[k][32] =
 * (query PAA, candidate PAA), the network's input.  rows = 4 * ceil((n-m+1) /
 * block) is written to *rows_out; with starts_dev and X_dev both NULL nothing else
 * happens, else max_rows must be >= rows (DTWS_EINVAL otherwise).  Uses the
 * context's workspace (calls on one context must not overlap); blocking. */
DTWS_API int dtws_propose(dtws_ctx *ctx, const float *T_dev, int64_t n, const float *Q_dev, int32_t m,
                          int64_t *starts_dev, float *X_dev, int64_t max_rows, int64_t *rows_out, void *stream);

/* 16-segment PAA of the z-normalised windows T[s .. s+m) for s in starts_dev[count]
 * into out_dev[count][16] (FP32; NaN rows for starts outside [0, n-m]). */
DTWS_API int dtws_paa(dtws_ctx *ctx, const float *T_dev, int64_t n, int32_t m, const int64_t *starts_dev,
                      int64_t count, float *out_dev, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DTWS_H */
