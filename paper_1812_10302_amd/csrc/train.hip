// Training of the learned block ordering inside the library: pair generation, labels, targets,
// shuffling and the Adam epochs all run here, on the context's stream, in this library's kernels.
//
// The network only orders work (the bounds and the exact DTW decide every result), so its training
// recipe is this library's own, not the paper's.  Pairs come from a training series T:
//   * queries: of every four, three are cuts of T at a seeded start plus Gaussian noise of standard
//     deviation noise_std x (0.5, 1, 2) in turn, and one is an independent random walk (cumulative
//     sum of N(0, 1) steps);
//   * candidates of a query: its proposals over all of T (the PAA-nearest start of every quarter
//     block, exactly the rows the learned order scores at search time, with the block the search will
//     use), `random` uniform starts, and for a cut query `near` starts within +-m/4 of its source and
//     `near` within +-2 proposal strides of it;
//   * features: the query's 16-segment PAA and the candidate's; label: the exact banded DTW distance
//     d (this library's DTW kernels, no abandoning), target log(d / m + 1e-4).
// Rows of empty quarters (past the last candidate) are dropped by an order-preserving compaction, so
// the pair set is a deterministic function of (T, configuration, seed).  Every epoch visits the rows
// in the order k -> (A k + C) mod rows with a seeded A coprime to rows, in batches of `batch` rows
// (a last partial batch is skipped), each batch one Adam step; the learning rate falls linearly from
// lr to lr_final over the epochs.
#include <math.h>
#include <string.h>

#include <vector>

#include "dtws_internal.h"

namespace dtws {
namespace {

constexpr double kTargetEps = 1e-4;

__host__ __device__ inline uint64_t tmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Draw number `i` of stream (seed, q, kind): a 64-bit counter-based value.
__host__ __device__ inline uint64_t draw(uint64_t seed, uint64_t q, uint64_t kind, uint64_t i) {
    return tmix(tmix(tmix(seed ^ 0xD1B54A32D192ED03ull) ^ (q * 0x9E3779B97F4A7C15ull + kind)) + i);
}

__device__ inline double unit_open(uint64_t h) {   // (0, 1]
    return ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

// Standard normal from two draws (Box-Muller).
__device__ inline double normal_of(uint64_t seed, uint64_t q, uint64_t kind, uint64_t i) {
    const double u1 = unit_open(draw(seed, q, kind, 2 * i)), u2 = unit_open(draw(seed, q, kind, 2 * i + 1));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Query q: a noisy cut of T at src (src >= 0) or an independent random walk (src < 0).
__global__ void k_train_query(const float *T, int m, int64_t src, double noise, uint64_t seed, uint64_t q,
                              float *Q) {
    if (src >= 0) {
        for (int j = threadIdx.x; j < m; j += blockDim.x)
            Q[j] = (float)((double)T[src + j] + noise * normal_of(seed, q, 1, (uint64_t)j));
        return;
    }
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int j = 0; j < m; ++j) {
        acc += normal_of(seed, q, 2, (uint64_t)j);
        Q[j] = (float)acc;
    }
}

// Extra candidates of query q: `random` uniform starts in [0, N), then for a cut query `near`
// within +-m/4 of src and `near` within +-2 strides of it, clipped to [0, N).
__global__ void k_train_extras(int64_t N, int m, int64_t src, int random, int near, uint64_t seed, uint64_t q,
                               int64_t *starts) {
    const int count = random + (src >= 0 ? 2 * near : 0);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const uint64_t h = draw(seed, q, 3, (uint64_t)k);
    int64_t s;
    if (k < random) {
        s = (int64_t)(h % (uint64_t)N);
    } else {
        const int64_t half = k < random + near ? m / 4 : 2 * (m >= 128 ? m / 64 : 1);
        s = src + (int64_t)(h % (uint64_t)(2 * half + 1)) - half;
        s = s < 0 ? 0 : (s > N - 1 ? N - 1 : s);
    }
    starts[k] = s;
}

// Feature rows of the extra candidates: the query's PAA, then the candidate's (PAA written by
// k_paa into cpaa[count][16]).
__global__ void k_train_extra_rows(const float *qpaa, const float *cpaa, int count, float *X) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count * 32) return;
    const int row = k >> 5, col = k & 31;
    X[(int64_t)row * 32 + col] = col < 16 ? qpaa[col] : cpaa[(int64_t)row * 16 + col - 16];
}

// Appends the valid rows (start >= 0 and a finite distance) of one query, in order, after the rows
// already held (*total); targets log(d / m + 1e-4).  One workgroup: block-wide scans over 1024-row
// chunks keep the order.
__global__ __launch_bounds__(1024) void k_train_append(const float *Xq, const int64_t *starts, const float *d,
                                                       int64_t count, int m, float *X, float *Y, int64_t *total) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t base_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) base_s = *total;
    __syncthreads();
    for (int64_t c0 = 0; c0 < count; c0 += 1024) {
        const int64_t k = c0 + tid;
        const bool ok = k < count && starts[k] >= 0 && isfinite(d[k]);
        const uint64_t mask = __ballot(ok);
        const int64_t before = __popcll(mask & (lane ? (~0ull >> (64 - lane)) : 0ull));
        if (lane == 0) wsum[wid] = __popcll(mask);
        __syncthreads();
        int64_t off = base_s;
        for (int w = 0; w < wid; ++w) off += wsum[w];
        int64_t tot = 0;
        for (int w = 0; w < 16; ++w) tot += wsum[w];
        if (ok) {
            const int64_t pos = off + before;
            for (int c = 0; c < 32; ++c) X[pos * 32 + c] = Xq[k * 32 + c];
            Y[pos] = (float)log((double)d[k] / m + kTargetEps);
        }
        __syncthreads();
        if (tid == 0) base_s += tot;
        __syncthreads();
    }
    if (tid == 0) *total = base_s;
}

// Batch b of an epoch: rows (A k + C) mod rows for k in [b0, b0 + batch).
__global__ void k_train_gather(const float *X, const float *Y, int64_t rows, uint64_t A, uint64_t C, int64_t b0,
                               int batch, float *Xb, float *Yb) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)batch * 32) return;
    const int64_t j = k >> 5;
    const int64_t row = (int64_t)((A * (uint64_t)(b0 + j) + C) % (uint64_t)rows);
    Xb[k] = X[row * 32 + (k & 31)];
    if ((k & 31) == 0) Yb[j] = Y[row];
}

__global__ void k_train_loss_add(const float *loss, double *sum) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *sum += (double)*loss;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) { return hipMalloc((void **)&p, sizeof(T) * (count ? count : 1)); }
};

#define TCHK(expr)                                 \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) {                    \
            set_hip_error(c, e_, #expr);           \
            return DTWS_EHIP;                      \
        }                                          \
    } while (0)

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// FNV-1a (64-bit) over a byte range: the content hash of saved parameters.
uint64_t fnv1a64(const void *p, size_t bytes) {
    const uint8_t *b = (const uint8_t *)p;
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace dtws

using namespace dtws;

namespace {
struct ModelHeader {
    char magic[8];        // "DTWSMLP1"
    uint32_t params;      // DTWS_MODEL_PARAMS
    uint32_t reserved0;
    int64_t block;        // work-item block the model was trained with (0: not recorded)
    uint64_t hash;        // FNV-1a 64 of the FP32 parameters
    uint8_t pad[32];
};
static_assert(sizeof(ModelHeader) == 64, "model header is 64 bytes");
constexpr char kMagic[8] = {'D', 'T', 'W', 'S', 'M', 'L', 'P', '1'};
}  // namespace

extern "C" {

DTWS_API int dtws_model_train(dtws_ctx *c, const float *T, int64_t n, const dtws_train_cfg *cfg, void *stream,
                              float *loss_curve_host, int64_t *pairs_host) {
    if (!c || !T || !cfg) return DTWS_EINVAL;
    const int ns = cfg->shapes;
    if (ns < 1 || ns > DTWS_TRAIN_MAX_SHAPES || cfg->queries_per_shape < 1 || cfg->random_per_query < 0 ||
        cfg->near_per_query < 0 || cfg->epochs < 0 || cfg->batch < 64 || cfg->batch > DTWS_MODEL_MAX_ROWS ||
        !(cfg->lr > 0.0f) || !(cfg->lr_final > 0.0f) || !(cfg->noise_std >= 0.0f) || n > c->max_n)
        return DTWS_EINVAL;
    for (int k = 0; k < ns; ++k)
        if (cfg->m[k] < 2 || cfg->m[k] > c->max_m || n < cfg->m[k] + 1 || cfg->r[k] < 0) return DTWS_EINVAL;
    if (!cfg->init && !c->has_model) return DTWS_ENOMODEL;
    TCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (cfg->init) {
        TCHK(mlp_init(c->mlp, cfg->seed, s));
        c->has_model = true;
        c->model_step = 0;
        c->model_block = c->block > 0 ? c->block : 4096;
    }
    // rows per shape (upper bound) and buffers
    int64_t max_rows = 0, max_q_rows = 0, max_extra = 0;
    for (int k = 0; k < ns; ++k) {
        const int64_t pr = propose_rows(c, n, cfg->m[k]);
        const int64_t ex = (int64_t)cfg->random_per_query + 2 * (int64_t)cfg->near_per_query;
        max_rows += (int64_t)cfg->queries_per_shape * (pr + ex);
        max_q_rows = pr + ex > max_q_rows ? pr + ex : max_q_rows;
        max_extra = ex > max_extra ? ex : max_extra;
    }
    DevBuf<float> X, Y, Xq, dq, cpaa, Qb, Xb, Yb;
    DevBuf<int64_t> starts, total;
    DevBuf<double> lsum;
    TCHK(X.alloc((size_t)max_rows * 32));
    TCHK(Y.alloc((size_t)max_rows));
    TCHK(Xq.alloc((size_t)max_q_rows * 32));
    TCHK(dq.alloc((size_t)max_q_rows));
    TCHK(starts.alloc((size_t)max_q_rows));
    TCHK(cpaa.alloc((size_t)max_extra * 16));
    TCHK(Qb.alloc((size_t)c->max_m));
    TCHK(Xb.alloc((size_t)cfg->batch * 32));
    TCHK(Yb.alloc((size_t)cfg->batch));
    TCHK(total.alloc(1));
    TCHK(lsum.alloc(1));
    TCHK(hipMemsetAsync(total.p, 0, sizeof(int64_t), s));

    const QueryBufs qb = query_bufs_of(c, 0);
    uint64_t qglobal = 0;
    for (int k = 0; k < ns; ++k) {
        const int m = cfg->m[k], r = cfg->r[k] > cfg->m[k] - 1 ? cfg->m[k] - 1 : cfg->r[k];
        const int64_t N = n - m + 1;
        const int64_t pr = propose_rows(c, n, m);
        for (int qq = 0; qq < cfg->queries_per_shape; ++qq, ++qglobal) {
            const uint64_t q = qglobal;
            const bool walk = qq % 4 == 3;
            // the cut's source: uniform in [0, n - m)
            const int64_t src = walk ? -1 : (int64_t)(draw(cfg->seed, q, 0, 0) % (uint64_t)(n - m));
            const double noise = (double)cfg->noise_std * (qq % 3 == 0 ? 0.5 : (qq % 3 == 1 ? 1.0 : 2.0));
            hipLaunchKernelGGL(k_train_query, dim3(1), dim3(256), 0, s, T, m, src, noise, cfg->seed, q, Qb.p);
            TCHK(hipGetLastError());
            TCHK(launch_query_prep(Qb.p, m, r, qb, s));
            // proposals (rows [0, pr)), then the extra candidates
            const int rc = enqueue_propose(c, T, n, m, starts.p, Xq.p, s);
            if (rc != DTWS_OK) return rc;
            const int ex = cfg->random_per_query + (walk ? 0 : 2 * cfg->near_per_query);
            if (ex > 0) {
                hipLaunchKernelGGL(k_train_extras, dim3(nb256(ex)), dim3(256), 0, s, N, m, src, cfg->random_per_query,
                                   cfg->near_per_query, cfg->seed, q, starts.p + pr);
                TCHK(hipGetLastError());
                TCHK(launch_paa(T, n, m, starts.p + pr, ex, cpaa.p, s));
                hipLaunchKernelGGL(k_train_extra_rows, dim3(nb256((int64_t)ex * 32)), dim3(256), 0, s, c->qpaa, cpaa.p,
                                   ex, Xq.p + pr * 32);
                TCHK(hipGetLastError());
            }
            // labels: exact banded DTW of every candidate (NaN for an empty quarter's start -1)
            DtwArgs d{};
            d.T = T;
            d.m = m;
            d.r = r;
            d.w = 2 * r + 1;
            d.qpad = qb.qpad;
            d.starts64 = starts.p;
            d.count = pr + ex;
            d.n = n;
            d.single = -1;
            d.abandon_at = INFINITY;
            d.nb_cap = kNearBestCap;
            d.dist_out = dq.p;
            if (r <= kDiagMaxBand && 2 * r + 1 > 16 * kMaxChunks) {
                const int64_t blocks = (d.count + 1) / 2;
                TCHK(launch_dtw_diag_list(d, false, (int)(blocks < c->num_cu * 8 ? blocks : c->num_cu * 8), s));
            } else {
                TCHK(launch_dtw(d, false, d.count, c->num_cu, c->gen_rows, c->gen_lanes, s));
            }
            hipLaunchKernelGGL(k_train_append, dim3(1), dim3(1024), 0, s, Xq.p, starts.p, dq.p, pr + ex, m, X.p, Y.p,
                               total.p);
            TCHK(hipGetLastError());
        }
        // the proposal staging of the next shape differs: let this shape's copies complete
        TCHK(hipStreamSynchronize(s));
    }
    int64_t rows = 0;
    TCHK(hipMemcpyAsync(&rows, total.p, sizeof(rows), hipMemcpyDeviceToHost, s));
    TCHK(hipStreamSynchronize(s));
    if (pairs_host) *pairs_host = rows;
    const int64_t steps = rows / cfg->batch;
    if (steps < 1 && cfg->epochs > 0) return DTWS_EINVAL;   // fewer pairs than one batch
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        const float lr = cfg->epochs > 1 ? cfg->lr + (cfg->lr_final - cfg->lr) * ((float)ep / (float)(cfg->epochs - 1))
                                         : cfg->lr;
        uint64_t A = 1 + draw(cfg->seed, 0xE90C11ull, 4, (uint64_t)ep) % (uint64_t)(rows > 1 ? rows - 1 : 1);
        while (rows > 1 && gcd_u64(A, (uint64_t)rows) != 1) A = A + 1 < (uint64_t)rows ? A + 1 : 1;
        const uint64_t C = draw(cfg->seed, 0xE90C11ull, 5, (uint64_t)ep) % (uint64_t)rows;
        TCHK(hipMemsetAsync(lsum.p, 0, sizeof(double), s));
        for (int64_t b = 0; b < steps; ++b) {
            hipLaunchKernelGGL(k_train_gather, dim3(nb256((int64_t)cfg->batch * 32)), dim3(256), 0, s, X.p, Y.p, rows,
                               A, C, b * cfg->batch, cfg->batch, Xb.p, Yb.p);
            TCHK(hipGetLastError());
            TCHK(mlp_backward(c->mlp, Xb.p, Yb.p, cfg->batch, s));
            TCHK(mlp_adam(c->mlp, ++c->model_step, lr, s));
            hipLaunchKernelGGL(k_train_loss_add, dim3(1), dim3(64), 0, s, c->mlp.loss, lsum.p);
            TCHK(hipGetLastError());
        }
        double sum = 0.0;
        TCHK(hipMemcpyAsync(&sum, lsum.p, sizeof(sum), hipMemcpyDeviceToHost, s));
        TCHK(hipStreamSynchronize(s));
        if (loss_curve_host) loss_curve_host[ep] = (float)(sum / (double)steps);
    }
    TCHK(hipStreamSynchronize(s));
    return DTWS_OK;
}

DTWS_API int dtws_model_save(dtws_ctx *c, void *buf_host, size_t *bytes_inout) {
    if (!c || !bytes_inout) return DTWS_EINVAL;
    const size_t need = sizeof(ModelHeader) + sizeof(float) * (size_t)kModelParams;
    if (!buf_host) {
        *bytes_inout = need;
        return DTWS_OK;
    }
    if (*bytes_inout < need) return DTWS_EINVAL;
    if (!c->has_model) return DTWS_ENOMODEL;
    TCHK(hipSetDevice(c->device));
    float *params = (float *)((uint8_t *)buf_host + sizeof(ModelHeader));
    TCHK(hipMemcpy(params, c->mlp.theta, sizeof(float) * kModelParams, hipMemcpyDeviceToHost));
    ModelHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kMagic, 8);
    h.params = (uint32_t)kModelParams;
    h.block = c->model_block;
    h.hash = fnv1a64(params, sizeof(float) * kModelParams);
    memcpy(buf_host, &h, sizeof(h));
    *bytes_inout = need;
    return DTWS_OK;
}

DTWS_API int dtws_model_load(dtws_ctx *c, const void *buf_host, size_t bytes) {
    const size_t need = sizeof(ModelHeader) + sizeof(float) * (size_t)kModelParams;
    if (!c || !buf_host || bytes != need) return DTWS_EINVAL;
    ModelHeader h;
    memcpy(&h, buf_host, sizeof(h));
    const float *params = (const float *)((const uint8_t *)buf_host + sizeof(ModelHeader));
    if (memcmp(h.magic, kMagic, 8) != 0 || h.params != (uint32_t)kModelParams ||
        h.hash != fnv1a64(params, sizeof(float) * kModelParams) || h.block < 0)
        return DTWS_EINVAL;
    const int rc = dtws_model_set(c, params, kModelParams);
    if (rc != DTWS_OK) return rc;
    c->model_block = h.block;
    return DTWS_OK;
}

}  // extern "C"
