// Learned block ordering: a small network that predicts log1p(DTW / m) of a candidate from the
// 16-segment PAA of the normalised query and of the normalised candidate.  It is not part of the
// paper's method and never decides a result: its scores only order the work items, the exact
// lower bounds and the exact DTW still prune and decide.
//
// Network 32 -> 256 -> 256 -> 1 with ReLU; products in bfloat16 on the matrix cores with FP32
// accumulation (v_mfma_f32_16x16x32_bf16), FP32 master parameters, Adam in FP32.
// Parameters are one flat FP32 vector: W1 (32 x 256, row = input), b1, W2 (256 x 256, row =
// layer-1 unit), b2, w3 (256), b3.  bfloat16 copies: W1T (256 x 32), W2T (256 x 256, row = layer-2
// unit) for the forward products and W2 (row-major) for the backward product.
//
// Rounding points (the CPU reference rounds at the same places): the inputs, W1, W2, the layer-1
// activations, and the back-propagated pre-activation gradients before they enter a product.
#include "device.h"

namespace dtws {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16 bits, round to nearest, ties to even.
__device__ inline uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ BF16 GEMM on the matrix cores
// C[M x N] (FP32, row stride ldc) = A[M x K] * B[K x N], with A row-major (row stride lda, K
// contiguous) and B given transposed, BT[N x K] row-major (row stride ldb).  M % 16 == 0,
// N % 64 == 0, K % 32 == 0, strides multiples of 8.  One wave per 16 x 64 output tile.
// Operand layout of v_mfma_f32_16x16x32_bf16 (16 x 32 by 32 x 16): lane l supplies A row l % 16
// and B column l % 16, each with k = 8 * (l / 16) .. + 7; the accumulator lane l holds column
// l % 16, rows 4 * (l / 16) .. + 3.
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ A, int64_t lda,
                                                    const uint16_t *__restrict__ BT, int64_t ldb,
                                                    float *__restrict__ C, int64_t ldc, int M, int N, int K) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t tiles_m = M / 16, tiles = tiles_m * (N / 64);
    if (wave >= tiles) return;
    const int64_t tm = wave % tiles_m, tn = wave / tiles_m;
    const int r = lane & 15, kq = 8 * (lane >> 4);
    f32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *arow = A + (tm * 16 + r) * lda + kq;
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = *(const bf16x8 *)(arow + k0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bf16x8 b = *(const bf16x8 *)(BT + (tn * 64 + 16 * c + r) * ldb + k0 + kq);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int t = 0; t < 4; ++t) C[(tm * 16 + 4 * (lane >> 4) + t) * ldc + tn * 64 + 16 * c + r] = acc[c][t];
}

// ------------------------------------------------------------------ fused inference
// Forward pass without the intermediate arrays, for scoring.  Both layers are computed transposed
// (units x data rows, 16 data rows per wave and tile), so the layer-1 accumulators are already in
// the lane layout of the layer-2 B operand: lane l holds data row l % 16 and units
// 16 u + 4 (l / 16) .. + 3 of tile u.  Layer 2 takes its 32 hidden units of step s in the order
// "units 32 s + 4 g .. + 3, then 32 s + 16 + 4 g .. + 3 for lane group g", the A operand (W2T rows)
// follows the same order, and the head (ReLU, dot with w3, + b3) is folded into the layer-2
// epilogue.  Rounding points are those of the unfused path: X, W1, W2 and the layer-1 activations
// in bfloat16, FP32 accumulation.  W2T (rows padded to kInferW2Stride to spread the LDS banks),
// W1T, b1, b2 and w3 are staged once per workgroup; workgroups loop over the row tiles.
constexpr int kInferW2Stride = 264;   // bfloat16 per staged W2T row
constexpr int kInferThreads = 512;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kInferThreads) void k_mlp_infer(const float *__restrict__ X, int64_t R,
                                                             const uint16_t *__restrict__ W1T,
                                                             const float *__restrict__ b1,
                                                             const uint16_t *__restrict__ W2T,
                                                             const float *__restrict__ b2,
                                                             const float *__restrict__ w3,
                                                             const float *__restrict__ b3, float *__restrict__ y) {
    __shared__ uint16_t sW2[256 * kInferW2Stride];
    __shared__ uint16_t sW1[256 * 32];
    __shared__ float sB1[256], sB2[256], sW3[256];
    for (int e = threadIdx.x; e < 256 * 256 / 8; e += blockDim.x) {
        const int n = e / 32, h8 = e % 32;
        *(uint4 *)(sW2 + n * kInferW2Stride + 8 * h8) = ((const uint4 *)W2T)[e];
    }
    for (int e = threadIdx.x; e < 256 * 32 / 8; e += blockDim.x) ((uint4 *)sW1)[e] = ((const uint4 *)W1T)[e];
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        sB1[e] = b1[e];
        sB2[e] = b2[e];
        sW3[e] = w3[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t tiles = (R + 15) / 16;
    const float bias3 = b3[0];
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t row = tile * 16 + r;
        // layer-1 B operand: features 8 g .. + 7 of this lane's data row (zero past the last row)
        float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0;
        if (row < R) {
            f0 = *(const float4 *)(X + row * 32 + 8 * g);
            f1 = *(const float4 *)(X + row * 32 + 8 * g + 4);
        }
        const u32x4 xw = u32x4{(uint32_t)f2bf(f0.x) | ((uint32_t)f2bf(f0.y) << 16), (uint32_t)f2bf(f0.z) | ((uint32_t)f2bf(f0.w) << 16),
                               (uint32_t)f2bf(f1.x) | ((uint32_t)f2bf(f1.y) << 16), (uint32_t)f2bf(f1.z) | ((uint32_t)f2bf(f1.w) << 16)};
        const bf16x8 xb = __builtin_bit_cast(bf16x8, xw);
        // the PAA-distance term (FP32 features): the lane of group g ^ 2 holds the other half of
        // the same 8 segments; the two query-half groups together cover all 16
        float dd = 0.0f;
        {
            const float p[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float e = p[k] - __shfl_xor(p[k], 32, 64);
                dd = fmaf(e, e, dd);
            }
            dd += __shfl_xor(dd, 16, 64);
        }
        // layer 1 and its epilogue, packed as the layer-2 B operands of the 8 K steps
        bf16x8 hb[8];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            uint32_t hw[4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int u = 2 * s8 + h;
                const bf16x8 a = *(const bf16x8 *)(sW1 + (16 * u + r) * 32 + 8 * g);
                const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xb, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                const float4 bb = *(const float4 *)(sB1 + 16 * u + 4 * g);
                hw[2 * h] = (uint32_t)f2bf(fmaxf(acc[0] + bb.x, 0.0f)) | ((uint32_t)f2bf(fmaxf(acc[1] + bb.y, 0.0f)) << 16);
                hw[2 * h + 1] = (uint32_t)f2bf(fmaxf(acc[2] + bb.z, 0.0f)) | ((uint32_t)f2bf(fmaxf(acc[3] + bb.w, 0.0f)) << 16);
            }
            hb[s8] = __builtin_bit_cast(bf16x8, u32x4{hw[0], hw[1], hw[2], hw[3]});
        }
        // layer 2 by tiles of 16 output units, head folded in
        float part = 0.0f;
#pragma unroll 2
        for (int v = 0; v < 16; ++v) {
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
            const uint16_t *wrow = sW2 + (16 * v + r) * kInferW2Stride + 4 * g;
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const uint2 lo = *(const uint2 *)(wrow + 32 * s8), hi = *(const uint2 *)(wrow + 32 * s8 + 16);
                const bf16x8 a = __builtin_bit_cast(bf16x8, u32x4{lo.x, lo.y, hi.x, hi.y});
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[s8], acc, 0, 0, 0);
            }
            const float4 bb = *(const float4 *)(sB2 + 16 * v + 4 * g), ww = *(const float4 *)(sW3 + 16 * v + 4 * g);
            part = fmaf(fmaxf(acc[0] + bb.x, 0.0f), ww.x, part);
            part = fmaf(fmaxf(acc[1] + bb.y, 0.0f), ww.y, part);
            part = fmaf(fmaxf(acc[2] + bb.z, 0.0f), ww.z, part);
            part = fmaf(fmaxf(acc[3] + bb.w, 0.0f), ww.w, part);
        }
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (g == 0 && row < R) y[row] = part + bias3 + logf(dd * (1.0f / 16.0f) + 1e-4f);
    }
}

// ------------------------------------------------------------------ elementwise pieces
// X (FP32 R x 32, rows >= R are zero padding) -> bfloat16 row-major and transposed (32 x Rp).
__global__ void k_mlp_x(const float *X, int64_t R, int64_t Rp, uint16_t *Xb, uint16_t *XbT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Rp * 32) return;
    const int64_t r = e / 32, k = e % 32;
    const uint16_t v = r < R ? f2bf(X[r * 32 + k]) : 0;
    Xb[e] = v;
    if (XbT) XbT[k * Rp + r] = v;
}

// Layer 1 epilogue: H1 = relu(C1 + b1) -> bfloat16 row-major (and transposed, for training).
__global__ void k_mlp_act1(const float *C1, const float *b1, int64_t Rp, uint16_t *H1b, uint16_t *H1T) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Rp * 256) return;
    const int64_t r = e / 256, n = e % 256;
    const float h = fmaxf(C1[e] + b1[n], 0.0f);
    const uint16_t v = f2bf(h);
    H1b[e] = v;
    if (H1T) H1T[n * Rp + r] = v;
}

// Layer 2 epilogue and head, one wave per row: H2 = relu(C2 + b2) (written back into C2 when
// training), y = H2 . w3 + b3 + log(d / 16 + 1e-4), d the squared distance of the row's two PAA
// halves (FP32 features X, rows >= Rx are padding without features).
__global__ void k_mlp_head(float *C2, const float *b2, const float *w3, const float *b3, int64_t R, float *y,
                           bool keep, const float *X, int64_t Rx) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= R) return;
    float dd = 0.0f;
    if (lane < 16 && row < Rx) {
        const float e = X[row * 32 + lane] - X[row * 32 + lane + 16];
        dd = e * e;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) dd += __shfl_xor(dd, off, 64);
    dd = __shfl(dd, 0, 64);
    float acc = 0.0f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int n = lane + 64 * u;
        const float h = fmaxf(C2[row * 256 + n] + b2[n], 0.0f);
        if (keep) C2[row * 256 + n] = h;
        acc = fmaf(h, w3[n], acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) y[row] = acc + b3[0] + logf(dd * (1.0f / 16.0f) + 1e-4f);
}

// Loss and output gradient: dy = 2 (y - t) / R (zero for padding rows), loss = mean (y - t)^2;
// dA2 = dy * w3 * [H2 > 0] -> bfloat16 row-major and transposed.
__global__ void k_mlp_bwd_head(const float *y, const float *t, const float *H2, const float *w3, int64_t R, int64_t Rp,
                               float *dy, uint16_t *dA2b, uint16_t *dA2T, float *loss) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Rp * 256) return;
    const int64_t r = e / 256, n = e % 256;
    const float d = r < R ? 2.0f * (y[r] - t[r]) / (float)R : 0.0f;
    if (n == 0) {
        dy[r] = d;
        if (r < R) atomicAdd(loss, (y[r] - t[r]) * (y[r] - t[r]) / (float)R);
    }
    const float g = r < R && H2[e] > 0.0f ? d * w3[n] : 0.0f;
    const uint16_t v = f2bf(g);
    dA2b[e] = v;
    dA2T[n * Rp + r] = v;
}

// dA1 = dH1 * [H1 > 0] -> bfloat16 transposed.
__global__ void k_mlp_bwd1(const float *dH1, const uint16_t *H1b, int64_t Rp, uint16_t *dA1T) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Rp * 256) return;
    const int64_t r = e / 256, n = e % 256;
    const float g = bf2f(H1b[e]) > 0.0f ? dH1[e] : 0.0f;
    dA1T[n * Rp + r] = f2bf(g);
}

// Column sums over the R rows for the bias gradients and the head weights (FP32, unrounded):
// db1[n] = sum dH1*[H1>0], db2[n] = sum dy*w3[n]*[H2>0], dw3[n] = sum dy*H2, db3 = sum dy.
// Two passes with a fixed summation order: kColsumGroups row groups into part, then part summed.
__global__ __launch_bounds__(256) void k_mlp_colsums_part(const float *dH1, const uint16_t *H1b, const float *H2,
                                                          const float *dy, const float *w3, int64_t R, float *part) {
    const int n = threadIdx.x, g = blockIdx.x;
    const int64_t r0 = R * g / kColsumGroups, r1 = R * (g + 1) / kColsumGroups;
    const float w = w3[n];
    float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t e = r * 256 + n;
        const float d = dy[r];
        if (bf2f(H1b[e]) > 0.0f) s1 += dH1[e];
        const float h2 = H2[e];
        if (h2 > 0.0f) s2 += d * w;
        s3 = fmaf(d, h2, s3);
        s4 += d;
    }
    float *p = part + (int64_t)g * 4 * 256;
    p[n] = s1;
    p[256 + n] = s2;
    p[512 + n] = s3;
    p[768 + n] = s4;
}

__global__ __launch_bounds__(256) void k_mlp_colsums(const float *part, float *g_b1, float *g_b2, float *g_w3,
                                                     float *g_b3) {
    const int n = threadIdx.x;
    float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
    for (int g = 0; g < kColsumGroups; ++g) {
        const float *p = part + (int64_t)g * 4 * 256;
        s1 += p[n];
        s2 += p[256 + n];
        s3 += p[512 + n];
        s4 += p[768 + n];
    }
    g_b1[n] = s1;
    g_b2[n] = s2;
    g_w3[n] = s3;
    if (n == 0) g_b3[0] = s4;
}

// Adam with bias correction on the FP32 master parameters.
__global__ void k_adam(float *theta, const float *g, float *m, float *v, int64_t count, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// bfloat16 copies of the weights: W1T[n][k] = W1[k][n], W2T[n][h] = W2[h][n], W2b = W2.
__global__ void k_mlp_refresh(const float *W1, const float *W2, uint16_t *W1T, uint16_t *W2T, uint16_t *W2b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 32 * 256) {
        const int64_t k = e / 256, n = e % 256;
        W1T[n * 32 + k] = f2bf(W1[e]);
    }
    if (e < 256 * 256) {
        const int64_t h = e / 256, n = e % 256;
        const uint16_t b = f2bf(W2[e]);
        W2T[n * 256 + h] = b;
        W2b[e] = b;
    }
}

// Counter-based He-normal initialisation of the hidden layers (Box-Muller on splitmix64 draws); zero
// biases and a zero output layer.
__device__ inline uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__global__ void k_mlp_init(float *theta, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int64_t oW1 = 0, ob1 = 32 * 256, oW2 = ob1 + 256, ob2 = oW2 + 65536, ow3 = ob2 + 256, ob3 = ow3 + 256;
    if (i > ob3) return;
    float scale = 0.0f;
    if (i < ob1) scale = sqrtf(2.0f / 32.0f);
    else if (i >= oW2 && i < ob2) scale = sqrtf(2.0f / 256.0f);
    // the output layer starts at zero: an untrained model orders by the PAA-distance term alone
    (void)oW1;
    const uint64_t h1 = mix64(seed ^ (uint64_t)(2 * i)), h2 = mix64(seed ^ (uint64_t)(2 * i + 1));
    const float u1 = ((h1 >> 40) + 1) * (1.0f / 16777217.0f), u2 = (h2 >> 40) * (1.0f / 16777216.0f);
    const float z = sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
    theta[i] = scale * z;
}

// ------------------------------------------------------------------ PAA features
// 16-segment PAA of the z-normalised window T[s .. s+m): segment t covers [floor(t m / 16),
// floor((t+1) m / 16)); mean and population sigma two-pass in FP64 (sigma <= 1e-8: all zero).
// One thread per window; out[k * 16 + t].
__device__ inline void paa16(const float *w, int m, float *out16) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += (double)w[j];
    const double mu = s / m;
    double v = 0.0;
    for (int j = 0; j < m; ++j) {
        const double d = (double)w[j] - mu;
        v += d * d;
    }
    const double sigma = sqrt(v / m);
    const double inv = sigma <= kSigmaFlat ? 0.0 : 1.0 / sigma;
    for (int t = 0; t < 16; ++t) {
        const int a = (t * m) / 16, b = ((t + 1) * m) / 16;
        double ss = 0.0;
        for (int j = a; j < b; ++j) ss += (double)w[j];
        out16[t] = (float)((ss / (b - a) - mu) * inv);
    }
}

__global__ void k_paa(const float *T, int64_t n, int m, const int64_t *starts, int64_t count, float *out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t s = starts[k];
    float f[16];
    if (s < 0 || s > n - m) {
        for (int t = 0; t < 16; ++t) out[k * 16 + t] = NAN;
        return;
    }
    paa16(T + s, m, f);
    for (int t = 0; t < 16; ++t) out[k * 16 + t] = f[t];
}

// ------------------------------------------------------------------ block scoring and order
// Query PAA from the FP64 normalised query: qpaa[q * 16 + t].
__global__ void k_query_paa(const BatchArgs a, float *qpaa) {
    const int q = blockIdx.x, t = threadIdx.x;
    if (t >= 16) return;
    const int m = a.bq[q].m;
    const double *x = a.qhat64 + (int64_t)q * a.max_m;
    const int lo = (t * m) / 16, hi = ((t + 1) * m) / 16;
    double s = 0.0;
    for (int j = lo; j < hi; ++j) s += x[j];
    qpaa[q * 16 + t] = (float)(s / (hi - lo));
}

// PAA of windows from the blocked prefix (see Prefix).  Windows are at most 2048 points, so they
// end in their first block or the next; every lookup is unconditional (the prefix has sentinels
// past its last block), so the loads of one window issue back to back.
struct PrefixView {
    Prefix pre;
    // 16-segment PAA of the z-normalised window T[i .. i+m) (segment t: [floor(t m/16),
    // floor((t+1) m/16)), inv_len[t] = 1 / its length, inv_m = 1 / m); all zero for a flat window.
    // Sums are FP64 differences of the prefix; the means and the scaling run in FP32.
    __device__ void paa(int64_t i, int m, double inv_m, const float (&inv_len)[16], float *out) const {
        const int64_t b0 = i / kPB, e0 = (b0 + 1) * kPB;
        const double delta = pre.anc[b0 + 1] - pre.anc[b0];
        const double2 t = pre.tot[b0];
        double2 p[17];
#pragma unroll
        for (int k = 0; k <= 16; ++k) p[k] = pre.at(i + ((k * m) >> 4));
        // sums relative to anc[b0] from the block start to x: P(x) in block b0, else the whole
        // block b0 plus P(x) re-anchored
        double g[17];
#pragma unroll
        for (int k = 0; k <= 16; ++k) {
            const int64_t x = i + ((k * m) >> 4);
            const double lx = (double)(x - e0);
            g[k] = x < e0 ? p[k].x : t.x + p[k].x + lx * delta;
        }
        const int64_t xe = i + m;
        const double lxe = (double)(xe - e0);
        const double g2 = xe < e0 ? p[16].y : t.y + p[16].y + 2.0 * delta * p[16].x + lxe * delta * delta;
        const double S1 = g[16] - g[0], S2 = g2 - p[0].y;
        const double md = S1 * inv_m, var = S2 * inv_m - md * md;
        const float inv = var > kSigmaFlat * kSigmaFlat ? rsqrtf((float)var) : 0.0f;
        const float mdf = (float)md;
#pragma unroll
        for (int k = 0; k < 16; ++k) out[k] = ((float)(g[k + 1] - g[k]) * inv_len[k] - mdf) * inv;
    }
    // Term t of the same PAA alone (the four prefix lookups it needs).
    __device__ float paa_term(int64_t i, int m, double inv_m, int t) const {
        const int64_t b0 = i / kPB, e0 = (b0 + 1) * kPB;
        const double delta = pre.anc[b0 + 1] - pre.anc[b0];
        const double2 tt = pre.tot[b0];
        const int64_t xs[4] = {i, i + ((t * m) >> 4), i + (((t + 1) * m) >> 4), i + m};
        double gx[4], gy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 p = pre.at(xs[k]);
            const double lx = (double)(xs[k] - e0);
            const bool cross = xs[k] >= e0;
            gx[k] = cross ? tt.x + p.x + lx * delta : p.x;
            gy[k] = cross ? tt.y + p.y + 2.0 * delta * p.x + lx * delta * delta : p.y;
        }
        const double md = (gx[3] - gx[0]) * inv_m, var = (gy[3] - gy[0]) * inv_m - md * md;
        const float inv = var > kSigmaFlat * kSigmaFlat ? rsqrtf((float)var) : 0.0f;
        const float len = (float)((((t + 1) * m) >> 4) - ((t * m) >> 4));
        return ((float)(gx[2] - gx[1]) / len - (float)md) * inv;
    }
};

// Minimum of a 64-bit value over the wave (every lane gets it).
__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// DPP move of an FP32 value; lanes without a source, and lanes of rows outside ROWS, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_or_zero(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

// Inclusive prefix sum over the 64 lanes of a wave (row shifts within each 16-lane row, then the
// row broadcasts of lanes 15 and 31 into the rows above them).
__device__ __forceinline__ float wave_scan_incl(float x) {
    x += dpp_or_zero<0x111, 0xF>(x);   // row_shr:1
    x += dpp_or_zero<0x112, 0xF>(x);   // row_shr:2
    x += dpp_or_zero<0x114, 0xF>(x);   // row_shr:4
    x += dpp_or_zero<0x118, 0xF>(x);   // row_shr:8
    x += dpp_or_zero<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_or_zero<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// Proposals: row (q, blk, j) covers the starts [blk * B + j * B / K, + B / K) of query q.  Every
// ps-th start of a row, ps = max(1, m / 64), is compared with the query by the squared Euclidean
// distance of the PAAs, and the nearest is kept (lowest start on ties).  Its features (query PAA,
// then candidate PAA) go to X and its start to sstart; an empty quarter gets start -1 and zero
// features.  One wave takes the K rows of a block: it walks the quarters in turn (the prefix grid
// of the fast path carries over from one quarter to the next when a quarter is a whole number of
// groups), keeps each quarter's winner in LDS, and computes the K feature rows together at the end.
// GRID selects the rows this instance serves: those of queries whose length is a multiple of 64
// (the grid path) or the others (general path); the two are separate instances so that each gets
// its own register allocation: five waves per SIMD for the grid path (the grid loads and LDS round
// trips of a group are latency-bound), no cap for the general path (17 prefix lookups per start).
template <bool GRID>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GRID ? 5 : 1))) void k_propose(const BatchArgs a, const ScoreArgs sa,
                                                                                       int64_t row0, int64_t R, float *X) {
    static_assert(kScoreSamples * 16 == 64, "one feature term per lane for all quarters of a block");
    __shared__ uint64_t winners[4][kScoreSamples];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // wave-uniform values are placed in scalar registers explicitly, so the walk below keeps its
    // positions and loop control on the scalar unit
    const int64_t k0 = uniform((((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * kScoreSamples);
    if (k0 >= R) return;
    const int64_t row = row0 + k0;   // rows of a block are consecutive and belong to one query
    int lo = 0, hi = a.nq;   // row_off[lo] <= row < row_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sa.row_off[mid] <= row) lo = mid;
        else hi = mid;
    }
    const int q = __builtin_amdgcn_readfirstlane(lo);
    const int64_t local = uniform(row - sa.row_off[q]);
    const BatchQ bq = a.bq[q];
    const int m = __builtin_amdgcn_readfirstlane(bq.m);
    const int64_t qN = uniform(bq.N);
    const int64_t quarter = a.block / kScoreSamples;
    const int64_t bfirst = (local / kScoreSamples) * a.block;
    float qp[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) qp[t] = sa.qpaa[q * 16 + t];
    const double inv_m = 1.0 / m;
    const PrefixView pv{sa.pre};
    const int64_t ps = m >= 128 ? m >> 6 : 1;
    if (((m & 63) == 0) != GRID) return;   // (wave-uniform) rows of the other instance
    if constexpr (GRID) {
        // m = 64 ps: the sampled starts and every segment boundary lie on the grid of step ps, so
        // the 64 starts of a group need the prefix at 128 grid points only (re-anchored to the
        // block of the group's first start).  Lane l holds grid points l and l + 64, the start and
        // end of its window; the segment sums (grid points 4 apart) go through LDS as FP32.
        __shared__ double gsh[4][128];
        __shared__ float dsh[4][128];
        double *gw = gsh[threadIdx.x >> 6];
        float *dw = dsh[threadIdx.x >> 6];
        const float inv_seg = 16.0f / (float)m;
        // a decimated copy with step ps when the prefix pass wrote one (ps a power of two)
        const int dl = __builtin_ctz((unsigned)ps);
        const bool use_dec = (ps & (ps - 1)) == 0 && dl >= kDecFirst && dl < kDecLevels && ((sa.dec_levels >> dl) & 1u);
        const double2 *dsrc = use_dec ? sa.dec.lv[dl] : nullptr;
        const int64_t nlast = use_dec ? ((a.n >> dl) << dl) : a.n;
        // raw prefix at grid point k of the current group (points past the series only serve idle
        // lanes); the upper half of one group's grid is the lower half of the next, and the
        // next group's upper half is loaded one group ahead
        auto grid_raw = [&](int64_t x) -> double2 {
            x = x < nlast ? x : nlast;
            return use_dec ? dsrc[x >> dl] : sa.pre.at(x);
        };
        // Short steps (ps <= 4) take the grid from the series itself, 4 bytes per point read
        // instead of a 16-byte prefix entry per grid point written and read again.  A group of 64
        // grid intervals is summed relative to its own first point a_g in FP32 (a wave scan of
        // small values), then shifted to the walk's anchor a (its first point) in FP64:
        // sum (t - a) = sum (t - a_g) + c delta and sum (t - a)^2 = sum (t - a_g)^2
        // + 2 delta sum (t - a_g) + c delta^2 over c points, delta = a_g - a.
        const bool from_series = ps <= 4;
        const float *T = a.T;
        const int64_t n = a.n;
        double anc = 0.0, run1 = 0.0, run2 = 0.0;
        int64_t xnext = 0;
        // the series points of the 64 grid intervals from x (lane l: points x + ps l + u, u < ps),
        // four loads per lane at 32-bit offsets from a uniform base, clamped to the last point of
        // the series (clamped points only reach grid points past it, which serve idle lanes)
        auto load_pts = [&](int64_t x, float (&t)[4]) {
            const float *base = T + x;
            const int64_t room = n - 1 - x;
            const int lim = room < 0x7fffffff ? (int)room : 0x7fffffff;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int o = (int)ps * lane + u;
                t[u] = base[o < lim ? o : lim];
            }
        };
        // prefix at grid points xnext + ps lane from those points, then xnext moves on 64 points
        auto grid_from = [&](const float (&t)[4]) -> double2 {
            const float ag = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t[0])));   // a_g
            float v1 = 0.0f, v2 = 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float d = u < ps ? t[u] - ag : 0.0f;
                v1 += d;
                v2 = fmaf(d, d, v2);
            }
            const float i1 = wave_scan_incl(v1), i2 = wave_scan_incl(v2);
            const double e1 = (double)dpp_or_zero<0x138, 0xF>(i1), e2 = (double)dpp_or_zero<0x138, 0xF>(i2);
            const double delta = (double)ag - anc, c = (double)(ps * lane);
            const double2 r = make_double2(run1 + fma(c, delta, e1), run2 + fma(c * delta, delta, fma(2.0 * delta, e1, e2)));
            const double s1 = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(i1), 63));
            const double s2 = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(i2), 63));
            const double cg = (double)(64 * ps);
            run1 += fma(cg, delta, s1);
            run2 += fma(cg * delta, delta, fma(2.0 * delta, s1, s2));
            xnext += 64 * ps;
            return r;
        };
        float tp[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // points of the next grid group, loaded a group ahead
        const bool carry = quarter % (64 * ps) == 0;   // quarters are whole groups: the grid carries over
        double2 rlo = make_double2(0.0, 0.0), rhi = rlo;
        for (int j = 0; j < kScoreSamples; ++j) {
          const int64_t first = bfirst + j * quarter;
          const int64_t last = first + quarter < qN ? first + quarter : qN;
          uint64_t best = ~0ull;
          if (first < last) {
          if (j == 0 || !carry) {
              if (from_series) {
                  xnext = first;
                  float t0[4];
                  load_pts(xnext, t0);
                  anc = (double)__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t0[0])));
                  run1 = run2 = 0.0;
                  rlo = grid_from(t0);
                  load_pts(xnext, t0);
                  rhi = grid_from(t0);
                  load_pts(xnext, tp);
              } else {
                  rlo = grid_raw(first + ps * lane);
                  rhi = grid_raw(first + ps * (lane + 64));
              }
          }
          // PAA distance of the 64 sampled starts g0 + ps lane from the grid prefix at their
          // window starts (g0v) and ends (g1v), both relative to one anchor
          auto score_group = [&](int64_t g0, double2 g0v, double2 g1v) {
            gw[lane] = g0v.x;
            gw[lane + 64] = g1v.x;
            wave_sync();
            // segment sums starting at grid points lane and lane + 64 (the last four are unused)
            dw[lane] = (float)(gw[lane + 4] - g0v.x);
            dw[lane + 64] = (float)(gw[(lane + 68) & 127] - g1v.x);
            wave_sync();
            const int64_t i = g0 + lane * ps;
            if (i < last) {
                const double md = (g1v.x - g0v.x) * inv_m, var = (g1v.y - g0v.y) * inv_m - md * md;
                const float inv = var > kSigmaFlat * kSigmaFlat ? rsqrtf((float)var) : 0.0f;
                // PAA term t: (segment sum / segment length - mean) / sigma - query term
                const float A = inv_seg * inv, C = (float)md * inv;
                float d = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const float e = fmaf(dw[lane + 4 * t], A, -(C + qp[t]));
                    d = fmaf(e, e, d);
                }
                const uint64_t key = ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(uint32_t)i;
                best = key < best ? key : best;
            }
          };
          if (from_series) {
            for (int64_t g0 = first; g0 < last; g0 += 64 * ps) {
              // take this group's points (loaded an iteration ago), then load the next group's
              // into the carried registers
              float tc[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) tc[u] = tp[u];
              load_pts(xnext + 64 * ps, tp);
              const double2 rnext = grid_from(tc);
              const double2 g0v = rlo, g1v = rhi;
              rlo = rhi;
              rhi = rnext;
              score_group(g0, g0v, g1v);
            }
          } else {
            // grid from the prefix: re-anchor the grid points past the block of the group's first
            // start (a window ends at most one block later), then score
            auto prefix_group = [&](int64_t g0, double2 rnext) {
              const int64_t b0 = g0 / kPB, e0 = (b0 + 1) * kPB;
              double2 gv[2] = {rlo, rhi};
              if (g0 + 127 * ps >= e0) {   // (wave-uniform) some grid point lies past the block
                  const double2 tb = sa.pre.tot[b0];
                  const double delta = sa.pre.anc[b0 + 1] - sa.pre.anc[b0];
#pragma unroll
                  for (int h = 0; h < 2; ++h) {
                      const int64_t x = g0 + ps * (lane + 64 * h);
                      const double2 p = h == 0 ? rlo : rhi;
                      const bool cross = x >= e0;
                      const double lx = (double)(x - e0);
                      gv[h].x = cross ? tb.x + p.x + lx * delta : p.x;
                      gv[h].y = cross ? tb.y + p.y + 2.0 * delta * p.x + lx * delta * delta : p.y;
                  }
              }
              rlo = rhi;
              rhi = rnext;
              score_group(g0, gv[0], gv[1]);
            };
            // (separate loops: the decimated copy is a plain load, the full prefix may need the
            // point before an odd grid position)
            if (use_dec) {
              for (int64_t g0 = first; g0 < last; g0 += 64 * ps) {
                int64_t x = g0 + ps * (lane + 128);
                x = x < nlast ? x : nlast;
                prefix_group(g0, dsrc[x >> dl]);
              }
            } else {
              for (int64_t g0 = first; g0 < last; g0 += 64 * ps) {
                int64_t x = g0 + ps * (lane + 128);
                x = x < nlast ? x : nlast;
                prefix_group(g0, sa.pre.at(x));
              }
            }
          }
          }
          best = wave_min_u64(best);
          if (lane == 0) winners[wid][j] = best;
        }
    } else {
        float inv_len[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) inv_len[t] = 1.0f / (float)((((t + 1) * m) >> 4) - ((t * m) >> 4));
        for (int j = 0; j < kScoreSamples; ++j) {
            const int64_t first = bfirst + j * quarter;
            const int64_t last = first + quarter < qN ? first + quarter : qN;
            uint64_t best = ~0ull;
            for (int64_t i = first + lane * ps; i < last; i += 64 * ps) {
                float f[16];
                pv.paa(i, m, inv_m, inv_len, f);
                float d = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const float e = f[t] - qp[t];
                    d = fmaf(e, e, d);
                }
                const uint64_t key = ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(uint32_t)i;
                best = key < best ? key : best;
            }
            best = wave_min_u64(best);
            if (lane == 0) winners[wid][j] = best;
        }
    }
    wave_sync();
    // features: lanes 16 j .. 16 j + 15 fill row k0 + j (term t = lane % 16 of both PAAs)
    const int j = lane >> 4, t = lane & 15;
    const uint64_t w = winners[wid][j];
    const bool empty = bfirst + j * quarter >= qN;
    float *x = X + (k0 + j) * 32;
    const int64_t i = empty ? bfirst : (int64_t)(uint32_t)w;   // a valid start either way
    const float f = pv.paa_term(i, m, inv_m, t);
    x[16 + t] = empty ? 0.0f : f;
    x[t] = empty ? 0.0f : sa.qpaa[q * 16 + t];
    if (t == 0) sa.sstart[k0 + j] = empty ? -1 : (int32_t)i;
}

// Score of a block = minimum predicted value over its proposals; bstart = that proposal's start.
__global__ void k_block_min(const float *y, const int32_t *sstart, int64_t R, int K, int64_t row0, float *score,
                            int32_t *bstart) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b * K >= R) return;
    float s = NAN;
    int32_t st = -1;
    for (int j = 0; j < K; ++j) {
        const int32_t sj = sstart[b * K + j];
        const float v = y[b * K + j];
        if (sj >= 0 && (st < 0 || v < s)) {
            s = v;
            st = sj;
        }
    }
    score[row0 / K + b] = s;
    bstart[row0 / K + b] = st;
}

// Round -1 of the learned order: the best-so-far of every query starts from the proposals of its
// kSeedBlocks best-scored blocks (repeating the last when a query has fewer blocks), each with the
// kSeedOffsets starts around it (offsets -8 .. +7, clipped to the candidates): a proposal lies on the
// sampling grid, so a near copy of the query is found at its own alignment, not only at the nearest
// grid start.
__global__ void k_seed_learned(BatchArgs a, const int32_t *bstart, const int64_t *row_off, int K) {
    // one thread per (query, seed)
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)a.nq * kSeedCands) return;
    const int q = (int)(e / kSeedCands), k = (int)(e % kSeedCands);
    const int kb = k / kSeedOffsets, off = k % kSeedOffsets - kSeedOffsets / 2;
    const BatchQ bq = a.bq[q];
    const int64_t nb = bq.nblocks;
    const int64_t blk = a.perm[(int64_t)q * a.maxblocks + (kb < nb ? kb : nb - 1)];
    int64_t st = (int64_t)bstart[row_off[q] / K + blk] + off;
    st = st < 0 ? 0 : (st > bq.N - 1 ? bq.N - 1 : st);
    a.surv_q[e] = q;
    a.surv_i[e] = (int32_t)st;
    a.surv_lb[e] = 0.0f;
    if (k == 0) a.qcnt[q * kCntStride] = kSeedCands;
    if (e == 0) *a.surv_count = (uint32_t)(a.nq * kSeedCands);
}

// Visiting order of a query's blocks by ascending score: counting sort into 2048 buckets between
// the minimum and maximum score (order inside a bucket is unspecified; it affects speed only).
constexpr int kOrderBuckets = 2048;
__global__ __launch_bounds__(1024) void k_block_order(const BatchArgs a, const float *score, const int64_t *row_off,
                                                      int K) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ float lo_s[32], hi_s[32];
    const int q = blockIdx.x, tid = threadIdx.x;
    const int64_t nb = a.bq[q].nblocks;
    const float *sc = score + row_off[q] / K;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t b = tid; b < nb; b += blockDim.x) {
        const float v = sc[b];
        if (v == v) {
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off, 64));
        hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    }
    if ((tid & 63) == 0) {
        lo_s[tid >> 6] = lo;
        hi_s[tid >> 6] = hi;
    }
    for (int k = tid; k < kOrderBuckets; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    lo = INFINITY;
    hi = -INFINITY;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        lo = fminf(lo, lo_s[w]);
        hi = fmaxf(hi, hi_s[w]);
    }
    const float scale = hi > lo ? (kOrderBuckets - 1) / (hi - lo) : 0.0f;
    auto bucket = [&](float v) -> int {
        if (!(v == v)) return kOrderBuckets - 1;
        int k = (int)((v - lo) * scale);
        return k < 0 ? 0 : (k >= kOrderBuckets ? kOrderBuckets - 1 : k);
    };
    for (int64_t b = tid; b < nb; b += blockDim.x) atomicAdd(&hist[bucket(sc[b])], 1u);
    __syncthreads();
    // exclusive prefix of the histogram: each thread owns kOrderBuckets / blockDim.x consecutive
    // buckets; a wave scan and a scan of the wave totals give every thread its offset
    {
        constexpr int kPer = kOrderBuckets / 1024;
        static_assert(kOrderBuckets % 1024 == 0, "buckets per thread");
        __shared__ uint32_t wsum[16];
        uint32_t own[kPer], tsum = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            own[u] = hist[tid * kPer + u];
            tsum += own[u];
        }
        uint32_t incl = tsum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, 64);
            if ((tid & 63) >= off) incl += o;
        }
        if ((tid & 63) == 63) wsum[tid >> 6] = incl;
        __syncthreads();
        uint32_t base = 0;
        for (int w = 0; w < (tid >> 6); ++w) base += wsum[w];
        uint32_t run = base + incl - tsum;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            hist[tid * kPer + u] = run;
            run += own[u];
        }
    }
    __syncthreads();
    int32_t *perm = a.perm + (int64_t)q * a.maxblocks;
    for (int64_t b = tid; b < nb; b += blockDim.x) {
        const uint32_t pos = atomicAdd(&hist[bucket(sc[b])], 1u);
        perm[pos] = (int32_t)b;
    }
}

// ------------------------------------------------------------------ host side
hipError_t mlp_gemm(const uint16_t *A, int64_t lda, const uint16_t *BT, int64_t ldb, float *C, int64_t ldc, int M, int N,
                    int K, hipStream_t s) {
    const int64_t waves = (int64_t)(M / 16) * (N / 64);
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, BT, ldb, C, ldc, M, N, K);
    return hipGetLastError();
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

hipError_t mlp_refresh(const MlpBufs &b, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_refresh, dim3(nblk(65536)), dim3(256), 0, s, b.theta, b.theta + kOffW2, b.W1T, b.W2T,
                       b.W2b);
    return hipGetLastError();
}

hipError_t mlp_init(const MlpBufs &b, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3(nblk(kModelParams)), dim3(256), 0, s, b.theta, seed);
    hipError_t e = launch_fill_u32((uint32_t *)b.adam_m, 0, kModelParams, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)b.adam_v, 0, kModelParams, s);
    if (e == hipSuccess) e = mlp_refresh(b, s);
    return e;
}

// Forward pass on R rows (R <= kMlpChunk).  Training keeps the transposed operands and H2.
hipError_t mlp_forward(const MlpBufs &b, const float *X, int64_t R, float *y, bool train, hipStream_t s) {
    if (!train) {
        // scoring: one fused pass, one workgroup per compute unit (its LDS holds the weights),
        // none without a tile
        const int64_t tiles = (R + 15) / 16, per_block = kInferThreads / 64;
        int64_t blocks = (tiles + per_block - 1) / per_block;
        if (blocks > b.num_cu) blocks = b.num_cu;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(kInferThreads), 0, s, X, R, b.W1T,
                           b.theta + kOffb1, b.W2T, b.theta + kOffb2, b.theta + kOffw3, b.theta + kOffb3, y);
        return hipGetLastError();
    }
    const int64_t Rp = (R + 63) / 64 * 64;
    hipLaunchKernelGGL(k_mlp_x, dim3(nblk(Rp * 32)), dim3(256), 0, s, X, R, Rp, b.Xb, train ? b.XbT : nullptr);
    hipError_t e = mlp_gemm(b.Xb, 32, b.W1T, 32, b.C1, 256, (int)Rp, 256, 32, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_act1, dim3(nblk(Rp * 256)), dim3(256), 0, s, b.C1, b.theta + kOffb1, Rp, b.H1b,
                       train ? b.H1T : nullptr);
    e = mlp_gemm(b.H1b, 256, b.W2T, 256, b.C2, 256, (int)Rp, 256, 256, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_head, dim3(nblk(Rp * 64)), dim3(256), 0, s, b.C2, b.theta + kOffb2, b.theta + kOffw3,
                       b.theta + kOffb3, Rp, y, train, X, R);
    return hipGetLastError();
}

// Gradient of the mean squared error on R rows into b.grad (and the loss into b.loss).
hipError_t mlp_backward(const MlpBufs &b, const float *X, const float *t, int64_t R, hipStream_t s) {
    const int64_t Rp = (R + 63) / 64 * 64;
    hipError_t e = mlp_forward(b, X, R, b.y, true, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32((uint32_t *)b.loss, 0, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_bwd_head, dim3(nblk(Rp * 256)), dim3(256), 0, s, b.y, t, b.C2, b.theta + kOffw3, R, Rp,
                       b.dy, b.dA2b, b.dA2T, b.loss);
    // dH1 = dA2 W2^T  (B^T of this product is W2 itself, row-major)
    e = mlp_gemm(b.dA2b, 256, b.W2b, 256, b.C1, 256, (int)Rp, 256, 256, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_bwd1, dim3(nblk(Rp * 256)), dim3(256), 0, s, b.C1, b.H1b, Rp, b.dA1T);
    // dW2 = H1^T dA2, dW1 = X^T dA1 (products over the rows)
    e = mlp_gemm(b.H1T, Rp, b.dA2T, Rp, b.grad + kOffW2, 256, 256, 256, (int)Rp, s);
    if (e != hipSuccess) return e;
    e = mlp_gemm(b.XbT, Rp, b.dA1T, Rp, b.grad + kOffW1, 256, 32, 256, (int)Rp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_colsums_part, dim3(kColsumGroups), dim3(256), 0, s, b.C1, b.H1b, b.C2, b.dy,
                       b.theta + kOffw3, R, b.part);
    hipLaunchKernelGGL(k_mlp_colsums, dim3(1), dim3(256), 0, s, b.part, b.grad + kOffb1, b.grad + kOffb2,
                       b.grad + kOffw3, b.grad + kOffb3);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpBufs &b, int step, float lr, hipStream_t s) {
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(kModelParams)), dim3(256), 0, s, b.theta, b.grad, b.adam_m, b.adam_v,
                       (int64_t)kModelParams, lr, c1, c2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = mlp_refresh(b, s);
    return e;
}

// PAA score of a feature row (the learned order's control): the squared Euclidean distance of its
// query half to its candidate half, as log(d / 16 + 1e-4): the network's PAA-distance term, so the
// control is the network with a zero output layer.
__global__ void k_paa_score(const float *X, int64_t R, float *y) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= R) return;
    const float4 *x = (const float4 *)(X + k * 32);
    float d = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float4 a = x[t], c = x[t + 4];
        d = fmaf(a.x - c.x, a.x - c.x, d);
        d = fmaf(a.y - c.y, a.y - c.y, d);
        d = fmaf(a.z - c.z, a.z - c.z, d);
        d = fmaf(a.w - c.w, a.w - c.w, d);
    }
    y[k] = logf(d * (1.0f / 16.0f) + 1e-4f);
}

// Scores every block of every query of the batch and writes the visiting order into a.perm: by the
// network's prediction, or (paa_only) by the proposals' PAA distance.
hipError_t mlp_order_blocks(const MlpBufs &b, const BatchArgs &a, const ScoreArgs &sa, bool paa_only, hipStream_t s) {
    hipLaunchKernelGGL(k_query_paa, dim3(a.nq), dim3(64), 0, s, a, sa.qpaa);
    const int64_t chunk = kMlpChunk / sa.K * sa.K;
    for (int64_t r0 = 0; r0 < sa.total_rows; r0 += chunk) {
        const int64_t R = sa.total_rows - r0 < chunk ? sa.total_rows - r0 : chunk;
        if (sa.kinds & 1u)
            hipLaunchKernelGGL(k_propose<true>, dim3(nblk(R / kScoreSamples * 64)), dim3(256), 0, s, a, sa, r0, R, b.Xf);
        if (sa.kinds & 2u)
            hipLaunchKernelGGL(k_propose<false>, dim3(nblk(R / kScoreSamples * 64)), dim3(256), 0, s, a, sa, r0, R, b.Xf);
        if (paa_only) {
            hipLaunchKernelGGL(k_paa_score, dim3(nblk(R)), dim3(256), 0, s, b.Xf, R, b.y);
        } else {
            hipError_t e = mlp_forward(b, b.Xf, R, b.y, false, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_block_min, dim3(nblk(R / sa.K)), dim3(256), 0, s, b.y, sa.sstart, R, sa.K, r0, sa.score,
                           sa.bstart);
    }
    hipLaunchKernelGGL(k_block_order, dim3(a.nq), dim3(1024), 0, s, a, sa.score, sa.row_off, sa.K);
    return hipGetLastError();
}

__global__ void k_widen_starts(const int32_t *s32, int64_t R, int64_t *s64) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < R) s64[k] = s32[k];
}

// Proposals of every quarter block of the batch's first query: features into X (rows x 32) and
// starts into starts (rows), rows = sa.total_rows.
hipError_t launch_propose(const BatchArgs &a, const ScoreArgs &sa, float *X, int64_t *starts, hipStream_t s) {
    hipLaunchKernelGGL(k_query_paa, dim3(a.nq), dim3(64), 0, s, a, sa.qpaa);
    for (int64_t r0 = 0; r0 < sa.total_rows; r0 += kMlpChunk) {
        const int64_t R = sa.total_rows - r0 < kMlpChunk ? sa.total_rows - r0 : kMlpChunk;
        if (sa.kinds & 1u)
            hipLaunchKernelGGL(k_propose<true>, dim3(nblk(R / kScoreSamples * 64)), dim3(256), 0, s, a, sa, r0, R,
                               X + r0 * 32);
        if (sa.kinds & 2u)
            hipLaunchKernelGGL(k_propose<false>, dim3(nblk(R / kScoreSamples * 64)), dim3(256), 0, s, a, sa, r0, R,
                               X + r0 * 32);
        hipLaunchKernelGGL(k_widen_starts, dim3(nblk(R)), dim3(256), 0, s, sa.sstart, R, starts + r0);
    }
    return hipGetLastError();
}

hipError_t launch_seed_learned(const BatchArgs &a, const ScoreArgs &sa, hipStream_t s) {
    hipLaunchKernelGGL(k_seed_learned, dim3(nblk((int64_t)a.nq * kSeedCands)), dim3(256), 0, s, a, sa.bstart, sa.row_off,
                       sa.K);
    return hipGetLastError();
}

hipError_t launch_paa(const float *T, int64_t n, int m, const int64_t *starts, int64_t count, float *out,
                      hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_paa, dim3(nblk(count)), dim3(256), 0, s, T, n, m, starts, count, out);
    return hipGetLastError();
}

}  // namespace dtws
