// The MLP surrogate of log L used by delayed acceptance: forward, backward
// and Adam on gfx950.
//
// Network (per row x of a batch): h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2),
// s = w3 . h2 + b3, gelu(t) = t (1 + erf(t / sqrt 2)) / 2 (Hendrycks & Gimpel
// 2016).  Loss: mean squared error.  Optimiser: Adam (Kingma & Ba 2015).
//
// Matrix products run on MFMA (v_mfma_f32_16x16x32_bf16): BF16 operands,
// FP32 accumulation.  One product kernel, C[M][N] = sum_k A[m][k] B[n][k]
// ("both operands K-contiguous"), covers the forward layers (B = W) and,
// after explicit transposes, the backward products dX = dZ W and dW = dZ^T X.
// Activations are stored in BF16 for the next product, pre-activations in
// FP32 for the GELU derivative; master weights, gradients and Adam moments
// are FP32 in one flat array [W1 | b1 | W2 | b2 | w3 | b3].
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace qst {

typedef __bf16 mlp_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float t) { return 0.5f * t * (1.0f + erff(t * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float t)
{
    return 0.5f * (1.0f + erff(t * 0.70710678118654752f)) + t * expf(-0.5f * t * t) * 0.39894228040143268f;
}

__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    const __bf16 h = static_cast<__bf16>(f);   // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float bf16_value(uint16_t b) { return static_cast<float>(__builtin_bit_cast(__bf16, b)); }

// ---------------------------------------------------------------------------
// C[M][N] = A[M][K] B[N][K]^T, K a multiple of 32 (rows of A and B beyond
// M and N read as zero and are not stored).
// 64x64 output tile per 256-thread workgroup, each wave a 32x32 quarter as
// 2x2 MFMA tiles; K in slices of 32 staged through LDS (rows padded to 40
// elements against bank conflicts).
// Epilogues: kStoreF32: C as FP32; kBiasGelu: z = C + bias[n] stored FP32 in
// Z and gelu(z) as BF16 in H; kGeluGrad: BF16 of C * gelu'(Zin[m][n]) in H.
// ---------------------------------------------------------------------------
enum : int { kStoreF32 = 0, kBiasGelu = 1, kGeluGrad = 2 };

constexpr int kMlpTile = 64;
constexpr int kMlpBK = 32;
constexpr int kMlpLdsRow = 40;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt_bf16(int M, int N, const uint16_t* __restrict__ A, int lda,
                                                      const uint16_t* __restrict__ B, int ldb, int K,
                                                      float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                                      const float* __restrict__ Zin, float* __restrict__ Zout,
                                                      uint16_t* __restrict__ H, int ldh)
{
    __shared__ uint16_t As[kMlpTile * kMlpLdsRow];
    __shared__ uint16_t Bs[kMlpTile * kMlpLdsRow];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    const int m0 = blockIdx.y * kMlpTile, n0 = blockIdx.x * kMlpTile;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    mlp_f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mlp_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // each thread stages 8 consecutive k of one row of A and of B per slice
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    for (int k0 = 0; k0 < K; k0 += kMlpBK) {
        const uint4 zero4 = {0u, 0u, 0u, 0u};
        const uint4 av = (m0 + lr < M) ? *reinterpret_cast<const uint4*>(A + static_cast<size_t>(m0 + lr) * lda + k0 + lk)
                                       : zero4;
        const uint4 bv = (n0 + lr < N) ? *reinterpret_cast<const uint4*>(B + static_cast<size_t>(n0 + lr) * ldb + k0 + lk)
                                       : zero4;
        __syncthreads();
        *reinterpret_cast<uint4*>(As + lr * kMlpLdsRow + lk) = av;
        *reinterpret_cast<uint4*>(Bs + lr * kMlpLdsRow + lk) = bv;
        __syncthreads();
        // MFMA 16x16x32: lane l supplies row l%16, k = 8 (l/16) .. +7
        mlp_bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const mlp_bf16x8*>(As + (wm + 16 * i + (l & 15)) * kMlpLdsRow + 8 * (l >> 4));
            b[i] = *reinterpret_cast<const mlp_bf16x8*>(Bs + (wn + 16 * i + (l & 15)) * kMlpLdsRow + 8 * (l >> 4));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // result register r of lane l: row 4 (l/16) + r, column l % 16 of the 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (l >> 4) + r;
                const int n = n0 + wn + 16 * j + (l & 15);
                if (m >= M || n >= N) continue;
                const float v = acc[i][j][r];
                if constexpr (EPI == kStoreF32) {
                    C[static_cast<size_t>(m) * ldc + n] = v;
                } else if constexpr (EPI == kBiasGelu) {
                    const float z = v + bias[n];
                    Zout[static_cast<size_t>(m) * ldc + n] = z;
                    H[static_cast<size_t>(m) * ldh + n] = bf16_bits(gelu_f(z));
                } else {
                    H[static_cast<size_t>(m) * ldh + n] = bf16_bits(v * gelu_grad_f(Zin[static_cast<size_t>(m) * ldc + n]));
                }
            }
}

// out[c][r] = in[r][c] for a rows x cols BF16 matrix (32x32 tiles through LDS)
__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t* __restrict__ in, int rows, int cols,
                                                        uint16_t* __restrict__ out)
{
    __shared__ uint16_t t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        t[y][tx] = (r < rows && c < cols) ? in[static_cast<size_t>(r) * cols + c] : 0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (c < cols && r < rows) out[static_cast<size_t>(c) * rows + r] = t[tx][y];
    }
}

// BF16 copy of an FP32 array (weights for the products)
__global__ void k_f32_to_bf16(const float* __restrict__ in, int64_t n, uint16_t* __restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = bf16_bits(in[i]);
}

// Last layer and loss: one 64-lane wave per row m.
// s[m] = w3 . h2[m] + b3; with targets: d = s - y, ds[m] = 2 d / n, sq[m] = d^2.
__global__ __launch_bounds__(256) void k_last_fwd(const uint16_t* __restrict__ H2, int h2, const float* __restrict__ w3,
                                                  const float* __restrict__ b3, int64_t n, float out_scale,
                                                  float out_shift, float* __restrict__ s_out,
                                                  const float* __restrict__ y, float* __restrict__ ds,
                                                  float* __restrict__ sq)
{
    const int64_t m = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (m >= n) return;
    float acc = 0.0f;
    for (int k = l; k < h2; k += 64) acc += bf16_value(H2[m * h2 + k]) * w3[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (l == 0) {
        const float s = acc + b3[0];
        if (s_out) s_out[m] = out_scale * s + out_shift;
        if (y) {
            const float d = s - y[m];
            ds[m] = 2.0f * d / static_cast<float>(n);
            sq[m] = d * d;
        }
    }
}

// dz2[m][k] = BF16(ds[m] w3[k] gelu'(z2[m][k]))
__global__ void k_last_bwd_dz(const float* __restrict__ ds, const float* __restrict__ w3, const float* __restrict__ Z2,
                              int64_t n, int h2, uint16_t* __restrict__ dz2)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * h2) return;
    const int64_t m = i / h2;
    const int k = static_cast<int>(i % h2);
    dz2[i] = bf16_bits(ds[m] * w3[k] * gelu_grad_f(Z2[i]));
}

// Column sums in a fixed order, two passes: part[chunk][c] = sum over the
// chunk's rows of w[r] * in[r][c] (w = 1 when NULL; in BF16), then
// out[c] = sum over chunks.  With in = NULL the matrix is all ones (so
// part = sum of w over the chunk: the bias gradient of the last layer).
constexpr int kColChunk = 64;

__global__ __launch_bounds__(256) void k_colsum_partial(const uint16_t* __restrict__ in, const float* __restrict__ w,
                                                        int64_t rows, int cols, float* __restrict__ part)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * kColChunk;
    if (c >= cols) return;
    float acc = 0.0f;
    for (int64_t r = r0; r < r0 + kColChunk && r < rows; ++r) {
        const float x = in ? bf16_value(in[r * cols + c]) : 1.0f;
        acc += w ? x * w[r] : x;
    }
    part[static_cast<int64_t>(blockIdx.y) * cols + c] = acc;
}

__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int nchunks, int cols,
                                                      float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.0f;
    for (int k = 0; k < nchunks; ++k) acc += part[static_cast<int64_t>(k) * cols + c];
    out[c] = acc;
}

// sum of n floats in a fixed order (one workgroup)
__global__ __launch_bounds__(256) void k_sum_f32(const float* __restrict__ in, int64_t n, float* __restrict__ out)
{
    __shared__ float part[256];
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += in[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int t = 0; t < 256; ++t) s += part[t];
        out[0] = s;
    }
}

// Mean, variance and count of non-finite values of n doubles, fixed order
// (one workgroup): out = {mean, var, nonfinite}.
__global__ __launch_bounds__(256) void k_moments_f64(const double* __restrict__ x, int64_t n, double* __restrict__ out)
{
    __shared__ double ps[256], pq[256], pb[256];
    double s = 0.0, bad = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = x[i];
        if (isfinite(v)) s += v;
        else bad += 1.0;
    }
    ps[threadIdx.x] = s;
    pb[threadIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < 256; ++t) {
            a += ps[t];
            b += pb[t];
        }
        ps[0] = a / static_cast<double>(n);
        pb[0] = b;
    }
    __syncthreads();
    const double mean = ps[0];
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = x[i] - mean;
        if (isfinite(v)) q += v * v;
    }
    pq[threadIdx.x] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int t = 0; t < 256; ++t) a += pq[t];
        out[0] = mean;
        out[1] = a / static_cast<double>(n);
        out[2] = pb[0];
    }
}

__global__ void k_standardise(const double* __restrict__ x, int64_t n, double mean, double sd, float* __restrict__ y)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = static_cast<float>((x[i] - mean) / sd);
}

// Row gather: xo[k] = x[idx[k]] (width BF16 values), yo[k] = y[idx[k]].
__global__ void k_gather_rows(const uint16_t* __restrict__ x, int width, const float* __restrict__ y,
                              const int64_t* __restrict__ idx, int64_t n, uint16_t* __restrict__ xo,
                              float* __restrict__ yo)
{
    const int64_t k = blockIdx.x;
    if (k >= n) return;
    const int64_t r = idx[k];
    for (int i = threadIdx.x; i < width; i += blockDim.x) xo[k * width + i] = x[r * width + i];
    if (threadIdx.x == 0) yo[k] = y[r];
}

// Adam (Kingma & Ba 2015) on the flat FP32 parameter array.
__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float beta1, float beta2, float eps,
                       float bc1, float bc2)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / bc1, vhat = vi / bc2;
    theta[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

}  // namespace qst
