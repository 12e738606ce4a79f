// mlp_kernels.hpp -- gfx950 kernels of the coordinate network that predicts
// warm-start fields (rho, u, v) for the cavity solver: a bfloat16 MFMA GEMM
// with FP32 accumulation (forward and both backward products), fused
// bias + SiLU epilogues, Fourier input features, the MSE gradient,
// deterministic reductions and the Adam update.
//
// Layouts: activations are row-major [rows][features]; weights W_l are
// row-major [in][out] so a layer is Z = X W + b.  bf16 values travel as
// uint16_t bit patterns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smrt {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round-to-nearest-even binary32 -> bfloat16 bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f_to_bf(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int TM = 64, TN = 64, TK = 32; // workgroup tile and K step
constexpr int GEMM_THREADS = 256;         // 4 waves, each a 32 x 32 quarter

// C[split][m][n] = sum over this split's k of opA(m, k) * opB(k, n), with
//   opA(m, k) = TA ? A[k * lda + m] : A[m * lda + k]
//   opB(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n],
// bf16 inputs, FP32 accumulation in v_mfma_f32_16x16x32_bf16.  The host
// guarantees M % 64 == 0, N % 64 == 0 and k_split % 32 == 0; split s covers
// k in [s * k_split, (s + 1) * k_split).  Grid: (N/64, M/64, splits).
//
// MFMA operand layout (16 x 16 x 32, checked on the device against a host
// product): lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16]
// for i < 8, and receives D[4 (l / 16) + r][l % 16] for r < 4.
template <bool TA, bool TB>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_bf16(const uint16_t* __restrict__ A,
                                                          const uint16_t* __restrict__ B, float* __restrict__ C,
                                                          int M, int N, int lda, int ldb, int ldc, int k_split)
{
    __shared__ uint16_t As[TM][TK + 8]; // +8: stagger rows across LDS banks
    __shared__ uint16_t Bs[TK][TN + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m_blk = blockIdx.y * TM, n_blk = blockIdx.x * TN;
    const int k_beg = blockIdx.z * k_split;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = k_beg; k0 < k_beg + k_split; k0 += TK) {
        // Stage the 64 x 32 slice of opA and the 32 x 64 slice of opB: 8
        // elements per thread each, the fastest index along the stored rows.
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + e * GEMM_THREADS; // 0 .. 2047
            if (TA) {
                const int m = idx & (TM - 1), k = idx >> 6; // contiguous along m
                As[m][k] = A[(int64_t)(k0 + k) * lda + m_blk + m];
            } else {
                const int k = idx & (TK - 1), m = idx >> 5; // contiguous along k
                As[m][k] = A[(int64_t)(m_blk + m) * lda + k0 + k];
            }
            if (TB) {
                const int k = idx & (TK - 1), n = idx >> 5;
                Bs[k][n] = B[(int64_t)(n_blk + n) * ldb + k0 + k];
            } else {
                const int n = idx & (TN - 1), k = idx >> 6;
                Bs[k][n] = B[(int64_t)(k0 + k) * ldb + n_blk + n];
            }
        }
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[f][i] = __builtin_bit_cast(__bf16, As[wm + f * 16 + (lane & 15)][8 * (lane >> 4) + i]);
                b[f][i] = __builtin_bit_cast(__bf16, Bs[8 * (lane >> 4) + i][wn + f * 16 + (lane & 15)]);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float* Cs = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m_blk + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n_blk + wn + j * 16 + (lane & 15);
                Cs[(int64_t)m * ldc + n] = acc[i][j][r];
            }
}

// Input features of a point p = (x, y, s): [x, y, s, sin(2 pi B p), cos(2 pi B p), 0...]
// with B the nf x 3 frequency matrix; written as bf16 rows of width `width`.
__global__ void features(const float* __restrict__ p, const float* __restrict__ Bf, int nf, int n, int width,
                         uint16_t* __restrict__ X)
{
    const int64_t total = (int64_t)n * width;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / width;
        const int c = (int)(t % width);
        const float x = p[i * 3 + 0], y = p[i * 3 + 1], s = p[i * 3 + 2];
        float v = 0.f;
        if (c < 3) {
            v = c == 0 ? x : (c == 1 ? y : s);
        } else if (c < 3 + 2 * nf) {
            const int j = (c - 3) % nf;
            const float arg = 6.283185307179586f * (Bf[j * 3 + 0] * x + Bf[j * 3 + 1] * y + Bf[j * 3 + 2] * s);
            v = c < 3 + nf ? sinf(arg) : cosf(arg);
        }
        X[t] = f_to_bf(v);
    }
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Hidden layer epilogue: Z = C + b (kept in FP32 for the backward pass),
// A = silu(Z) = Z sigmoid(Z) as bf16.  Output layer (act == 0): Y = C + b for
// the first `keep` columns, written densely [n][keep].
__global__ void bias_act(const float* __restrict__ Cm, const float* __restrict__ b, int n, int N, int act,
                         float* __restrict__ Z, uint16_t* __restrict__ A, int keep, float* __restrict__ Y)
{
    const int64_t total = (int64_t)n * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % N);
        const float z = Cm[t] + b[c];
        if (act) {
            Z[t] = z;
            A[t] = f_to_bf(z * sigmoid(z));
        } else if (c < keep) {
            Y[(t / N) * keep + c] = z;
        }
    }
}

// MSE over the `keep` outputs of n rows: loss = sum (y - t)^2 / (n keep).
// dY (bf16, [n][N], zero in the padding columns) = 2 (y - t) / (n keep);
// per-block FP64 partial sums of the squared error.
__global__ void __launch_bounds__(256) mse_grad(const float* __restrict__ Y, const float* __restrict__ T, int n,
                                                int keep, int N, uint16_t* __restrict__ dY,
                                                double* __restrict__ partial)
{
    __shared__ double lds[4];
    double acc = 0.0;
    const float scale = 2.0f / ((float)n * keep);
    const int64_t total = (int64_t)n * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % N);
        const int64_t i = t / N;
        float g = 0.f;
        if (c < keep) {
            const float e = Y[i * keep + c] - T[i * keep + c];
            acc += (double)e * e;
            g = scale * e;
        }
        dY[t] = f_to_bf(g);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// dZ = dA * silu'(Z), silu'(z) = sigmoid(z) (1 + z (1 - sigmoid(z))); bf16 out.
__global__ void silu_backward(const float* __restrict__ dA, const float* __restrict__ Z, int64_t total,
                              uint16_t* __restrict__ dZ)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const float z = Z[t], sg = sigmoid(z);
        dZ[t] = f_to_bf(dA[t] * sg * (1.0f + z * (1.0f - sg)));
    }
}

// out[c] = sum over r < rows of in[r * ld + c] for c < cols, in row order
// (deterministic).  One thread per column; used for split-K sums and biases.
template <typename T>
__global__ void column_sums(const T* __restrict__ in, int rows, int cols, int64_t ld, float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) {
        if constexpr (sizeof(T) == 2)
            s += bf_to_f(in[(int64_t)r * ld + c]);
        else
            s += in[(int64_t)r * ld + c];
    }
    out[c] = s;
}

// First stage of a column sum over many rows: partial[chunk][c] = sum of
// in[r][c] over the rows of chunk blockIdx.y (row order).  Grid:
// (ceil(cols / blockDim.x), chunks).
template <typename T>
__global__ void column_sums_chunked(const T* __restrict__ in, int rows, int cols, int64_t ld, int rows_per_chunk,
                                    float* __restrict__ partial)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int r0 = blockIdx.y * rows_per_chunk;
    const int r1 = min(rows, r0 + rows_per_chunk);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) {
        if constexpr (sizeof(T) == 2)
            s += bf_to_f(in[(int64_t)r * ld + c]);
        else
            s += in[(int64_t)r * ld + c];
    }
    partial[(int64_t)blockIdx.y * cols + c] = s;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master parameters, with
// bias-corrected step size lr_t; refreshes the bf16 copy when given.
__global__ void adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                     float* __restrict__ v, int64_t n, float lr_t, uint16_t* __restrict__ w_bf)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr_t * mi / (sqrtf(vi) + 1e-8f);
        w[i] = wi;
        if (w_bf) w_bf[i] = f_to_bf(wi);
    }
}

// dst = bf16(src), elementwise.
__global__ void to_bf16(const float* __restrict__ src, int64_t n, uint16_t* __restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f_to_bf(src[i]);
}

// Copies a rows x cols block between a dense array and a padded one:
// padded[r * ld + c] <-> dense[r * cols + c].
__global__ void pad_copy(const float* __restrict__ src, float* __restrict__ dst, int rows, int cols, int ld,
                         int to_padded)
{
    const int64_t total = (int64_t)rows * cols;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cols;
        const int c = (int)(t % cols);
        if (to_padded)
            dst[r * ld + c] = src[t];
        else
            dst[t] = src[r * ld + c];
    }
}

} // namespace mlp
} // namespace smrt
