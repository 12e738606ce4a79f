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
// guarantees M % 64 == 0, N % 64 == 0, k_split % 32 == 0, lda % 8 == 0,
// ldb % 8 == 0 and 16-byte aligned A and B; split s covers k in
// [s * k_split, (s + 1) * k_split).  Grid: (N/64, M/64, splits).
//
// Each K-step stages a 64 x 32 slice of opA and a 32 x 64 slice of opB with
// one 16-byte load per thread and operand, kept in LDS in the layout of the
// stored rows (so the LDS writes are 16 bytes too); the next slice's loads
// are issued before the current slice's matrix-core work.
//
// MFMA operand layout (16 x 16 x 32, checked on the device against a host
// product): lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16]
// for i < 8, and receives D[4 (l / 16) + r][l % 16] for r < 4.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }

// What a product does with its result v at (m, n) (EPI_STORE for any split
// count, the others with one split; rows of Z, A, dZ have stride ldc):
//   EPI_STORE      C[split][m][n] = v
//   EPI_BIAS_SILU  hidden layer: Z = v + b[n] (FP32, kept for the backward
//                  pass), A = silu(Z) = Z sigmoid(Z) (bf16)
//   EPI_BIAS_OUT   output layer: Y[m][n] = v + b[n] for n < keep ([m][keep])
//   EPI_SILU_GRAD  input gradient: dZ = v silu'(Z), silu'(z) = sigmoid(z)
//                  (1 + z (1 - sigmoid(z))) (bf16), Z read
//   EPI_STORE_DB   weight gradient X^T dZ (opA transposed): as EPI_STORE, and
//                  the workgroups of the first row block also write the
//                  column sums of this split's opB rows (the bias gradient's
//                  partial) to the N floats after the split's M x ldc block
// Split s writes at C + s * split_stride.
enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS_OUT = 2, EPI_SILU_GRAD = 3, EPI_STORE_DB = 4 };
struct Epilogue {
    const float* bias = nullptr;
    float* z = nullptr;       // EPI_BIAS_SILU: written; EPI_SILU_GRAD: read
    uint16_t* act = nullptr;  // A (EPI_BIAS_SILU) or dZ (EPI_SILU_GRAD)
    float* y = nullptr;
    int keep = 0;
};

template <bool TA, bool TB, int EPI = EPI_STORE>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_bf16(const uint16_t* __restrict__ A,
                                                          const uint16_t* __restrict__ B, float* __restrict__ C,
                                                          int M, int N, int lda, int ldb, int ldc, int k_split,
                                                          int64_t split_stride, Epilogue ep)
{
    // Rows padded by 8 elements (16 bytes) to stagger them across LDS banks.
    // opA: [m][k] (TA false) or [k][m] (TA true); opB: [k][n] or [n][k].
    constexpr int AR = TA ? TK : TM, AC = (TA ? TM : TK) + 8;
    constexpr int BR = TB ? TN : TK, BC = (TB ? TK : TN) + 8;
    __shared__ __attribute__((aligned(16))) uint16_t As[AR][AC];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BR][BC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m_blk = blockIdx.y * TM, n_blk = blockIdx.x * TN;
    const int k_beg = blockIdx.z * k_split, k_end = k_beg + k_split;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    // This thread's 8 elements of each slice: row r and column c8 of the
    // stored layout (rows of 32 elements: 4 threads a row; of 64: 8).
    const int ar = TA ? tid >> 3 : tid >> 2, ac = TA ? (tid & 7) * 8 : (tid & 3) * 8;
    const int br = TB ? tid >> 2 : tid >> 3, bc = TB ? (tid & 3) * 8 : (tid & 7) * 8;
    const auto a_src = [&](int k0) {
        return TA ? A + (int64_t)(k0 + ar) * lda + m_blk + ac : A + (int64_t)(m_blk + ar) * lda + k0 + ac;
    };
    const auto b_src = [&](int k0) {
        return TB ? B + (int64_t)(n_blk + br) * ldb + k0 + bc : B + (int64_t)(k0 + br) * ldb + n_blk + bc;
    };
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // EPI_STORE_DB: thread t sums rows 8 (t / 64) .. + 7 of column t % 64 of
    // every staged opB slice (row order), combined over t / 64 at the end
    constexpr bool DB = EPI == EPI_STORE_DB;
    static_assert(!DB || (TA && !TB), "bias-gradient sums need opB stored as [k][n]");
    const bool db_blk = DB && blockIdx.y == 0;
    float db = 0.f;

    u32x4 ga = *reinterpret_cast<const u32x4*>(a_src(k_beg));
    u32x4 gb = *reinterpret_cast<const u32x4*>(b_src(k_beg));
    for (int k0 = k_beg; k0 < k_end; k0 += TK) {
        *reinterpret_cast<u32x4*>(&As[ar][ac]) = ga;
        *reinterpret_cast<u32x4*>(&Bs[br][bc]) = gb;
        __syncthreads();
        if (k0 + TK < k_end) {
            ga = *reinterpret_cast<const u32x4*>(a_src(k0 + TK));
            gb = *reinterpret_cast<const u32x4*>(b_src(k0 + TK));
        }
        if (db_blk) {
#pragma unroll
            for (int i = 0; i < 8; ++i) db += bf_to_f(Bs[8 * (tid >> 6) + i][tid & 63]);
        }
        bf16x8 a[2], b[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const int am = wm + f * 16 + (lane & 15), bn = wn + f * 16 + (lane & 15), k8 = 8 * (lane >> 4);
            if constexpr (TA) {
#pragma unroll
                for (int i = 0; i < 8; ++i) a[f][i] = __builtin_bit_cast(__bf16, As[k8 + i][am]);
            } else {
                a[f] = *reinterpret_cast<const bf16x8*>(&As[am][k8]);
            }
            if constexpr (TB) {
                b[f] = *reinterpret_cast<const bf16x8*>(&Bs[bn][k8]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) b[f][i] = __builtin_bit_cast(__bf16, Bs[k8 + i][bn]);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float* Cs = C + (int64_t)blockIdx.z * split_stride;
    if constexpr (DB) {
        if (db_blk) { // uniform over the workgroup
            __shared__ float part[4][64];
            part[tid >> 6][tid & 63] = db;
            __syncthreads();
            if (tid < 64) Cs[(int64_t)M * ldc + n_blk + tid] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m_blk + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n_blk + wn + j * 16 + (lane & 15);
                const int64_t t = (int64_t)m * ldc + n;
                const float v = acc[i][j][r];
                if constexpr (EPI == EPI_STORE || EPI == EPI_STORE_DB) {
                    Cs[t] = v;
                } else if constexpr (EPI == EPI_BIAS_SILU) {
                    const float z = v + ep.bias[n];
                    ep.z[t] = z;
                    ep.act[t] = f_to_bf(z * sigmoid(z));
                } else if constexpr (EPI == EPI_BIAS_OUT) {
                    if (n < ep.keep) ep.y[(int64_t)m * ep.keep + n] = v + ep.bias[n];
                } else {
                    const float z = ep.z[t], sg = sigmoid(z);
                    ep.act[t] = f_to_bf(v * sg * (1.0f + z * (1.0f - sg)));
                }
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
