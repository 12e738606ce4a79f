// mlp_kernels.hpp -- gfx950 kernels of the coordinate network that predicts
// warm-start fields (rho, u, v) for the cavity solver.
//
// Layouts: activations are row-major [rows][features] bf16; a layer is
// Z = X W + b with W row-major [in][out], kept as FP32 master values, a bf16
// copy and a transposed bf16 copy ([out][in]).  bf16 values travel as
// uint16_t bit patterns.  Products run on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation.
//
// A training step over n rows:
//   features        X0 = [x, y, s, sin(2 pi B p), cos(2 pi B p), 0...]
//   layer_forward   A_l = silu(A_{l-1} W_l + b_l) (bf16); for the output
//                   layer Y = A W + b, with the MSE gradient dY and the
//                   squared-error partials in the same epilogue
//   backward_and_grad  dZ_{l-1} = (dZ_l W_l^T) silu'(Z_{l-1}), where
//                   Z_{l-1} = A_{l-2} W_{l-1} + b_{l-1} is recomputed with the
//                   forward pass's own instruction sequence (bitwise the
//                   forward value, so Z is never stored)
//                   and in the same grid, per block of rows, A_{l-1}^T dZ_l
//                   and the column sums of dZ_l (the weight and bias
//                   gradient partials)
//   weight_grad     the same partials for the first layer
//   reduce_adam     the row-block partials of every layer summed in a fixed
//                   order, then Adam
// The row-tile kernels keep a layer's weights resident in LDS and read every
// activation row once, which is what these products are bound by: with 128
// features a row, each byte of activations meets 64 multiply-adds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smrt {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round-to-nearest-even binary32 -> bfloat16 bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f_to_bf(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two binary32 values rounded to nearest-even bfloat16 in one v_cvt_pk_bf16_f32,
// a in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

// sigmoid(z) = 1 / (1 + exp(-z)) with the hardware reciprocal (1 ulp)
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// MFMA operand layout (16 x 16 x 32, checked on the device against a host
// product): lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16]
// for i < 8, and receives D[4 (l / 16) + r][l % 16] for r < 4.
__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// General product (the library's GEMM entry point)
// ---------------------------------------------------------------------------

constexpr int TM = 64, TN = 64, TK = 32; // workgroup tile and K step
constexpr int GEMM_THREADS = 256;         // 4 waves, each a 32 x 32 quarter

// C[split][m][n] = sum over this split's k of opA(m, k) * opB(k, n), with
//   opA(m, k) = TA ? A[k * lda + m] : A[m * lda + k]
//   opB(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n],
// bf16 inputs, FP32 accumulation.  The host guarantees M % 64 == 0,
// N % 64 == 0, k_split % 32 == 0, lda % 8 == 0, ldb % 8 == 0 and 16-byte
// aligned A and B; split s covers k in [s * k_split, (s + 1) * k_split) and
// writes at C + s * split_stride.  Grid: (N/64, M/64, splits).
//
// Each K-step stages a 64 x 32 slice of each operand with one 16-byte load
// per thread and operand, kept in LDS in the layout of the stored rows; the
// next slice's loads are issued before the current slice's matrix-core work.
template <bool TA, bool TB>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_bf16(const uint16_t* __restrict__ A,
                                                          const uint16_t* __restrict__ B, float* __restrict__ C,
                                                          int M, int N, int lda, int ldb, int ldc, int k_split,
                                                          int64_t split_stride)
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
        bf16x8 a[2], b[2];
        const int k8 = 8 * (lane >> 4);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const int am = wm + f * 16 + (lane & 15);
            if constexpr (TA) {
#pragma unroll
                for (int i = 0; i < 8; ++i) a[f][i] = __builtin_bit_cast(__bf16, As[k8 + i][am]);
            } else {
                a[f] = *reinterpret_cast<const bf16x8*>(&As[am][k8]);
            }
            const int bn = wn + f * 16 + (lane & 15);
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
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
        __syncthreads();
    }
    float* Cs = C + (int64_t)blockIdx.z * split_stride;
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

// ---------------------------------------------------------------------------
// Training step
// ---------------------------------------------------------------------------

// Input features of a point p = (x, y, s): [x, y, s, sin(2 pi B p), cos(2 pi B p), 0...]
// with B the nf x 3 frequency matrix; written as bf16 rows of `width`
// elements (a multiple of 64, at most kMaxFeatureWidth).  A workgroup builds
// 64 rows, four threads a row: first the sines and cosines into LDS (one
// thread a frequency, so no wave takes both branches), then each thread
// assembles 16-byte pieces of its row and stores them.  Grid: n / 64.
constexpr int kMaxFeatureWidth = 192;
__global__ void __launch_bounds__(256) features(const float* __restrict__ p, const float* __restrict__ Bf, int nf,
                                                int n, int width, uint16_t* __restrict__ X)
{
    constexpr int FS = 2 * 64 + 2; // sines then cosines of one row (at most 64 frequencies)
    __shared__ uint16_t trig[64 * FS];
    const int r = threadIdx.x >> 2, part = threadIdx.x & 3;
    const int64_t row = (int64_t)blockIdx.x * 64 + r;
    const float x = p[row * 3 + 0], y = p[row * 3 + 1], s = p[row * 3 + 2];
    for (int j = part; j < nf; j += 4) {
        const float arg = 6.283185307179586f * (Bf[j * 3 + 0] * x + Bf[j * 3 + 1] * y + Bf[j * 3 + 2] * s);
        float sv, cv;
        sincosf(arg, &sv, &cv); // one argument reduction for both
        trig[r * FS + j] = f_to_bf(sv);
        trig[r * FS + nf + j] = f_to_bf(cv);
    }
    __syncthreads();
    const uint16_t xyz[3] = {f_to_bf(x), f_to_bf(y), f_to_bf(s)};
    for (int c8 = part * 8; c8 < width; c8 += 32) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            uint32_t h[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = c8 + e + u;
                h[u] = c < 3 ? xyz[c] : (c < 3 + 2 * nf ? trig[r * FS + c - 3] : 0u);
            }
            w[e >> 1] = h[0] | (h[1] << 16);
        }
        *reinterpret_cast<u32x4*>(X + row * width + c8) = u32x4{w[0], w[1], w[2], w[3]};
    }
}

constexpr int RT = 64;           // rows of a row tile, 16 per wave
constexpr int KC = 128;          // contraction chunk staged in LDS
constexpr int WS = KC + 8;       // LDS row stride of a staged chunk (elements)
constexpr int ROW_THREADS = 256; // 4 waves

// Stages rows [n0, n0 + bn) x columns [k0, k0 + kc) of a row-major bf16
// matrix with row stride ld into Ws[bn][WS] with 16-byte copies.  The
// 68-word row stride puts the 16 rows one MFMA operand read touches on 16
// distinct groups of four banks.
__device__ __forceinline__ void stage_chunk(uint16_t* Ws, const uint16_t* __restrict__ src, int ld, int n0, int bn,
                                            int k0, int kc)
{
    const int cpr = kc >> 3;
    for (int c = threadIdx.x; c < bn * cpr; c += ROW_THREADS) {
        const int r = c / cpr, k8 = (c - r * cpr) * 8;
        *reinterpret_cast<u32x4*>(Ws + r * WS + k8) =
            *reinterpret_cast<const u32x4*>(src + (int64_t)(n0 + r) * ld + k0 + k8);
    }
}

// The MFMA's second operands for 16 rows of X: lane (r = lane % 16,
// q = lane / 16) reads row m0 + r, elements k0 + 32 kk + 8 q .. + 7 for
// 32 kk < kc (kc a multiple of 32, at most KC).
__device__ __forceinline__ void load_rows(bf16x8 (&xf)[KC / 32], const uint16_t* __restrict__ X, int ldx, int m0,
                                          int k0, int kc)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const uint16_t* xr = X + (int64_t)(m0 + r) * ldx + k0 + 8 * q;
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk)
        if (kk * 32 < kc) xf[kk] = *reinterpret_cast<const bf16x8*>(xr + kk * 32);
}

// acc[j] += the 16 x 16 block (the 16 rows of xf; staged rows 16 j .. 16 j + 15
// of Ws) of X[:, k0 .. k0 + kc) Ws^T.  The staged matrix is the MFMA's first
// operand and X its second, so lane (r, q) receives row m0 + r, columns
// 16 j + 4 q .. 16 j + 4 q + 3: four consecutive outputs of one row.
template <int FJ>
__device__ __forceinline__ void rows_times_staged(f32x4 (&acc)[FJ], const bf16x8 (&xf)[KC / 32], int kc,
                                                  const uint16_t* Ws)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
        if (kk * 32 < kc) {
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const bf16x8 w = *reinterpret_cast<const bf16x8*>(Ws + (16 * j + r) * WS + kk * 32 + 8 * q);
                acc[j] = mfma(w, xf[kk], acc[j]);
            }
        }
    }
}

__device__ __forceinline__ void store_bf16x4(uint16_t* dst, const float (&v)[4])
{
    *reinterpret_cast<uint2*>(dst) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
}

// What layer_forward does with v = (X W)[m][n] + b[n]:
//   FWD_HIDDEN   act[m][n] = bf16(silu(v)), silu(v) = v sigmoid(v)
//   FWD_OUT      y[m][n] = v for n < keep
//   FWD_OUT_MSE  as FWD_OUT, and with e = v - target[m][n]:
//                dy[m][n] = bf16(scale e) (0 for n >= keep) and per
//                workgroup loss[blockIdx.x] = sum of e^2 (FP64)
enum { FWD_HIDDEN = 0, FWD_OUT = 1, FWD_OUT_MSE = 2 };
struct FwdOut {
    uint16_t* act = nullptr;
    float* y = nullptr;
    int keep = 0;
    const float* target = nullptr;
    uint16_t* dy = nullptr;
    float scale = 0.f;
    double* loss = nullptr;
};

// One layer over `tiles` row tiles of 64 rows: X [rows][K], Wt = W^T
// ([N][K], bf16), output columns [BN blockIdx.y, BN (blockIdx.y + 1)).
// K and N are multiples of 64.  Workgroups loop over the row tiles; with
// K <= 128 the weights are staged once and stay resident.
// Grid: (row groups, N / BN); the FWD_OUT modes need N == BN.
template <int BN, int MODE>
__global__ void __launch_bounds__(ROW_THREADS, 3) layer_forward(const uint16_t* __restrict__ X, int K,
                                                             const uint16_t* __restrict__ Wt,
                                                             const float* __restrict__ bias, int N, int tiles,
                                                             FwdOut o)
{
    constexpr int FJ = BN / 16;
    __shared__ __attribute__((aligned(16))) uint16_t Ws[BN * WS];
    __shared__ __attribute__((aligned(16))) float bs[BN];
    __shared__ double lds[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int n0 = blockIdx.y * BN;
    const int chunks = (K + KC - 1) / KC;
    if (threadIdx.x < BN) bs[threadIdx.x] = bias[n0 + threadIdx.x];
    double lsum = 0.0;
    const auto epilogue = [&](const f32x4 (&acc)[FJ], int tile) {
        const int64_t m = tile * RT + wave * 16 + r;
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int n = n0 + 16 * j + 4 * q;
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(&bs[16 * j + 4 * q]);
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[j][i] + b4[i];
                if constexpr (MODE == FWD_HIDDEN) {
                    h[i] = v * sigmoid(v);
                } else {
                    h[i] = 0.f;
                    if (n + i < o.keep) {
                        o.y[m * o.keep + n + i] = v;
                        if constexpr (MODE == FWD_OUT_MSE) {
                            const float e = v - o.target[m * o.keep + n + i];
                            lsum += (double)e * e;
                            h[i] = o.scale * e;
                        }
                    }
                }
            }
            if constexpr (MODE == FWD_HIDDEN) store_bf16x4(o.act + m * N + n, h);
            if constexpr (MODE == FWD_OUT_MSE) store_bf16x4(o.dy + m * N + n, h);
        }
    };
    bf16x8 xf[KC / 32], xn[KC / 32];
    if (chunks == 1) {
        // weights resident; the next tile's rows are in flight during this
        // tile's products and epilogue
        stage_chunk(Ws, Wt, K, n0, BN, 0, K);
        int tile = blockIdx.x;
        if (tile < tiles) load_rows(xf, X, K, tile * RT + wave * 16, 0, K);
        __syncthreads();
        for (; tile < tiles; tile += gridDim.x) {
            const int next = tile + gridDim.x;
            if (next < tiles) load_rows(xn, X, K, next * RT + wave * 16, 0, K);
            f32x4 acc[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            rows_times_staged<FJ>(acc, xf, K, Ws);
            epilogue(acc, tile);
#pragma unroll
            for (int kk = 0; kk < KC / 32; ++kk) xf[kk] = xn[kk];
        }
    } else {
        for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
            f32x4 acc[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int c = 0; c < chunks; ++c) {
                const int k0 = c * KC, kc = min(KC, K - k0);
                __syncthreads();
                stage_chunk(Ws, Wt, K, n0, BN, k0, kc);
                load_rows(xf, X, K, tile * RT + wave * 16, k0, kc);
                __syncthreads();
                rows_times_staged<FJ>(acc, xf, kc, Ws);
            }
            epilogue(acc, tile);
        }
    }
    if constexpr (MODE == FWD_OUT_MSE) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        if (lane == 0) lds[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) o.loss[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    }
}

// The whole forward pass in one launch, for networks whose transposed bf16
// weights fit in LDS together (input width K0, hidden width H, 64 output
// columns).  Each wave takes 16 rows at a time through every layer: the
// layer's sums come from the same operands in the same MFMA order as
// layer_forward's (so the activations, outputs and loss terms are bitwise
// theirs), and the bf16 activations go both to HBM (the backward pass reads
// them) and, through lane permutes, into the MFMA operand layout of the next
// layer: the sums leave lane (r, q) four consecutive columns of row r, the
// next product wants eight.  Every layer's W^T is staged once per workgroup
// (row stride K + 8 elements: the 16 rows one operand read touches land on
// distinct groups of four banks for K = 64 and 128); with the weights filling
// the LDS, a workgroup of 12 waves per CU keeps three waves on every SIMD.
// Rows of the wave's next 16-row block are in flight while the current one
// runs.
// The loss partial of workgroup b goes to o.loss[b].
constexpr int kFusedMaxLayers = 8;
constexpr int kFusedWeightElems = 70144; // 140,288 bytes of LDS
constexpr int kFusedBiasFloats = 1024;
constexpr int FUSED_THREADS = 768;
struct FusedArgs {
    const uint16_t* X0;                      // [rows][K0] input features
    int layers;                              // hidden layers + 1
    const uint16_t* wt[kFusedMaxLayers];     // W_l^T, [N_l][K_l] bf16
    const float* bias[kFusedMaxLayers];      // b_l, N_l floats
    uint16_t* act[kFusedMaxLayers];          // A_l, [rows][H] bf16, hidden layers
    int blocks;                              // rows / 16
    FwdOut o;                                // output layer (N = 64)
    // with the MSE target: W_{L-1} ([H][64] bf16, not transposed) and, when
    // set, dZ_{L-2} = (dY W_{L-1}^T) silu'(Z_{L-2}) into dz_last ([rows][H])
    const uint16_t* w_last;
    uint16_t* dz_last;
};

// LDS elements of the packed transposed weights of such a network
constexpr int fused_weight_elems(int k0, int h, int layers)
{
    return h * (k0 + 8) + (layers - 2) * h * (h + 8) + 64 * (h + 8);
}

// acc[j] += the 16 x 16 block of X Ws^T (staged rows 16 j .. 16 j + 15,
// row stride LD) for the K columns held in xf; the operand order of
// rows_times_staged.
template <int FJ, int K, int LD>
__device__ __forceinline__ void rows_times_resident(f32x4 (&acc)[FJ], const bf16x8 (&xf)[KC / 32],
                                                    const uint16_t* Ws)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < K / 32; ++kk) {
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const bf16x8 w = *reinterpret_cast<const bf16x8*>(Ws + (16 * j + r) * LD + kk * 32 + 8 * q);
            acc[j] = mfma(w, xf[kk], acc[j]);
        }
    }
}

// Lane (r, q) holds pk[j] = bf16 columns 16 j + 4 q .. + 3 of row r; returns
// in xf[kk] columns 32 kk + 8 q .. + 7: the first four from lane group
// 2q mod 4, the next four from 2q + 1 mod 4, of column block j = 2 kk + q / 2.
template <int FJ>
__device__ __forceinline__ void regroup_rows(const uint2 (&pk)[FJ], bf16x8 (&xf)[KC / 32])
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int src_a = (r + 16 * ((2 * q) & 3)) * 4, src_b = (r + 16 * ((2 * q + 1) & 3)) * 4;
    const bool upper = q >= 2;
    const auto take = [&](int src, uint32_t lo, uint32_t hi) {
        const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)lo);
        const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)hi);
        return upper ? b : a;
    };
#pragma unroll
    for (int kk = 0; kk < FJ / 2; ++kk) {
        const uint2 e = pk[2 * kk], o = pk[2 * kk + 1];
        const u32x4 v{take(src_a, e.x, o.x), take(src_a, e.y, o.y), take(src_b, e.x, o.x), take(src_b, e.y, o.y)};
        xf[kk] = __builtin_bit_cast(bf16x8, v);
    }
}

template <int K0, int H, int MODE>
__global__ void __launch_bounds__(FUSED_THREADS, 1) forward_fused(FusedArgs a)
{
    static_assert(K0 % 64 == 0 && K0 <= KC && (H == 64 || H == 128), "fused forward shapes");
    constexpr int FJ = H / 16, WAVES = FUSED_THREADS / 64;
    constexpr bool MSE = MODE == FWD_OUT_MSE;
    __shared__ __attribute__((aligned(16))) uint16_t Ws[kFusedWeightElems];
    __shared__ __attribute__((aligned(16))) float bs[kFusedBiasFloats];
    __shared__ __attribute__((aligned(16))) uint16_t Wl[MSE ? H * 72 : 8]; // W_{L-1}, row stride 72
    __shared__ double lds[WAVES];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int L = a.layers;
    const bool dz = MSE && a.dz_last != nullptr;
    // stage every layer's W^T and bias
    {
        int off = 0;
        for (int l = 0; l < L; ++l) {
            const int K = l == 0 ? K0 : H, N = l == L - 1 ? 64 : H, cpr = K >> 3;
            for (int c = threadIdx.x; c < N * cpr; c += FUSED_THREADS) {
                const int row = c / cpr, k8 = (c - row * cpr) * 8;
                *reinterpret_cast<u32x4*>(Ws + off + row * (K + 8) + k8) =
                    *reinterpret_cast<const u32x4*>(a.wt[l] + (int64_t)row * K + k8);
            }
            for (int c = threadIdx.x; c < N; c += FUSED_THREADS) bs[l * 128 + c] = a.bias[l][c];
            off += N * (K + 8);
        }
        if constexpr (MSE) {
            if (dz)
                for (int c = threadIdx.x; c < H * 8; c += FUSED_THREADS) {
                    const int row = c >> 3, k8 = (c & 7) * 8;
                    *reinterpret_cast<u32x4*>(Wl + row * 72 + k8) =
                        *reinterpret_cast<const u32x4*>(a.w_last + (int64_t)row * 64 + k8);
                }
        }
    }
    __syncthreads();
    double lsum = 0.0;
    bf16x8 xf[KC / 32], xn[KC / 32];
    // blocks blockIdx.x + gridDim.x t, t = wave, wave + WAVES, ...: every
    // workgroup gets the same number of blocks, spread over its SIMDs
    const int stride = gridDim.x * WAVES;
    int b = blockIdx.x + gridDim.x * wave;
    if (b < a.blocks) load_rows(xf, a.X0, K0, b * 16, 0, K0);
    for (; b < a.blocks; b += stride) {
        if (b + stride < a.blocks) load_rows(xn, a.X0, K0, (b + stride) * 16, 0, K0);
        const int64_t m = (int64_t)b * 16 + r;
        const uint16_t* W = Ws;
        f32x4 zl[MSE ? FJ : 1]; // the last hidden layer's pre-activations
        for (int l = 0; l < L - 1; ++l) {
            f32x4 acc[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (l == 0) {
                rows_times_resident<FJ, K0, K0 + 8>(acc, xf, W);
                W += H * (K0 + 8);
            } else {
                rows_times_resident<FJ, H, H + 8>(acc, xf, W);
                W += H * (H + 8);
            }
            uint16_t* act = a.act[l];
            uint2 pk[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const int n = 16 * j + 4 * q;
                const f32x4 b4 = *reinterpret_cast<const f32x4*>(&bs[l * 128 + n]);
                float h[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[j][i] + b4[i];
                    h[i] = v * sigmoid(v);
                    if constexpr (MSE) zl[j][i] = v; // kept from the last hidden layer
                }
                pk[j] = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
                *reinterpret_cast<uint2*>(act + m * H + n) = pk[j];
            }
            regroup_rows<FJ>(pk, xf);
        }
        f32x4 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        rows_times_resident<4, H, H + 8>(acc, xf, W);
        uint2 pdy[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = 16 * j + 4 * q;
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(&bs[(L - 1) * 128 + n]);
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[j][i] + b4[i];
                h[i] = 0.f;
                if (n + i < a.o.keep) {
                    a.o.y[m * a.o.keep + n + i] = v;
                    if constexpr (MSE) {
                        const float e = v - a.o.target[m * a.o.keep + n + i];
                        lsum += (double)e * e;
                        h[i] = a.o.scale * e;
                    }
                }
            }
            if constexpr (MSE) {
                pdy[j] = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
                *reinterpret_cast<uint2*>(a.o.dy + m * 64 + n) = pdy[j];
            }
        }
        if constexpr (MSE) {
            if (dz) {
                // the output layer's input gradient, with the backward pass's
                // operands in its order: g = dY W_{L-1}^T from the bf16 dY,
                // then dZ = g s (1 + z (1 - s)), s = sigmoid(z)
                bf16x8 xg[KC / 32];
                regroup_rows<4>(pdy, xg);
                f32x4 g[FJ];
#pragma unroll
                for (int j = 0; j < FJ; ++j) g[j] = f32x4{0.f, 0.f, 0.f, 0.f};
                rows_times_resident<FJ, 64, 72>(g, xg, Wl);
#pragma unroll
                for (int j = 0; j < FJ; ++j) {
                    float h[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float zz = zl[j][i], s = sigmoid(zz);
                        h[i] = g[j][i] * s * (1.0f + zz * (1.0f - s));
                    }
                    store_bf16x4(a.dz_last + m * H + 16 * j + 4 * q, h);
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC / 32; ++kk) xf[kk] = xn[kk];
    }
    if constexpr (MODE == FWD_OUT_MSE) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        if (lane == 0) lds[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < WAVES; ++w) t += lds[w];
            a.o.loss[blockIdx.x] = t;
        }
    }
}

// Input gradient of layer l over `tiles` row tiles, output columns
// [BN blockIdx.y, BN (blockIdx.y + 1)) of K:
//   dZout[m][n] = bf16(g silu'(z)),  g = (dZ W_l^T)[m][n],
//   z = (Xp W_{l-1})[m][n] + bp[n],  silu'(z) = s (1 + z (1 - s)), s = sigmoid(z)
// with dZ [rows][N], W = W_l ([K][N] bf16), Xp = A_{l-2} or X0 ([rows][Kp]),
// Wpt = W_{l-1}^T ([K][Kp] bf16).  z is accumulated exactly as layer_forward
// accumulated it (same chunks, same operand order).  Grid: (row groups, K / BN).
struct BackArgs {
    const uint16_t* dZ;
    int N;
    const uint16_t* W;
    const uint16_t* Xp;
    int Kp;
    const uint16_t* Wpt;
    const float* bp;
    int K, tiles;
    uint16_t* dZout;
};

// The input-gradient tiles of workgroup (bx, by) of a (gx, K / BN) grid,
// with its LDS: Wz and Wg BN x WS elements each, bs BN floats.
template <int BN>
__device__ __forceinline__ void backward_tiles(const BackArgs& a, int bx, int by, int gx, uint16_t* Wz, uint16_t* Wg,
                                               float* bs)
{
    const uint16_t* __restrict__ dZ = a.dZ;
    const uint16_t* __restrict__ W = a.W;
    const uint16_t* __restrict__ Xp = a.Xp;
    const uint16_t* __restrict__ Wpt = a.Wpt;
    const float* __restrict__ bp = a.bp;
    uint16_t* __restrict__ dZout = a.dZout;
    const int N = a.N, Kp = a.Kp, K = a.K, tiles = a.tiles;
    constexpr int FJ = BN / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int n0 = by * BN;
    const int cz = (Kp + KC - 1) / KC, cg = (N + KC - 1) / KC;
    if (threadIdx.x < BN) bs[threadIdx.x] = bp[n0 + threadIdx.x];
    const auto epilogue = [&](const f32x4 (&z)[FJ], const f32x4 (&g)[FJ], int tile) {
        const int64_t m = tile * RT + wave * 16 + r;
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int n = n0 + 16 * j + 4 * q;
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(&bs[16 * j + 4 * q]);
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float zz = z[j][i] + b4[i], s = sigmoid(zz);
                h[i] = g[j][i] * s * (1.0f + zz * (1.0f - s));
            }
            store_bf16x4(dZout + m * K + n, h);
        }
    };
    bf16x8 xz[KC / 32], xg[KC / 32];
    if (cz == 1 && cg == 1) {
        // both weight blocks resident; the next tile's rows are in flight
        // during this tile's products and epilogue
        bf16x8 nz[KC / 32], ng[KC / 32];
        stage_chunk(Wz, Wpt, Kp, n0, BN, 0, Kp);
        stage_chunk(Wg, W, N, n0, BN, 0, N);
        int tile = bx;
        if (tile < tiles) {
            load_rows(xz, Xp, Kp, tile * RT + wave * 16, 0, Kp);
            load_rows(xg, dZ, N, tile * RT + wave * 16, 0, N);
        }
        __syncthreads();
        for (; tile < tiles; tile += gx) {
            const int next = tile + gx;
            if (next < tiles) {
                load_rows(nz, Xp, Kp, next * RT + wave * 16, 0, Kp);
                load_rows(ng, dZ, N, next * RT + wave * 16, 0, N);
            }
            f32x4 z[FJ], g[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) z[j] = g[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            rows_times_staged<FJ>(z, xz, Kp, Wz);
            rows_times_staged<FJ>(g, xg, N, Wg);
            epilogue(z, g, tile);
#pragma unroll
            for (int kk = 0; kk < KC / 32; ++kk) {
                xz[kk] = nz[kk];
                xg[kk] = ng[kk];
            }
        }
    } else {
        for (int tile = bx; tile < tiles; tile += gx) {
            const int m0 = tile * RT + wave * 16;
            f32x4 z[FJ], g[FJ];
#pragma unroll
            for (int j = 0; j < FJ; ++j) z[j] = g[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int c = 0; c < cz; ++c) {
                const int k0 = c * KC, kc = min(KC, Kp - k0);
                __syncthreads();
                stage_chunk(Wz, Wpt, Kp, n0, BN, k0, kc);
                load_rows(xz, Xp, Kp, m0, k0, kc);
                __syncthreads();
                rows_times_staged<FJ>(z, xz, kc, Wz);
            }
            for (int c = 0; c < cg; ++c) {
                const int k0 = c * KC, kc = min(KC, N - k0);
                __syncthreads();
                stage_chunk(Wg, W, N, n0, BN, k0, kc);
                load_rows(xg, dZ, N, m0, k0, kc);
                __syncthreads();
                rows_times_staged<FJ>(g, xg, kc, Wg);
            }
            epilogue(z, g, tile);
        }
    }
}


// Row-block partials of a layer's gradient: for split s (rows
// [s rps, (s + 1) rps), rps a multiple of 64), output tile (m, n) of
//   part[s][m][n] = sum over the block's rows r of X[r][m] dZ[r][n]
// with X [rows][M], dZ [rows][N] (bf16), and from the workgroups of the
// first row of tiles part[s][M N + n] = sum over the rows of dZ[r][n] (the
// bias gradient's partial), in row order.  Split s writes at
// part + s * split_stride.  Grid: (N / BN, M / BM, splits).
//
// Each 64-row slice of X and dZ is staged transposed, as row pairs packed in
// 32-bit words (word j of column c holds rows 2j and 2j + 1 of column c), so
// an MFMA operand -- eight consecutive rows of one column -- is one 16-byte
// LDS read; the 36-word column stride spreads the 16 columns one read
// touches over all banks.  Two buffers: the next slice's loads (eight
// 16-byte loads a thread) are in flight during the current slice's
// products, with one barrier a slice.
constexpr int WG_ROWS = 64;
struct GradArgs {
    const uint16_t* X;
    const uint16_t* dZ;
    int M, N, rps;
    float* part;
    int64_t split_stride;
};

template <int BM, int BN> struct GradLds {
    static constexpr int RS = WG_ROWS / 2 + 4; // words per staged column
    uint32_t Xt[2][BM * RS];
    uint32_t Dt[2][BN * RS];
    float dbh[2][BN];
};

// The weight-gradient partials of block (bx, by, bz) of a (N / BN, M / BM, splits) grid.
template <int BM, int BN>
__device__ __forceinline__ void grad_partials(const GradArgs& a, int bx, int by, int bz, GradLds<BM, BN>& L)
{
    const uint16_t* __restrict__ X = a.X;
    const uint16_t* __restrict__ dZ = a.dZ;
    float* __restrict__ part = a.part;
    const int M = a.M, N = a.N, rps = a.rps;
    const int64_t split_stride = a.split_stride;
    constexpr int RS = GradLds<BM, BN>::RS;
    constexpr int FI = BM / 32, FJ = BN / 32;
    auto& Xt = L.Xt;
    auto& Dt = L.Dt;
    auto& dbh = L.dbh;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
    const int m0 = by * BM, n0 = bx * BN;
    const int64_t r0 = (int64_t)bz * rps;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    // loader: row pairs j and j + 16, columns c8 .. c8 + 7 of the tile
    const int j = tid & 15, c8 = (tid >> 4) * 8;
    const bool lx = c8 < BM, ldz = c8 < BN;
    const bool db_blk = by == 0;
    const int dn = tid % BN, dh = tid / BN; // bias-gradient column and half of the slice's rows
    u32x4 xa[2], xb[2], da[2], db[2];
    const auto load = [&](int s) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t row = r0 + WG_ROWS * s + 2 * (j + 16 * h);
            if (lx) {
                xa[h] = *reinterpret_cast<const u32x4*>(X + row * M + m0 + c8);
                xb[h] = *reinterpret_cast<const u32x4*>(X + (row + 1) * M + m0 + c8);
            }
            if (ldz) {
                da[h] = *reinterpret_cast<const u32x4*>(dZ + row * N + n0 + c8);
                db[h] = *reinterpret_cast<const u32x4*>(dZ + (row + 1) * N + n0 + c8);
            }
        }
    };
    // word jj of column c8 + e = (row 2jj element e) | (row 2jj + 1 element e) << 16
    const auto put = [&](uint32_t* T, const u32x4 (&a)[2], const u32x4 (&b)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                T[(c8 + 2 * w) * RS + j + 16 * h] = (a[h][w] & 0xffffu) | (b[h][w] << 16);
                T[(c8 + 2 * w + 1) * RS + j + 16 * h] = (a[h][w] >> 16) | (b[h][w] & 0xffff0000u);
            }
    };
    f32x4 acc[FI][FJ];
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fj = 0; fj < FJ; ++fj) acc[fi][fj] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dsum = 0.f;
    const int steps = rps / WG_ROWS;
    load(0);
    for (int s = 0; s < steps; ++s) {
        const int b = s & 1;
        if (lx) put(Xt[b], xa, xb);
        if (ldz) put(Dt[b], da, db);
        __syncthreads();
        if (s + 1 < steps) load(s + 1);
        if (db_blk && tid < 2 * BN) {
#pragma unroll
            for (int w = 0; w < WG_ROWS / 4; ++w) {
                const uint32_t v = Dt[b][dn * RS + (WG_ROWS / 4) * dh + w];
                dsum += bf_to_f((uint16_t)(v & 0xffffu));
                dsum += bf_to_f((uint16_t)(v >> 16));
            }
        }
#pragma unroll
        for (int kk = 0; kk < WG_ROWS / 32; ++kk) {
            bf16x8 xf[FI], df[FJ];
#pragma unroll
            for (int fi = 0; fi < FI; ++fi)
                xf[fi] = *reinterpret_cast<const bf16x8*>(&Xt[b][(wm + 16 * fi + r) * RS + 16 * kk + 4 * q]);
#pragma unroll
            for (int fj = 0; fj < FJ; ++fj)
                df[fj] = *reinterpret_cast<const bf16x8*>(&Dt[b][(wn + 16 * fj + r) * RS + 16 * kk + 4 * q]);
            // dZ as the first operand: lane (r, q) receives row m = wm + 16 fi + r,
            // columns n = wn + 16 fj + 4 q .. + 3
#pragma unroll
            for (int fi = 0; fi < FI; ++fi)
#pragma unroll
                for (int fj = 0; fj < FJ; ++fj) acc[fi][fj] = mfma(df[fj], xf[fi], acc[fi][fj]);
        }
    }
    float* Cs = part + (int64_t)bz * split_stride;
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fj = 0; fj < FJ; ++fj) {
            const int64_t m = m0 + wm + 16 * fi + r;
            const int n = n0 + wn + 16 * fj + 4 * q;
            *reinterpret_cast<f32x4*>(Cs + m * N + n) = acc[fi][fj];
        }
    if (db_blk) { // uniform over the workgroup
        if (tid < 2 * BN) dbh[dh][dn] = dsum;
        __syncthreads();
        if (tid < BN) Cs[(int64_t)M * N + n0 + tid] = dbh[0][tid] + dbh[1][tid];
    }
}


template <int BM, int BN>
__global__ void __launch_bounds__(ROW_THREADS) weight_grad(GradArgs a)
{
    __shared__ __attribute__((aligned(16))) GradLds<BM, BN> L;
    grad_partials<BM, BN>(a, blockIdx.x, blockIdx.y, blockIdx.z, L);
}

// An input-gradient layer and the weight-gradient partials of the same
// layer in one grid: both read dZ_l and neither waits on the other, and both
// are bound by memory latency, so sharing CUs overlaps their waits.  The
// two kinds of workgroup are spread evenly over the grid; the LDS is one
// buffer that each role lays out for itself.  nb = gx_back x gy_back input-gradient workgroups (gx_back
// row groups), ng = gx x gy x gz gradient workgroups.
template <int BN, int BM2, int BN2>
__global__ void __launch_bounds__(ROW_THREADS, 2) backward_and_grad(BackArgs ba, int gx_back, int gy_back, GradArgs ga,
                                                                 int gx, int gy, int gz)
{
    constexpr size_t kBack = 2 * BN * WS * sizeof(uint16_t) + BN * sizeof(float);
    constexpr size_t kGrad = sizeof(GradLds<BM2, BN2>);
    __shared__ __attribute__((aligned(16))) unsigned char smem[kBack > kGrad ? kBack : kGrad];
    const int64_t nb = gx_back * gy_back, ng = gx * gy * gz, T = nb + ng;
    const int64_t b = blockIdx.x;
    // the ng gradient workgroups spread evenly over the grid: workgroup b is
    // one when floor((b + 1) ng / T) steps up; it is then gradient workgroup
    // floor(b ng / T), otherwise input-gradient workgroup b - floor(b ng / T)
    const int64_t before = b * ng / T;
    const bool is_grad = (b + 1) * ng / T > before;
    const int back = is_grad ? -1 : (int)(b - before), grad = is_grad ? (int)before : -1;
    if (back >= 0 && back < nb) {
        uint16_t* Wz = reinterpret_cast<uint16_t*>(smem);
        uint16_t* Wg = Wz + BN * WS;
        float* bs = reinterpret_cast<float*>(Wg + BN * WS);
        backward_tiles<BN>(ba, back % gx_back, back / gx_back, gx_back, Wz, Wg, bs);
    } else if (grad >= 0 && grad < ng) {
        grad_partials<BM2, BN2>(ga, grad % gx, (grad / gx) % gy, grad / (gx * gy),
                                *reinterpret_cast<GradLds<BM2, BN2>*>(smem));
    }
}

// Parameter blocks of the layers in the padded parameter vector: layer l's
// W (in[l] x out[l], row-major) starts at off[l], its b right after;
// off[layers] is the total.
constexpr int kMaxLayers = 16;
struct LayerTable {
    int layers = 0;
    int64_t off[kMaxLayers + 1] = {};
    int in[kMaxLayers] = {}, out[kMaxLayers] = {};
};

__device__ __forceinline__ int layer_of(const LayerTable& T, int64_t i)
{
    int l = 0;
    while (l + 1 < T.layers && i >= T.off[l + 1]) ++l;
    return l;
}

// bf16 copies of the FP32 parameters: wbf[i] for every entry, and for the
// weights also wbf_t at the transposed place (layer l's W^T, [out][in], in
// the same block).
__device__ __forceinline__ void write_bf16(const LayerTable& T, int l, int64_t i, float v, uint16_t* wbf,
                                           uint16_t* wbf_t)
{
    const uint16_t h = f_to_bf(v);
    wbf[i] = h;
    const int64_t o = i - T.off[l];
    if (o < (int64_t)T.in[l] * T.out[l]) {
        const int k = (int)(o / T.out[l]), n = (int)(o - (int64_t)k * T.out[l]);
        wbf_t[T.off[l] + (int64_t)n * T.in[l] + k] = h;
    }
}

__global__ void weights_to_bf16(const float* __restrict__ w, LayerTable T, uint16_t* __restrict__ wbf,
                                uint16_t* __restrict__ wbf_t)
{
    const int64_t total = T.off[T.layers];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        write_bf16(T, layer_of(T, i), i, w[i], wbf, wbf_t);
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master parameters with
// bias-corrected step size lr_t, refreshing both bf16 copies.
struct AdamArgs {
    float* w = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float lr_t = 0.f;
    uint16_t* wbf = nullptr;
    uint16_t* wbf_t = nullptr;
};

// g[i] = sum over the S row-block partials of parameter i: the splits in
// sixteen consecutive groups, each summed in split order, the group sums
// added in group order (independent of scheduling).  Layer l's partials sit
// at part + S off[l] + s (off[l + 1] - off[l]) + (i - off[l]).  Without Adam
// (a.w null) grad[i] = g; with it, Adam updates parameter i.  A workgroup of
// 256 threads takes 64 parameters of [i0, i1) (i0, i1 and every layer's
// offset multiples of 64): 16 lanes cover them with 16-byte loads, so each
// wave holds four groups and every load instruction reads four partials.
constexpr int RED_PARAMS = 64, RED_GROUPS = 16, REDUCE_THREADS = 256;
struct ReduceArgs {
    const float* part;
    int S;
    LayerTable T;
    float* grad;
    AdamArgs a;
    int64_t i0, i1;
};

__global__ void __launch_bounds__(REDUCE_THREADS) reduce_adam(ReduceArgs r)
{
    __shared__ __attribute__((aligned(16))) float gs[RED_GROUPS][RED_PARAMS];
    const int c = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const LayerTable& T = r.T;
    const int S = r.S;
    const int64_t base = r.i0 + (int64_t)blockIdx.x * RED_PARAMS;
    const int64_t i4 = base + 4 * c;
    f32x4 s{0.f, 0.f, 0.f, 0.f};
    if (i4 < r.i1) {
        const int l = layer_of(T, i4);
        const int64_t wb = T.off[l + 1] - T.off[l];
        const float* p = r.part + (int64_t)S * T.off[l] + (i4 - T.off[l]);
        const int per = (S + RED_GROUPS - 1) / RED_GROUPS, s0 = grp * per, s1 = min(S, s0 + per);
        // eight loads in flight, then added in split order
        for (int k = s0; k < s1; k += 8) {
            f32x4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = k + u < s1 ? *reinterpret_cast<const f32x4*>(p + (int64_t)(k + u) * wb) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k + u < s1) s += v[u];
        }
    }
    *reinterpret_cast<f32x4*>(&gs[grp][4 * c]) = s;
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t i = base + t;
    if (t >= RED_PARAMS || i >= r.i1) return;
    float gi = gs[0][t];
#pragma unroll
    for (int g = 1; g < RED_GROUPS; ++g) gi += gs[g][t];
    const AdamArgs& a = r.a;
    if (!a.w) {
        r.grad[i] = gi;
        return;
    }
    const float mi = 0.9f * a.m[i] + 0.1f * gi;
    const float vi = 0.999f * a.v[i] + 0.001f * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float wi = a.w[i] - a.lr_t * mi / (sqrtf(vi) + 1e-8f);
    a.w[i] = wi;
    write_bf16(T, layer_of(T, i), i, wi, a.wbf, a.wbf_t);
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
