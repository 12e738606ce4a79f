// moment_kernels.hpp -- SmrtLBM with the post-collision state stored as its
// moments.
//
// Eq. (SmrtLBM-1) makes the post-collision populations of a node a function
// of five numbers: f*_a = f^eq_a(rho, u) + (-1)^a g_grp(a), g_1 = (1 - 1/tau) C_1
// over the axis links (a = 1..4), g_2 = (1 - 1/tau) C_2 over the diagonal links
// (a = 5..8), f*_0 = f^eq_0.  Storing (rho - 1, j = rho u, g_1, g_2) is therefore
// an exact rewrite of the SmrtLBM state, and it separates the large
// equilibrium part, kept in binary32 (or FP64), from the small non-equilibrium
// amplitudes, which carry the viscous stress and can be held in 16 bits with
// their own relative precision (FP16 scaled by 2^12, or bfloat16).  Per node:
// 3 x 4 B + 2 x 2 B = 16 B, against 36 B for nine 16-bit populations.
//
// One step per launch.  A workgroup stages its TX x TY tile plus a one-node
// ring in LDS as (A = drho - 3/2 j.u, j, u, g_1, g_2); each node then rebuilds
// the nine populations it pulls, f*_a(x - e_a) - w_a
//   = w_a (A + (e_a.j)(3 + 9/2 e_a.u)) + (-1)^a g_grp(a)   (deviation form of Eq. feq-full),
// from its neighbours' moments (its own, for a link whose source lies beyond
// a cavity wall: half-way bounce-back, plus the moving-lid term), forms the
// new moments and group sums (Eq. fea-0, Eq. sigma1-2-0) and stores the five
// numbers.  Only SmrtLBM has a five-number post-collision state.
#pragma once

#include "lbm_kernels.hpp"

namespace smrt {

// Element type of a moment-storage buffer: planes 0..2 hold drho, j_x, j_y
// (type MT), then two amplitude planes g_1, g_2 of type H with the same element
// count per plane.
template <typename MT, typename H> struct MomStore {
    MT v;
};
using m64 = MomStore<double, double>;  // FP64 throughout (the exact rewrite, for checks)
using m16 = MomStore<float, _Float16>; // binary32 moments, FP16 amplitudes (x 2^12)
using mbf16 = MomStore<float, bf16>;   // binary32 moments, bfloat16 amplitudes

// Amplitude conversions.  FP16 holds g * 2^12: amplitudes from 1.5e-8 to 16
// sit in its normal range (a cavity's stay within 1e-7 .. 1e-1 of the lid
// speed 0.1), so the only rounding is FP16's own (relative 2^-11).
template <typename H> struct Amp;
template <> struct Amp<double> {
    static __device__ __forceinline__ double load(const double* p) { return *p; }
    static __device__ __forceinline__ void store(double* p, double v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ double to_f64(const double* p) { return *p; }
    static __device__ __forceinline__ void from_f64(double* p, double v) { *p = v; }
};
template <> struct Amp<_Float16> {
    static __device__ __forceinline__ float load(const _Float16* p) { return (float)*p * (1.0f / 4096.0f); }
    static __device__ __forceinline__ void store(_Float16* p, float v)
    {
        __builtin_nontemporal_store((_Float16)(v * 4096.0f), p);
    }
    static __device__ __forceinline__ double to_f64(const _Float16* p) { return (double)((float)*p * (1.0f / 4096.0f)); }
    static __device__ __forceinline__ void from_f64(_Float16* p, double v) { *p = (_Float16)((float)v * 4096.0f); }
};
template <> struct Amp<bf16> {
    static __device__ __forceinline__ float load(const bf16* p) { return bf16_to_f32(p->bits); }
    static __device__ __forceinline__ void store(bf16* p, float v) { __builtin_nontemporal_store(f32_to_bf16(v), &p->bits); }
    static __device__ __forceinline__ double to_f64(const bf16* p) { return (double)bf16_to_f32(p->bits); }
    static __device__ __forceinline__ void from_f64(bf16* p, double v) { p->bits = f32_to_bf16((float)v); }
};

template <typename MS> struct MomPlanes;
template <typename MT_, typename H_> struct MomPlanes<MomStore<MT_, H_>> {
    using MT = MT_;
    using H = H_;
    using C = MT; // arithmetic: FP64 for m64, binary32 otherwise
    using S = MomStore<MT, H>;
    static __device__ __forceinline__ const MT* m(const S* p, int64_t plane, int k)
    {
        return reinterpret_cast<const MT*>(p) + (int64_t)k * plane;
    }
    static __device__ __forceinline__ MT* m(S* p, int64_t plane, int k) { return reinterpret_cast<MT*>(p) + (int64_t)k * plane; }
    static __device__ __forceinline__ const H* g(const S* p, int64_t plane, int k)
    {
        return reinterpret_cast<const H*>(reinterpret_cast<const MT*>(p) + 3 * plane) + (int64_t)k * plane;
    }
    static __device__ __forceinline__ H* g(S* p, int64_t plane, int k)
    {
        return reinterpret_cast<H*>(reinterpret_cast<MT*>(p) + 3 * plane) + (int64_t)k * plane;
    }
};

// (-1)^a for a >= 1, and the group of each link (0: axis, 1: diagonal).
__device__ constexpr int SGN[9] = {0, -1, 1, -1, 1, -1, 1, -1, 1};
__device__ constexpr int GRP[9] = {0, 0, 0, 0, 0, 1, 1, 1, 1};

template <typename C> __device__ __forceinline__ C link_weight(int a)
{
    return a == 0 ? C(4.0 / 9.0) : (a <= 4 ? W<C>::axis : W<C>::diag);
}

// Staged quantities of the tile plus its ring, in LDS.
template <typename C, int FX, int FY> struct MomTile {
    C A[FY][FX], jx[FY][FX], jy[FY][FX], ux[FY][FX], uy[FY][FX], g[2][FY][FX];
};

// Population b of the staged node (px, py), as a deviation from w_b.
template <typename C, int FX, int FY>
__device__ __forceinline__ C rebuild(const MomTile<C, FX, FY>& t, int b, int px, int py)
{
    const C ej = C(EX[b]) * t.jx[py][px] + C(EY[b]) * t.jy[py][px];
    const C eu = C(EX[b]) * t.ux[py][px] + C(EY[b]) * t.uy[py][px];
    const C s = link_weight<C>(b) * (t.A[py][px] + ej * (C(3) + C(4.5) * eu));
    return s + C(SGN[b]) * t.g[GRP[b]][py][px];
}

// One SmrtLBM time step on moment storage.  Grid: tiles_x * tiles_y
// workgroups of TX * TY threads in row-major tile order, one node a thread.
template <typename MS, int BC, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) stream_collide_mom(const MS* __restrict__ src, MS* __restrict__ dst, Geom g,
                                                              Coef<typename MomPlanes<MS>::C> k)
{
    using P = MomPlanes<MS>;
    using C = typename P::C;
    using H = typename P::H;
    constexpr int NT = TX * TY, FX = TX + 2, FY = TY + 2;
    __shared__ MomTile<C, FX, FY> t;
    const int tile = blockIdx.x;
    const int X0 = (tile % g.tiles_x) * TX, Y0 = (tile / g.tiles_x) * TY;
    // stage the tile and its ring; a periodic ring wraps once, and again (by
    // a remainder) only on lattices narrower or lower than a tile, where one
    // wrap can leave the lattice
    for (int i = threadIdx.x; i < FX * FY; i += NT) {
        const int lx = i % FX, ly = i / FX;
        int x = X0 - 1 + lx, y = Y0 - 1 + ly;
        if constexpr (BC == PERIODIC) {
            x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
            y = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
            if ((unsigned)x >= (unsigned)g.nx) x = ((x % g.nx) + g.nx) % g.nx;
            if ((unsigned)y >= (unsigned)g.ny) y = ((y % g.ny) + g.ny) % g.ny;
        } else if ((unsigned)x >= (unsigned)g.nx || (unsigned)y >= (unsigned)g.ny) {
            continue; // beyond a wall or the last tile: never read
        }
        const int64_t off = (int64_t)y * g.pitch + x;
        const C drho = (C)P::m(src, g.plane, 0)[off];
        const C jx = (C)P::m(src, g.plane, 1)[off], jy = (C)P::m(src, g.plane, 2)[off];
        const C inv = reciprocal(C(1) + drho);
        const C ux = jx * inv, uy = jy * inv;
        t.A[ly][lx] = drho - C(1.5) * (jx * ux + jy * uy);
        t.jx[ly][lx] = jx;
        t.jy[ly][lx] = jy;
        t.ux[ly][lx] = ux;
        t.uy[ly][lx] = uy;
        t.g[0][ly][lx] = (C)Amp<H>::load(P::g(src, g.plane, 0) + off);
        t.g[1][ly][lx] = (C)Amp<H>::load(P::g(src, g.plane, 1) + off);
    }
    __syncthreads();
    const int lx = threadIdx.x % TX + 1, ly = threadIdx.x / TX + 1;
    const int x = X0 + lx - 1, y = Y0 + ly - 1;
    if (x >= g.nx || y >= g.ny) return;
    // pull (streaming, walls, lid)
    C d[9];
    d[0] = link_weight<C>(0) * t.A[ly][lx];
    const bool edge = BC == CAVITY && ((x == 0) | (x == g.nx - 1) | (y == 0) | (y == g.ny - 1));
    if (!edge) {
#pragma unroll
        for (int a = 1; a < 9; ++a) d[a] = rebuild(t, a, lx - EX[a], ly - EY[a]);
    } else {
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int sx = x - EX[a], sy = y - EY[a];
            if ((unsigned)sx < (unsigned)g.nx && (unsigned)sy < (unsigned)g.ny)
                d[a] = rebuild(t, a, lx - EX[a], ly - EY[a]);
            else // half-way bounce-back of the node's own opposite population
                d[a] = rebuild(t, OPP[a], lx, ly) + (sy == g.ny ? C(EX[a]) * k.lid : C(0));
        }
    }
    // moments (Eq. fea-0) and the group sums of Eq. (sigma1-2-0) times 4:
    // sum_k (-1)^k (f_k - f^eq_k), whose equilibrium share is
    // 2 (s_y - s_x) = j_y u_y - j_x u_x over the axis links and
    // 2 (s_6 - s_5) = -j_x u_y over the diagonal ones
    const C p13 = d[1] + d[3], p24 = d[2] + d[4], p57 = d[5] + d[7], p68 = d[6] + d[8];
    const C m13 = d[1] - d[3], m24 = d[2] - d[4], m57 = d[5] - d[7], m68 = d[6] - d[8];
    const C drho = d[0] + ((p13 + p24) + (p57 + p68));
    const C jx = m13 + (m57 - m68);
    const C jy = m24 + (m57 + m68);
    const C inv = reciprocal(C(1) + drho);
    const C ux = jx * inv, uy = jy * inv;
    const C c1x4 = (p24 - p13) - (jy * uy - jx * ux);
    const C c2x4 = (p68 - p57) + jx * uy;
    // Eq. (SmrtLBM-1): the post-collision amplitudes (1 - 1/tau) C_1, C_2;
    // density and momentum pass through the collision unchanged
    const C qa = C(0.25) * k.a;
    const int64_t off = (int64_t)y * g.pitch + x;
    __builtin_nontemporal_store((typename P::MT)drho, P::m(dst, g.plane, 0) + off);
    __builtin_nontemporal_store((typename P::MT)jx, P::m(dst, g.plane, 1) + off);
    __builtin_nontemporal_store((typename P::MT)jy, P::m(dst, g.plane, 2) + off);
    Amp<H>::store(P::g(dst, g.plane, 0) + off, qa * c1x4);
    Amp<H>::store(P::g(dst, g.plane, 1) + off, qa * c2x4);
}

// Off the step path (FP64 arithmetic): f = f^eq(rho, u) from fields; the
// state from full post-collision populations f (projected onto the
// five-number form: its moments and group sums; exact for any SmrtLBM
// post-collision state); the populations of the state; its moments.
template <typename MS, typename F>
__global__ void init_moments(MS* __restrict__ dst, Geom g, const F* __restrict__ rho, const F* __restrict__ ux,
                             const F* __restrict__ uy)
{
    using P = MomPlanes<MS>;
    using H = typename P::H;
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        const double r = rho ? (double)rho[i] : 1.0;
        const double vx = ux ? (double)ux[i] : 0.0, vy = uy ? (double)uy[i] : 0.0;
        const int64_t off = (int64_t)y * g.pitch + x;
        P::m(dst, g.plane, 0)[off] = (typename P::MT)(r - 1.0);
        P::m(dst, g.plane, 1)[off] = (typename P::MT)(r * vx);
        P::m(dst, g.plane, 2)[off] = (typename P::MT)(r * vy);
        Amp<H>::from_f64(P::g(dst, g.plane, 0) + off, 0.0);
        Amp<H>::from_f64(P::g(dst, g.plane, 1) + off, 0.0);
    }
}

__device__ __forceinline__ double feq_dev_f64(int a, double drho, double jx, double jy, double ux, double uy)
{
    const double ej = EX[a] * jx + EY[a] * jy, eu = EX[a] * ux + EY[a] * uy;
    return weight_f64(a) * (drho + 3.0 * ej + 4.5 * ej * eu - 1.5 * (jx * ux + jy * uy));
}

template <typename MS, typename F>
__global__ void set_populations_mom(MS* __restrict__ dst, Geom g, const F* __restrict__ f)
{
    using P = MomPlanes<MS>;
    using H = typename P::H;
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        double d[9], drho = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            d[a] = (double)f[a * n + i] - weight_f64(a);
            drho += d[a];
            jx += EX[a] * d[a];
            jy += EY[a] * d[a];
        }
        const double ux = jx / (1.0 + drho), uy = jy / (1.0 + drho);
        double c[2] = {0.0, 0.0};
        for (int a = 1; a < 9; ++a) c[GRP[a]] += SGN[a] * (d[a] - feq_dev_f64(a, drho, jx, jy, ux, uy));
        const int64_t off = (int64_t)y * g.pitch + x;
        P::m(dst, g.plane, 0)[off] = (typename P::MT)drho;
        P::m(dst, g.plane, 1)[off] = (typename P::MT)jx;
        P::m(dst, g.plane, 2)[off] = (typename P::MT)jy;
        Amp<H>::from_f64(P::g(dst, g.plane, 0) + off, 0.25 * c[0]);
        Amp<H>::from_f64(P::g(dst, g.plane, 1) + off, 0.25 * c[1]);
    }
}

template <typename MS, typename F>
__global__ void get_populations_mom(const MS* __restrict__ src, Geom g, F* __restrict__ f)
{
    using P = MomPlanes<MS>;
    using H = typename P::H;
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        const int64_t off = (int64_t)y * g.pitch + x;
        const double drho = (double)P::m(src, g.plane, 0)[off];
        const double jx = (double)P::m(src, g.plane, 1)[off], jy = (double)P::m(src, g.plane, 2)[off];
        const double ux = jx / (1.0 + drho), uy = jy / (1.0 + drho);
        const double gg[2] = {Amp<H>::to_f64(P::g(src, g.plane, 0) + off), Amp<H>::to_f64(P::g(src, g.plane, 1) + off)};
        for (int a = 0; a < 9; ++a) {
            const double amp = a ? SGN[a] * gg[GRP[a]] : 0.0;
            f[a * n + i] = (F)(weight_f64(a) + feq_dev_f64(a, drho, jx, jy, ux, uy) + amp);
        }
    }
}

// Density deviation and momentum of a stored node (used by the export and
// reduction kernels of lbm_kernels.hpp).
template <typename MT, typename H>
__device__ __forceinline__ void node_moments_f64(const MomStore<MT, H>* __restrict__ src, const Geom& g, int64_t off,
                                                 double& drho, double& jx, double& jy)
{
    using P = MomPlanes<MomStore<MT, H>>;
    drho = (double)P::m(src, g.plane, 0)[off];
    jx = (double)P::m(src, g.plane, 1)[off];
    jy = (double)P::m(src, g.plane, 2)[off];
}

} // namespace smrt
