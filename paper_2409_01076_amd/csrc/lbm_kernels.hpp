// lbm_kernels.hpp -- gfx950 device code for the D2Q9 SRT / SmrtLBM update.
//
// State: post-collision populations stored as deviations d_a = f*_a - w_a in
// nine structure-of-arrays planes.  Element (x, y) of plane a sits at
// a * plane + y * pitch + x.  Two such buffers alternate (ping-pong), so every
// step reads one buffer and writes the other: inputs are read-only and each
// output element has exactly one writer.
//
// The stream-collide kernels are a pull scheme: node x gathers d_a(x - e_a)
// from the previous step, which is the streaming half of Eq. (lb.srt) /
// Eq. (SmrtLBM-1), then forms the moments (Eq. fea-0), the equilibrium
// (Eq. feq-full) and the collision, and writes nine aligned values.  One step
// per launch (stream_collide) is bound by HBM traffic: 9 loads and 9 stores
// per node, about 70 vector instructions.  The multi-step kernels
// (stream_collide_x2 .. _x5) keep the intermediate steps of a tile in LDS, so
// HBM traffic per node-update falls to 1/S; the latency between their HBM
// and LDS phases and the vector ALU then bound them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smrt {

enum { SRT = 0, SMRT = 1, TRT = 2 };
// CAVITY: half-way bounce-back walls, the lid a moving wall half a link above
// the top row.  CAVITY_EQLID: the same walls, but the top row of nodes is the
// lid itself (the second lid reading; one step per launch only).
enum { CAVITY = 0, PERIODIC = 1, CAVITY_EQLID = 2 };

// bfloat16 storage: the upper half of an IEEE binary32.
struct bf16 {
    uint16_t bits;
};

// Storage traits: how a stored population d_a converts to and from the
// arithmetic type C.  FP64 storage and the FP32-storage/FP64-arithmetic type
// (f32x) compute in FP64, everything else in FP32.
//   load / store        the hot path (stores are non-temporal: written once,
//                       read by the next step from HBM);
//   stored_value(v, a)  v exactly as a store followed by a load returns it;
//   to_f64 / from_f64   initialisation, export and reductions;
//   M                   the type a multi-step launch keeps its intermediate
//                       steps in (LDS): C, or the stored type where C is
//                       wider and every value is already on its grid.
// kRounds is true when stored_value is not the identity.
template <typename T> struct Storage;

template <> struct Storage<double> {
    using C = double;
    using M = double;
    static constexpr bool kRounds = false;
    static __device__ __forceinline__ C load(const double* p, int) { return *p; }
    static __device__ __forceinline__ void store(double* p, int, C v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ C stored_value(C v, int) { return v; }
    static __device__ __forceinline__ double to_f64(const double* p, int) { return *p; }
    static __device__ __forceinline__ void from_f64(double* p, int, double v) { *p = v; }
};

template <> struct Storage<float> {
    using C = float;
    using M = float;
    static constexpr bool kRounds = false;
    static __device__ __forceinline__ C load(const float* p, int) { return *p; }
    static __device__ __forceinline__ void store(float* p, int, C v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ C stored_value(C v, int) { return v; }
    static __device__ __forceinline__ double to_f64(const float* p, int) { return (double)*p; }
    static __device__ __forceinline__ void from_f64(float* p, int, double v) { *p = (float)v; }
};

// FP16 holds h_a = d_a * 2^8 * {2, 8, 32} (rest, axis, diagonal): about
// 230 d_a / w_a, so the deviations of a flow at lattice Mach numbers up to
// ~0.3 sit between FP16's normal minimum (6.1e-5) and a few hundred, far
// from both the subnormal range and overflow (65504).  Powers of two scale
// exactly, so the only rounding is FP16's own (relative 2^-11).
__device__ __forceinline__ float f16_scale(int a) { return a == 0 ? 512.0f : (a <= 4 ? 2048.0f : 8192.0f); }
__device__ __forceinline__ float f16_unscale(int a)
{
    return a == 0 ? 1.0f / 512.0f : (a <= 4 ? 1.0f / 2048.0f : 1.0f / 8192.0f);
}

template <> struct Storage<_Float16> {
    using C = float;
    using M = float;
    static constexpr bool kRounds = true;
    static __device__ __forceinline__ C load(const _Float16* p, int a) { return (float)*p * f16_unscale(a); }
    static __device__ __forceinline__ void store(_Float16* p, int a, C v)
    {
        __builtin_nontemporal_store((_Float16)(v * f16_scale(a)), p);
    }
    static __device__ __forceinline__ C stored_value(C v, int a)
    {
        return (float)(_Float16)(v * f16_scale(a)) * f16_unscale(a);
    }
    static __device__ __forceinline__ double to_f64(const _Float16* p, int a)
    {
        return (double)((float)*p * f16_unscale(a));
    }
    static __device__ __forceinline__ void from_f64(_Float16* p, int a, double v)
    {
        *p = (_Float16)((float)v * f16_scale(a));
    }
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round-to-nearest-even binary32 -> bfloat16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// bfloat16 keeps binary32's exponent range, so it needs no scaling.
template <> struct Storage<bf16> {
    using C = float;
    using M = float;
    static constexpr bool kRounds = true;
    static __device__ __forceinline__ C load(const bf16* p, int) { return bf16_to_f32(p->bits); }
    static __device__ __forceinline__ void store(bf16* p, int, C v)
    {
        __builtin_nontemporal_store(f32_to_bf16(v), &p->bits);
    }
    static __device__ __forceinline__ C stored_value(C v, int) { return bf16_to_f32(f32_to_bf16(v)); }
    static __device__ __forceinline__ double to_f64(const bf16* p, int) { return (double)bf16_to_f32(p->bits); }
    static __device__ __forceinline__ void from_f64(bf16* p, int, double v) { p->bits = f32_to_bf16((float)v); }
};

// FP32 storage with FP64 arithmetic: every collision is computed in FP64
// from the stored binary32 values and rounded once per stored value, so the
// only FP32 error is that of the stored values themselves (binary32
// arithmetic in the collision biases the momentum balance enough to move a
// slowly converging cavity by 1e-5 of the lid speed within 2,000 steps).
// Intermediate steps of a multi-step launch stay binary32 in LDS, exactly as
// a store and load would leave them.
struct f32x {
    float v;
};

template <> struct Storage<f32x> {
    using C = double;
    using M = float;
    static constexpr bool kRounds = true;
    static __device__ __forceinline__ C load(const f32x* p, int) { return (double)p->v; }
    static __device__ __forceinline__ void store(f32x* p, int, C v) { __builtin_nontemporal_store((float)v, &p->v); }
    static __device__ __forceinline__ C stored_value(C v, int) { return (double)(float)v; }
    static __device__ __forceinline__ double to_f64(const f32x* p, int) { return (double)p->v; }
    static __device__ __forceinline__ void from_f64(f32x* p, int, double v) { p->v = (float)v; }
};

// D2Q9 in the paper's order; OPP[a] is the direction with e = -e_a.
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename C> struct W {
    static constexpr C axis = C(1) / C(9);
    static constexpr C diag = C(1) / C(36);
};

__device__ __forceinline__ double weight_f64(int a)
{
    return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}

struct Geom {
    int nx, ny;
    int pitch;     // elements per row (>= nx)
    int64_t plane; // elements per direction plane
    int bx, by, rows;
    int tiles_x;   // tiles along x
    int panel;     // multi-step kernels: tile order, 0 = row-major, P > 0 = XCD panels of P tile columns
};

// Workgroups are dealt to the 8 XCDs round-robin.  This renumbering gives
// each XCD one contiguous range of positions.
__device__ __forceinline__ int xcd_contiguous(int bid, int nblocks)
{
    constexpr int NXCD = 8;
    const int xcd = bid % NXCD, local = bid / NXCD;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Tile at position `pos` of the panel order: the lattice's tile columns are
// cut into panels of P columns (the last may be narrower), each walked row by
// row from the top.  With each XCD taking one contiguous run of positions, a
// tile's vertical neighbour is P positions away on the same XCD, so the halo
// rows they share are still in that XCD's L2.  P = 0: row-major.
__device__ __forceinline__ void panel_tile(int pos, int tiles_x, int tiles_y, int P, int& tx, int& ty)
{
    if (P <= 0) {
        tx = pos % tiles_x;
        ty = pos / tiles_x;
        return;
    }
    const int full = tiles_x / P, per_panel = P * tiles_y;
    const int panel = pos / per_panel;
    if (panel < full) {
        const int w = pos - panel * per_panel;
        ty = w / P;
        tx = panel * P + w % P;
    } else {
        const int w = pos - full * per_panel, pw = tiles_x - full * P;
        ty = w / pw;
        tx = full * P + w % pw;
    }
}

template <typename C> struct Coef {
    C omega;   // 1/tau
    C omega_s; // 1/tau_s (TRT)
    C a;       // 1 - 1/tau (SmrtLBM)
    C b;       // 1/tau_s - 1/tau (TRT)
    C lid;     // 6 w_diag u_lid = u_lid / 6: the moving-lid term of a diagonal link
    C ulid;    // u_lid itself (equilibrium lid)
};

// Moments, equilibrium deviation and collision of one node, in deviation form.
// With j = rho u and drho = rho - 1 (sum_a w_a e_a = 0, sum_a w_a = 1):
//   drho = sum_a d_a,  j = sum_a e_a d_a,
//   f^eq_a - w_a = w_a (drho + 3 e_a.j + 9/2 (e_a.j)(e_a.u) - 3/2 j.u),
// an exact rewrite of Eq. (feq-full) that keeps FP32 rounding relative to the
// small deviations instead of to f ~ w.
//
// Each opposite pair (a, opp(a)) is written as s +- t, with s the even and t
// the odd part.  Rounded weights would make the equilibrium's own mass and
// momentum (1 + 7.5e-9) drho and (1 + 7.5e-9) j in FP32, a bias that compounds
// every step (1e-5 of the lid speed after 2000 steps); so the axis odd parts
// and the rest population are formed from what the other terms leave of j and
// drho, which restores conservation up to unbiased rounding:
//   t_x = j_x / 2 - (t_5 - t_6),  t_y = j_y / 2 - (t_5 + t_6)  (both j / 3),
//   q_0 = drho - 2 (s_x + s_y + s_5 + s_6)                      (w_0 (...)).
//
// 1/rho enters only the terms quadratic in u, so FP32 takes the hardware
// reciprocal (1 ulp) instead of a correctly rounded division.  FP64 refines
// the hardware reciprocal with two Newton steps, r <- r + r (1 - x r), each of
// which squares the relative error: about one ulp, in 5 instructions where a
// correctly rounded division takes 11.
__device__ __forceinline__ float reciprocal(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double reciprocal(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// e / 12, the odd part 3 w_diag (e_a . j) of a diagonal link.  In binary32
// 1/12 rounds up by 2^-25 of itself, and that bias is the same at every node
// and step: the diagonal odd parts t5, t6 come out too large and the axis
// ones (j/2 - (t5 -/+ t6)) too small.  Momentum stays exact, but the
// equilibrium's third moments are biased, and the slow modes of a long
// cavity run integrate it: in a float32 emulation of this collision, 4.7e-5 U
// after 20,000 steps of the 1024^2 cavity at Re 1000 with the single rounded
// constant, 2.8e-7 U with 1/12 as the pair hi + lo (FP64 arithmetic: 9e-8).
// The pair costs one multiply; FP64 keeps the plain constant (its rounding,
// 4.6e-18, is below every other error).
template <typename C> __device__ __forceinline__ C twelfth_of(C e) { return C(1.0 / 12.0) * e; }
template <> __device__ __forceinline__ float twelfth_of<float>(float e)
{
    constexpr float hi = (float)(1.0 / 12.0), lo = (float)(1.0 / 12.0 - (double)(float)(1.0 / 12.0));
    return __builtin_fmaf(hi, e, lo * e);
}

template <int SCHEME, typename T, typename C = typename Storage<T>::C>
__device__ __forceinline__ void collide(C d[9], const Coef<C>& k)
{
    // Sums and differences of the opposite pairs (1,3), (2,4), (5,7), (6,8)
    // give the moments and, below, the group sums with few operations.
    const C p13 = d[1] + d[3], p24 = d[2] + d[4], p57 = d[5] + d[7], p68 = d[6] + d[8];
    const C m13 = d[1] - d[3], m24 = d[2] - d[4], m57 = d[5] - d[7], m68 = d[6] - d[8];
    const C drho = d[0] + ((p13 + p24) + (p57 + p68));
    const C jx = m13 + (m57 - m68); // e_x = +1 for 1, 5, 8 and -1 for 3, 6, 7
    const C jy = m24 + (m57 + m68); // e_y = +1 for 2, 5, 6 and -1 for 4, 7, 8
    const C inv = reciprocal(C(1) + drho);
    const C ux = jx * inv, uy = jy * inv;
    // j.u splits into j_x u_x + j_y u_y; on the diagonals (e.j)(e.u) is
    // j.u + 2 j_x u_y (links 5, 7) or j.u - 2 j_x u_y (links 6, 8), since
    // j_x u_y = j_y u_x.
    const C jxux = jx * ux, jyuy = jy * uy, jxuy = jx * uy;
    const C ju = jxux + jyuy;
    const C base = drho - C(1.5) * ju;

    // s = w (base + 9/2 (e.j)(e.u)): 9/2 w_axis = 1/2, 9/2 w_diag = 1/8
    const C abase = W<C>::axis * base;
    const C dmid = W<C>::diag * base + C(0.125) * ju;
    const C sx = abase + C(0.5) * jxux;
    const C sy = abase + C(0.5) * jyuy;
    const C s5 = dmid + C(0.25) * jxuy;
    const C s6 = dmid - C(0.25) * jxuy;
    const C e5j = jx + jy; // e_5 = (1, 1) = -e_7
    const C e6j = jy - jx; // e_6 = (-1, 1) = -e_8
    const C t5 = twelfth_of(e5j); // 3 w_diag (e_5 . j)
    const C t6 = twelfth_of(e6j);
    const C tx = C(0.5) * jx - (t5 - t6);
    const C ty = C(0.5) * jy - (t5 + t6);

    // Group sums of Eq. (sigma1-2-0), times 4: C_1 over the axis links, C_2
    // over the diagonal links, each sum_k (-1)^k (f_k - f^eq_k).  The odd
    // parts cancel in the equilibrium's share, which leaves
    // q_2 + q_4 - q_1 - q_3 = 2 (s_y - s_x) = j_y u_y - j_x u_x and
    // q_6 + q_8 - q_5 - q_7 = 2 (s_6 - s_5) = -j_x u_y.
    const C c1x4 = (p24 - p13) - (jyuy - jxux);
    const C c2x4 = (p68 - p57) + jxuy;
    if constexpr (SCHEME == SMRT) {
        // Eq. (SmrtLBM-1): f*_a = f^eq_a + (-1)^a (1 - 1/tau) C_g(a); both
        // members of an opposite pair get the same correction.
        const C qa = C(0.25) * k.a;
        const C g1 = qa * c1x4, g2 = qa * c2x4;
        const C ax = sx - g1, ay = sy + g1, a5 = s5 - g2, a6 = s6 + g2;
        d[1] = ax + tx;
        d[3] = ax - tx;
        d[2] = ay + ty;
        d[4] = ay - ty;
        d[5] = a5 + t5;
        d[7] = a5 - t5;
        d[6] = a6 + t6;
        d[8] = a6 - t6;
    } else {
        C q[9];
        q[0] = drho - C(2) * ((sx + sy) + (s5 + s6));
        q[1] = sx + tx;
        q[3] = sx - tx;
        q[2] = sy + ty;
        q[4] = sy - ty;
        q[5] = s5 + t5;
        q[7] = s5 - t5;
        q[6] = s6 + t6;
        q[8] = s6 - t6;
        if constexpr (SCHEME == SRT) {
            // Eq. (lb.srt): f* = f - (f - f^eq)/tau
#pragma unroll
            for (int a = 0; a < 9; ++a) d[a] = d[a] + k.omega * (q[a] - d[a]);
        } else {
            // Eq. (SmrtLBM-lb.1.5): f*_a = f_a - (f_a - f^eq_a)/tau_s + (-1)^a (1/tau_s - 1/tau) C_g(a)
            const C qb = C(0.25) * k.b;
            const C g1 = qb * c1x4, g2 = qb * c2x4;
#pragma unroll
            for (int a = 0; a < 9; ++a) d[a] = d[a] + k.omega_s * (q[a] - d[a]);
            d[1] -= g1;
            d[2] += g1;
            d[3] -= g1;
            d[4] += g1;
            d[5] -= g2;
            d[6] += g2;
            d[7] -= g2;
            d[8] += g2;
        }
    }
    // The collision conserves mass, so the rest population is what the other
    // eight leave of drho.  Forming it from the rounded values removes a
    // rounding bias of about 1e-11 per node and step in FP32 that otherwise
    // makes the total mass drift steadily.  With 16-bit storage the eight are
    // first put on the storage grid, so only the rest population's own
    // rounding (unbiased) changes the stored mass.
    if constexpr (Storage<T>::kRounds) {
#pragma unroll
        for (int a = 1; a < 9; ++a) d[a] = Storage<T>::stored_value(d[a], a);
    }
    d[0] = drho - (((d[1] + d[2]) + (d[3] + d[4])) + ((d[5] + d[6]) + (d[7] + d[8])));
}

// The equilibrium lid (second lid reading): a node of the top row is set to
// f^eq(rho, (U, 0)) (Eq. feq-full), with rho from the populations it received
// from inside the cavity.  For a wall moving along itself the unknown d_4,
// d_7, d_8 carry as much mass as the d_2, d_5, d_6 that left, so
// rho - 1 = d_0 + d_1 + d_3 + 2 (d_2 + d_5 + d_6) (the weights of that sum add up
// to 1).  In deviation form, with e_x = +1, 0, -1:
//   d_a = w_a (drho + rho (3 e_x U + 9/2 e_x^2 U^2 - 3/2 U^2)).
template <typename T, typename C = typename Storage<T>::C>
__device__ __forceinline__ void lid_equilibrium(C d[9], const Coef<C>& k)
{
    const C drho = (d[0] + (d[1] + d[3])) + C(2) * ((d[2] + d[5]) + d[6]);
    const C rho = C(1) + drho, U = k.ulid;
    const C base = drho - C(1.5) * rho * U * U;
    const C quad = C(4.5) * rho * U * U, lin = C(3) * rho * U;
    const C plus = base + (quad + lin), minus = base + (quad - lin);
    d[0] = C(4.0 / 9.0) * base;
    d[2] = d[4] = W<C>::axis * base;
    d[1] = W<C>::axis * plus;
    d[3] = W<C>::axis * minus;
    d[5] = d[8] = W<C>::diag * plus;
    d[6] = d[7] = W<C>::diag * minus;
}

// Interior pulls and stores address each direction's plane through a
// workgroup-uniform base pointer held in scalar registers plus one per-lane
// 32-bit byte offset shared by all nine directions; the load/store
// instructions add the two themselves, so no per-access 64-bit address
// arithmetic remains.  The bases are rebased to a row row0 of the workgroup's
// tile, which keeps the offsets to a few rows.
template <typename T> using global_ptr = __attribute__((address_space(1))) T*;

// Pins a workgroup-uniform pointer in scalar registers.  The empty asm emits
// no instruction; it only stops the compiler from folding the base into every
// lane's address.
template <typename T> __device__ __forceinline__ global_ptr<T> scalar_base(T* p)
{
    global_ptr<T> q = (global_ptr<T>)p;
    asm("" : "+s"(q));
    return q;
}

template <typename T> struct PullBases {
    global_ptr<const T> p[9]; // plane a, row row0, shifted by -e_a
    int row0;
};

// Bases for pulls into nodes (x, y) with y - 1 >= row0.
template <typename T>
__device__ __forceinline__ PullBases<T> pull_bases(const T* __restrict__ src, const Geom& g, int row0)
{
    PullBases<T> b;
    b.row0 = row0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
        b.p[a] = scalar_base(src + (int64_t)a * g.plane + (int64_t)(row0 + 1 - EY[a]) * g.pitch + (1 - EX[a]));
    return b;
}

// Pull of the nine incoming populations of an interior node: every source
// x - e_a lies inside the lattice.
template <typename T>
__device__ __forceinline__ void gather_interior(const PullBases<T>& b, const Geom& g, int x, int y,
                                                typename Storage<T>::C d[9])
{
    const uint32_t off = (uint32_t)(((y - 1 - b.row0) * g.pitch + (x - 1)) * (int)sizeof(T));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const global_ptr<const char> q = (global_ptr<const char>)b.p[a] + off;
        d[a] = Storage<T>::load((const T*)(global_ptr<const T>)q, a);
    }
}

template <typename T> struct StoreBases {
    global_ptr<T> p[9]; // plane a, row row0
    int row0;
};

// Bases for stores to nodes (x, y) with y >= row0.
template <typename T>
__device__ __forceinline__ StoreBases<T> store_bases(T* __restrict__ dst, const Geom& g, int row0)
{
    StoreBases<T> b;
    b.row0 = row0;
#pragma unroll
    for (int a = 0; a < 9; ++a) b.p[a] = scalar_base(dst + (int64_t)a * g.plane + (int64_t)row0 * g.pitch);
    return b;
}

// Pull at a node on the outer ring.  Periodic: sources wrap around.  Cavity:
// a source beyond a wall is replaced by the node's own opposite population
// (half-way bounce-back); a link from the lid row (y = ny, corners included)
// gains 6 w_a (e_a . u_lid), which is -u_lid/6 for a = 7, +u_lid/6 for a = 8
// and 0 for a = 4.  Branch-free: each direction selects its address and
// issues one load, so the nine loads stay in flight together (a branch per
// direction made the compiler wait on each load in turn).
template <typename T, int BC>
__device__ __forceinline__ void gather_edge(const T* __restrict__ src, const Geom& g, int x, int y,
                                            typename Storage<T>::C d[9], typename Storage<T>::C lid)
{
    using S = Storage<T>;
    using C = typename Storage<T>::C;
    const int64_t own = (int64_t)y * g.pitch + x; // a plane may exceed 2^31 elements
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int sx = x - EX[a], sy = y - EY[a];
        const T* plane_a = src + a * g.plane; // uniform per workgroup
        if constexpr (BC == PERIODIC) {
            sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
            sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
            d[a] = S::load(plane_a + ((int64_t)sy * g.pitch + sx), a);
        } else {
            const T* plane_o = src + OPP[a] * g.plane;
            const bool inside = (unsigned)sx < (unsigned)g.nx && (unsigned)sy < (unsigned)g.ny;
            const T* p = inside ? plane_a + ((int64_t)sy * g.pitch + sx) : plane_o + own;
            // a and OPP[a] share a weight class, hence a storage scale
            const C v = S::load(p, a);
            d[a] = (!inside && sy == g.ny) ? v + C(EX[a]) * lid : v;
        }
    }
}

// Store of the nine post-collision populations of node (x, y).
template <typename T>
__device__ __forceinline__ void scatter_store(const StoreBases<T>& b, const Geom& g, int x, int y,
                                              const typename Storage<T>::C d[9])
{
    const uint32_t off = (uint32_t)(((y - b.row0) * g.pitch + x) * (int)sizeof(T));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const global_ptr<char> q = (global_ptr<char>)b.p[a] + off;
        Storage<T>::store((T*)(global_ptr<T>)q, a, d[a]);
    }
}

// One time step.  Block (bx, by) threads; each thread updates `rows` nodes
// spaced by by along y, so a block covers a bx x (by * rows) tile.
template <typename T, int SCHEME, int BC>
__global__ void __launch_bounds__(1024) stream_collide(const T* __restrict__ src, T* __restrict__ dst,
                                                       Geom g, Coef<typename Storage<T>::C> k)
{
    using C = typename Storage<T>::C;
    // Tiles in row-major block order.  Workgroups are dealt to the 8 XCDs
    // round-robin, so when tiles_x is a multiple of 8 the tiles above and
    // below a tile run on the same XCD and share its L2 for the y-halo rows;
    // all XCDs stream through neighbouring memory at any moment.  (Giving each
    // XCD one contiguous slab of tiles measured 8% slower on 4096^2.)
    const int tile = blockIdx.x;
    const int tx = tile % g.tiles_x, ty = tile / g.tiles_x;
    const int x = tx * g.bx + threadIdx.x;
    if (x >= g.nx) return;
    const int ytile = ty * g.by * g.rows; // first row of the tile
    const PullBases<T> pb = pull_bases(src, g, ytile > 0 ? ytile - 1 : 0);
    const StoreBases<T> sb = store_bases(dst, g, ytile);
    const int y0 = ytile + threadIdx.y;
    constexpr int GBC = BC == PERIODIC ? PERIODIC : CAVITY; // the equilibrium lid pulls like the cavity
    for (int r = 0; r < g.rows; ++r) {
        const int y = y0 + r * g.by;
        if (y >= g.ny) break;
        C d[9];
        const bool edge = (x == 0) | (x == g.nx - 1) | (y == 0) | (y == g.ny - 1);
        if (edge)
            gather_edge<T, GBC>(src, g, x, y, d, k.lid);
        else
            gather_interior<T>(pb, g, x, y, d);
        if (BC == CAVITY_EQLID && y == g.ny - 1)
            lid_equilibrium<T>(d, k); // d_4, d_7, d_8 pulled from beyond the lid are not used
        else
            collide<SCHEME, T>(d, k);
        scatter_store<T>(sb, g, x, y, d);
    }
}

// Several time steps per launch (temporal blocking).  A workgroup owns a
// TX x TY tile of outputs; the steps before the last are computed on the
// tile plus a ring of nodes and kept in LDS (multi_tile below).  Per node the
// arithmetic is that of stream_collide (same gather, collide and, for 16-bit
// storage, the same rounding to the storage grid between the steps), so the
// results are bitwise those of one-step launches.

// The first step of a multi-step launch, in two halves over a region of
// RX x RY nodes: the tile (X0, Y0, TX x TY) plus a ring of RING nodes.
// ring_load issues the loads of all the thread's region nodes (up to 9 P
// loads per lane in flight together); ring_collide collides them and writes
// the step to LDS.  Periodic regions wrap once; region nodes more than RING -
// 1 past column nx or row ny feed no output of the tile and are skipped, and
// every wrapped node takes the edge path (explicit wrap), so interior pulls
// all have y - 1 >= Y0 - RING - 1, the row the pull bases start at.  Cavity
// regions skip the nodes beyond the walls.
template <typename T, int RX, int RY, int NT> struct RingRegs {
    using C = typename Storage<T>::C;
    static constexpr int P = (RX * RY + NT - 1) / NT; // region nodes per thread
    C d[P][9];
    bool live[P];
};

template <typename T, int BC, int RX, int RY, int NT, int RING, bool INNER>
__device__ __forceinline__ void ring_load(const T* __restrict__ src, const Geom& g, typename Storage<T>::C lid,
                                          int X0, int Y0, RingRegs<T, RX, RY, NT>& r)
{
    const PullBases<T> pb = pull_bases(src, g, Y0 > RING ? Y0 - RING - 1 : 0);
#pragma unroll
    for (int j = 0; j < RingRegs<T, RX, RY, NT>::P; ++j) {
        const int i = threadIdx.x + j * NT;
        const int lx = i % RX, ly = i / RX;
        const int xu = X0 - RING + lx, yu = Y0 - RING + ly;
        if constexpr (INNER) {
            // the whole region lies inside the lattice, off its outer ring
            r.live[j] = i < RX * RY;
            if (r.live[j]) gather_interior<T>(pb, g, xu, yu, r.d[j]);
            continue;
        }
        int x = xu, y = yu;
        if constexpr (BC == PERIODIC) {
            r.live[j] = i < RX * RY && xu <= g.nx + RING - 1 && yu <= g.ny + RING - 1;
            x = xu < 0 ? xu + g.nx : (xu >= g.nx ? xu - g.nx : xu);
            y = yu < 0 ? yu + g.ny : (yu >= g.ny ? yu - g.ny : yu);
        } else {
            r.live[j] = i < RX * RY && (unsigned)xu < (unsigned)g.nx && (unsigned)yu < (unsigned)g.ny;
        }
        if (r.live[j]) {
            const bool edge = (x != xu) | (y != yu) | (x == 0) | (x == g.nx - 1) | (y == 0) | (y == g.ny - 1);
            if (edge)
                gather_edge<T, BC>(src, g, x, y, r.d[j], lid);
            else
                gather_interior<T>(pb, g, x, y, r.d[j]);
        }
    }
}

template <typename T, int SCHEME, int RX, int RY, int NT>
__device__ __forceinline__ void ring_collide(const Coef<typename Storage<T>::C>& k, RingRegs<T, RX, RY, NT>& r,
                                             typename Storage<T>::M (&m)[9][RY][RX])
{
    using M = typename Storage<T>::M;
#pragma unroll
    for (int j = 0; j < RingRegs<T, RX, RY, NT>::P; ++j) {
        if (!r.live[j]) continue;
        const int i = threadIdx.x + j * NT;
        const int lx = i % RX, ly = i / RX;
        collide<SCHEME, T>(r.d[j], k);
        if constexpr (Storage<T>::kRounds) r.d[j][0] = Storage<T>::stored_value(r.d[j][0], 0);
#pragma unroll
        for (int a = 0; a < 9; ++a) m[a][ly][lx] = (M)r.d[j][a];
    }
}

// Pull of node (x, y) of the lattice from a step held in LDS as m[9][FY][FX],
// the node at frame position (fx, fy): bounce-back from the node's own
// opposite population where the source lies beyond a cavity wall (plus the
// lid term from the lid row).  Periodic regions hold the wrapped nodes'
// values, so their pulls need no wrap.  Every source is a constant offset
// from the node's own cell.
template <typename T, int BC, int FX, int FY, bool INNER = false>
__device__ __forceinline__ void pull_lds(const typename Storage<T>::M (&m)[9][FY][FX], const Geom& g,
                                         typename Storage<T>::C lid, int fx, int fy, int x, int y,
                                         typename Storage<T>::C d[9])
{
    using C = typename Storage<T>::C;
    using M = typename Storage<T>::M;
    constexpr int PL = FX * FY;
    const M* own = &m[0][fy][fx];
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = (C)own[a * PL - EY[a] * FX - EX[a]];
    if constexpr (BC == CAVITY && !INNER) {
        // only lanes on the lattice's outer ring have sources beyond a wall:
        // x - e_x < 0 only at x = 0 with e_x = 1, x - e_x = nx only at
        // x = nx - 1 with e_x = -1, likewise in y; the lid row y = ny feeds
        // the links with e_y = -1 at y = ny - 1, corners included
        const bool wl = x == 0, wr = x == g.nx - 1, wb = y == 0, wt = y == g.ny - 1;
        if (wl | wr | wb | wt) {
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const bool bx = EX[a] > 0 ? wl : (EX[a] < 0 ? wr : false);
                const bool by = EY[a] > 0 ? wb : (EY[a] < 0 ? wt : false);
                const C back = (C)own[OPP[a] * PL];
                if (EY[a] < 0) // folded once the loop is unrolled
                    d[a] = (bx | by) ? (wt ? back + C(EX[a]) * lid : back) : d[a];
                else
                    d[a] = (bx | by) ? back : d[a];
            }
        }
    }
}

// Last step of a multi-step launch: pull the previous step from LDS (held on
// the tile plus a one-node ring, inside a frame of the tile plus R rings),
// collide, store to HBM.
template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int R, bool INNER = false>
__device__ __forceinline__ void lds_to_hbm(T* __restrict__ dst, const Geom& g, const Coef<typename Storage<T>::C>& k,
                                           int X0, int Y0,
                                           const typename Storage<T>::M (&m)[9][TY + 2 * R][TX + 2 * R])
{
    using C = typename Storage<T>::C;
    const StoreBases<T> sb = store_bases(dst, g, Y0);
    for (int i = threadIdx.x; i < TX * TY; i += NT) {
        const int tx = i % TX, ty = i / TX;
        const int x = X0 + tx, y = Y0 + ty;
        if (!INNER && (x >= g.nx || y >= g.ny)) continue;
        C d[9];
        pull_lds<T, BC, TX + 2 * R, TY + 2 * R, INNER>(m, g, k.lid, tx + R, ty + R, x, y, d);
        collide<SCHEME, T>(d, k);
        scatter_store<T>(sb, g, x, y, d);
    }
}

// Tile of this workgroup (row-major or XCD panel order).
__device__ __forceinline__ void workgroup_tile(const Geom& g, int TX, int TY, int& X0, int& Y0)
{
    const int tiles_y = (int)gridDim.x / g.tiles_x;
    const int pos = g.panel > 0 ? xcd_contiguous(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int tx, ty;
    panel_tile(pos, g.tiles_x, tiles_y, g.panel, tx, ty);
    X0 = tx * TX;
    Y0 = ty * TY;
}

// S time steps per launch (S = 2 .. 5) on a TX x TY tile.  Step t+1 is
// computed on the tile plus a ring of S - 1 nodes (pulled from HBM) into LDS;
// each further step t+s (s < S) is pulled from LDS on the tile plus a ring of
// S - s nodes, collided into registers and, after a barrier, written over the
// same LDS; step t+S is pulled from LDS for the tile only and stored.  HBM
// traffic per node-update falls to 1/S of a one-step launch; the rings add
// sum_r (TX + 2r)(TY + 2r) / (TX TY) - (S - 1) redundant collisions.  Same
// per-node arithmetic, so the results are bitwise those of S one-step
// launches.  A periodic lattice needs nx >= TX + 2(S - 1), ny >= TY + 2(S - 1).
//
// All steps share one LDS frame of the tile plus R = S - 1 rings, 9 planes of
// FY x FX; the step held on the tile plus r rings occupies the frame's
// window from (R - r, R - r), so a node has one frame position for every
// step: it writes its new values where it pulled its own rest population.
template <typename T, int TX, int TY, int S> struct MultiTile {
    using M = typename Storage<T>::M;
    static constexpr int R = S - 1, FX = TX + 2 * R, FY = TY + 2 * R;
    M m[9][FY][FX];
};

// A middle step: pull from the ring-(r+1) step in LDS, collide on the tile
// plus a ring of r nodes, then (after every pull is done) write over the LDS.
template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int S, int r, bool INNER>
__device__ __forceinline__ void middle_step(const Geom& g, const Coef<typename Storage<T>::C>& k, int X0, int Y0,
                                            MultiTile<T, TX, TY, S>& sh)
{
    using C = typename Storage<T>::C;
    using Tile = MultiTile<T, TX, TY, S>;
    constexpr int BX = TX + 2 * r, BY = TY + 2 * r, OFF = Tile::R - r, FX = Tile::FX, FY = Tile::FY;
    constexpr int P = (BX * BY + NT - 1) / NT;
    C d[P][9];
    bool live[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = threadIdx.x + j * NT;
        const int lx = i % BX, ly = i / BX;
        const int x = X0 - r + lx, y = Y0 - r + ly; // unwrapped
        if constexpr (INNER)
            live[j] = i < BX * BY;
        else if constexpr (BC == PERIODIC)
            live[j] = i < BX * BY && x <= g.nx + r - 1 && y <= g.ny + r - 1;
        else
            live[j] = i < BX * BY && (unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny;
        if (live[j]) {
            pull_lds<T, BC, FX, FY, INNER>(sh.m, g, k.lid, lx + OFF, ly + OFF, x, y, d[j]);
            collide<SCHEME, T>(d[j], k);
            if constexpr (Storage<T>::kRounds) d[j][0] = Storage<T>::stored_value(d[j][0], 0);
        }
    }
    __syncthreads(); // every pull from the wider ring is done before it is overwritten
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (!live[j]) continue;
        const int i = threadIdx.x + j * NT;
        const int lx = i % BX, ly = i / BX;
        typename Storage<T>::M* own = &sh.m[0][ly + OFF][lx + OFF];
#pragma unroll
        for (int a = 0; a < 9; ++a) own[a * FX * FY] = (typename Storage<T>::M)d[j][a];
    }
    __syncthreads();
}

// The middle steps on rings r, r - 1, .., 1.
template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int S, int r, bool INNER>
__device__ __forceinline__ void middle_steps(const Geom& g, const Coef<typename Storage<T>::C>& k, int X0, int Y0,
                                             MultiTile<T, TX, TY, S>& sh)
{
    if constexpr (r >= 1) {
        middle_step<T, SCHEME, BC, TX, TY, NT, S, r, INNER>(g, k, X0, Y0, sh);
        middle_steps<T, SCHEME, BC, TX, TY, NT, S, r - 1, INNER>(g, k, X0, Y0, sh);
    }
}

// Steps t+2 .. t+S of a tile whose step t+1 is in LDS.
template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int S, bool INNER>
__device__ __forceinline__ void later_steps(T* __restrict__ dst, const Geom& g, const Coef<typename Storage<T>::C>& k,
                                            int X0, int Y0, MultiTile<T, TX, TY, S>& sh)
{
    middle_steps<T, SCHEME, BC, TX, TY, NT, S, S - 2, INNER>(g, k, X0, Y0, sh);
    lds_to_hbm<T, SCHEME, BC, TX, TY, NT, S - 1, INNER>(dst, g, k, X0, Y0, sh.m);
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int S, bool INNER>
__device__ __forceinline__ void multi_tile_body(const T* __restrict__ src, T* __restrict__ dst, const Geom& g,
                                                const Coef<typename Storage<T>::C>& k, int X0, int Y0,
                                                MultiTile<T, TX, TY, S>& sh)
{
    constexpr int R = S - 1;
    {
        RingRegs<T, TX + 2 * R, TY + 2 * R, NT> r;
        ring_load<T, BC, TX + 2 * R, TY + 2 * R, NT, R, INNER>(src, g, k.lid, X0, Y0, r);
        ring_collide<T, SCHEME, TX + 2 * R, TY + 2 * R, NT>(k, r, sh.m);
    }
    __syncthreads();
    later_steps<T, SCHEME, BC, TX, TY, NT, S, INNER>(dst, g, k, X0, Y0, sh);
}

// A tile whose widest region (the tile plus S - 1 rings) lies inside the
// lattice, off its outer ring, needs no wrap, bounce-back or bounds checks:
// most tiles of a large lattice take that copy of the code (same
// arithmetic, so the same results).
__device__ __forceinline__ bool inner_tile(const Geom& g, int X0, int Y0, int TX, int TY, int R)
{
    return X0 - R >= 1 && X0 + TX + R <= g.nx - 1 && Y0 - R >= 1 && Y0 + TY + R <= g.ny - 1;
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT, int S>
__device__ __forceinline__ void multi_tile(const T* __restrict__ src, T* __restrict__ dst, const Geom& g,
                                           const Coef<typename Storage<T>::C>& k, int X0, int Y0,
                                           MultiTile<T, TX, TY, S>& sh)
{
    constexpr int R = S - 1;
    const bool inner = inner_tile(g, X0, Y0, TX, TY, R);
    if (inner)
        multi_tile_body<T, SCHEME, BC, TX, TY, NT, S, true>(src, dst, g, k, X0, Y0, sh);
    else
        multi_tile_body<T, SCHEME, BC, TX, TY, NT, S, false>(src, dst, g, k, X0, Y0, sh);
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stream_collide_x2(const T* __restrict__ src, T* __restrict__ dst, Geom g,
                                                        Coef<typename Storage<T>::C> k)
{
    __shared__ MultiTile<T, TX, TY, 2> sh;
    int X0, Y0;
    workgroup_tile(g, TX, TY, X0, Y0);
    multi_tile<T, SCHEME, BC, TX, TY, NT, 2>(src, dst, g, k, X0, Y0, sh);
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stream_collide_x3(const T* __restrict__ src, T* __restrict__ dst, Geom g,
                                                        Coef<typename Storage<T>::C> k)
{
    __shared__ MultiTile<T, TX, TY, 3> sh;
    int X0, Y0;
    workgroup_tile(g, TX, TY, X0, Y0);
    multi_tile<T, SCHEME, BC, TX, TY, NT, 3>(src, dst, g, k, X0, Y0, sh);
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stream_collide_x4(const T* __restrict__ src, T* __restrict__ dst, Geom g,
                                                        Coef<typename Storage<T>::C> k)
{
    __shared__ MultiTile<T, TX, TY, 4> sh;
    int X0, Y0;
    workgroup_tile(g, TX, TY, X0, Y0);
    multi_tile<T, SCHEME, BC, TX, TY, NT, 4>(src, dst, g, k, X0, Y0, sh);
}

template <typename T, int SCHEME, int BC, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) stream_collide_x5(const T* __restrict__ src, T* __restrict__ dst, Geom g,
                                                        Coef<typename Storage<T>::C> k)
{
    __shared__ MultiTile<T, TX, TY, 5> sh;
    int X0, Y0;
    workgroup_tile(g, TX, TY, X0, Y0);
    multi_tile<T, SCHEME, BC, TX, TY, NT, 5>(src, dst, g, k, X0, Y0, sh);
}

// ---------------------------------------------------------------------------
// Initialisation, export and reductions (off the per-step path).

// d_a = f^eq_a(rho, u) - w_a in FP64, rounded once to the storage type.
template <typename T, typename F>
__global__ void init_equilibrium(T* __restrict__ dst, Geom g, const F* __restrict__ rho,
                                 const F* __restrict__ ux, const F* __restrict__ uy)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        const double r = rho ? (double)rho[i] : 1.0;
        const double vx = ux ? (double)ux[i] : 0.0, vy = uy ? (double)uy[i] : 0.0;
        const double uu = vx * vx + vy * vy;
        T* p = dst + (int64_t)y * g.pitch + x;
        for (int a = 0; a < 9; ++a) {
            const double eu = EX[a] * vx + EY[a] * vy;
            const double dev = weight_f64(a) * ((r - 1.0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
            Storage<T>::from_f64(p + a * g.plane, a, dev);
        }
    }
}

// State <-> dense full populations f = w + d, layout [9][ny][nx].
template <typename T, typename F>
__global__ void set_populations(T* __restrict__ dst, Geom g, const F* __restrict__ f)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        for (int a = 0; a < 9; ++a)
            Storage<T>::from_f64(dst + a * g.plane + (int64_t)y * g.pitch + x, a,
                                 (double)f[a * n + i] - weight_f64(a));
    }
}

template <typename T, typename F>
__global__ void get_populations(const T* __restrict__ src, Geom g, F* __restrict__ f)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        for (int a = 0; a < 9; ++a)
            f[a * n + i] = (F)(weight_f64(a) + Storage<T>::to_f64(src + a * g.plane + (int64_t)y * g.pitch + x, a));
    }
}

// Density deviation and momentum of a stored node, in FP64.
template <typename T>
__device__ __forceinline__ void node_moments_f64(const T* __restrict__ src, const Geom& g, int64_t off,
                                                 double& drho, double& jx, double& jy)
{
    double d[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = Storage<T>::to_f64(src + a * g.plane + off, a);
    drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
}

// rho, ux, uy of the stored state (Eq. fea-0) into dense [ny][nx] arrays.
template <typename T, typename F>
__global__ void export_moments(const T* __restrict__ src, Geom g, F* __restrict__ rho,
                               F* __restrict__ ux, F* __restrict__ uy)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        double drho, jx, jy;
        node_moments_f64(src, g, (int64_t)y * g.pitch + x, drho, jx, jy);
        const double r = 1.0 + drho;
        if (rho) rho[i] = (F)r;
        if (ux) ux[i] = (F)(jx / r);
        if (uy) uy[i] = (F)(jy / r);
    }
}

// Sum over a 64-wide wavefront with xor shuffles (fixed pairing order).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int RED_THREADS = 256;
constexpr int RED_WAVES = RED_THREADS / 64;
constexpr int RED_VALUES = 4; // sum |u - u_snap|^2, sum |u|^2, sum (rho - 1), non-finite nodes

// Per-block FP64 partial sums for the residual and the mass.  Each thread
// walks a fixed, grid-strided set of nodes; lanes combine by xor shuffles and
// waves in index order, so the result does not depend on timing.  With
// `update` set, the node's velocity replaces the snapshot.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) reduce_partials(const T* __restrict__ src, Geom g,
                                                               double* __restrict__ snap_ux,
                                                               double* __restrict__ snap_uy, int update,
                                                               double* __restrict__ partials)
{
    __shared__ double lds[RED_VALUES][RED_WAVES];
    const int64_t n = (int64_t)g.nx * g.ny;
    double s[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * RED_THREADS) {
        const int y = (int)(i / g.nx), x = (int)(i % g.nx);
        double drho, jx, jy;
        node_moments_f64(src, g, (int64_t)y * g.pitch + x, drho, jx, jy);
        const double r = 1.0 + drho;
        const double vx = jx / r, vy = jy / r;
        const double ox = snap_ux[i], oy = snap_uy[i];
        const double dx = vx - ox, dy = vy - oy;
        s[0] += dx * dx + dy * dy;
        s[1] += vx * vx + vy * vy;
        s[2] += drho;
        s[3] += (__builtin_isfinite(r) && __builtin_isfinite(vx) && __builtin_isfinite(vy)) ? 0.0 : 1.0;
        if (update) {
            snap_ux[i] = vx;
            snap_uy[i] = vy;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < RED_VALUES; ++v) {
        const double t = wave_sum(s[v]);
        if (lane == 0) lds[v][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < RED_VALUES) {
        double t = 0.0;
        for (int w = 0; w < RED_WAVES; ++w) t += lds[threadIdx.x][w];
        partials[(int64_t)blockIdx.x * RED_VALUES + threadIdx.x] = t;
    }
}

} // namespace smrt
