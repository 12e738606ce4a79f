// batch_kernels.hpp -- gfx950 device code for many independent lid-driven
// cavities advanced together, one launch per time step for the whole batch.
//
// Every cavity keeps its own two structure-of-arrays population buffers and
// its own velocity snapshot inside one workspace.  A device table lists the
// tiles (bx x by nodes) of the cavities still running; a fixed grid of
// workgroups walks that table (grid-stride), so one launch covers any mix of
// sizes and the table can shrink as cavities finish without changing the
// launch or a captured graph.  The per-node update is the same gather /
// collide / store as the single-lattice kernel, so a cavity in a batch is
// bitwise identical to the same cavity run alone.
#pragma once

#include "lbm_kernels.hpp"

namespace smrt {

struct CavityDesc {
    int nx, ny, pitch, tiles_x;
    int64_t plane;   // elements per direction plane
    int64_t off[2];  // element offsets of buffer 0 and buffer 1
    int64_t snap;    // offset (doubles) of the ux snapshot; uy follows after nx*ny
    double omega, omega_s, a, b, lid;
};

struct BatchLaunch {
    int bx, by; // tile (and, for one-step launches, block) shape
};

// Descriptor tables are read-only during a launch and the same for a whole
// workgroup; reading them through the constant address space lets the
// compiler use scalar loads instead of vector loads plus a wait.
typedef __attribute__((address_space(4))) const CavityDesc ConstDesc;

__device__ __forceinline__ CavityDesc load_desc(const CavityDesc* cav, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((ConstDesc*)cav)[i];
#else
    return cav[i]; // host pass: never executed
#endif
}

template <typename C> __device__ __forceinline__ Coef<C> coef_of(const CavityDesc& c)
{
    Coef<C> k;
    k.omega = (C)c.omega;
    k.omega_s = (C)c.omega_s;
    k.a = (C)c.a;
    k.b = (C)c.b;
    k.lid = (C)c.lid;
    k.ulid = (C)0; // the batch's lid is the moving wall
    return k;
}

// One time step of every listed tile.  `parity` selects the source buffer.
// Block: bx x by_block threads (by_block <= by, at most 1024 threads);
// thread (x, y) updates rows y, y + by_block, ... of the tile, so a
// multi-step tile shape taller than 1024 / bx rows can take a one-step
// remainder launch on its own table.
template <typename T, int SCHEME>
__global__ void __launch_bounds__(1024) batch_stream_collide(const CavityDesc* __restrict__ cav,
                                                             const int2* __restrict__ tiles,
                                                             const int* __restrict__ ntiles_p,
                                                             T* __restrict__ base, int parity,
                                                             BatchLaunch L)
{
    using C = typename Storage<T>::C;
    const int ntiles = *ntiles_p;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tt = tiles[t];
        // The tile entry is the same for the whole workgroup: keep it, and the
        // descriptor it points to, in scalar registers (scalar loads), so the
        // population loads can be issued without waiting on vector loads.
        const CavityDesc c = load_desc(cav, __builtin_amdgcn_readfirstlane(tt.x));
        Geom g;
        g.nx = c.nx;
        g.ny = c.ny;
        g.pitch = c.pitch;
        g.plane = c.plane;
        g.bx = L.bx;
        g.by = L.by;
        g.rows = 1;
        g.tiles_x = c.tiles_x;
        g.panel = 0;
        const int ti = __builtin_amdgcn_readfirstlane(tt.y);
        const int ytile = (ti / c.tiles_x) * L.by;
        const int x = (ti % c.tiles_x) * L.bx + threadIdx.x;
        // select, not c.off[parity]: a runtime index into the local copy of
        // the descriptor would put it in scratch memory
        const T* src = base + (parity ? c.off[1] : c.off[0]);
        T* dst = base + (parity ? c.off[0] : c.off[1]);
        const PullBases<T> pb = pull_bases(src, g, ytile > 0 ? ytile - 1 : 0);
        const StoreBases<T> sb = store_bases(dst, g, ytile);
        if (x >= c.nx) continue;
        const Coef<C> k = coef_of<C>(c);
        for (int yy = threadIdx.y; yy < L.by; yy += blockDim.y) {
            const int y = ytile + yy;
            if (y >= c.ny) break;
            C d[9];
            const bool edge = (x == 0) | (x == c.nx - 1) | (y == 0) | (y == c.ny - 1);
            if (edge)
                gather_edge<T, CAVITY>(src, g, x, y, d, (C)c.lid);
            else
                gather_interior<T>(pb, g, x, y, d);
            collide<SCHEME, T>(d, k);
            scatter_store<T>(sb, g, x, y, d);
        }
    }
}

// Every multi-step kernel below is built for two resident workgroups per CU
// (the LDS allows two): NT / 128 waves per SIMD, which caps the registers.
//
// S time steps of one listed tile per workgroup: the batch form of the
// multi-step kernels (stream_collide_x2 .. _x5, same phases through LDS), for
// tiles of TX x TY nodes and NT threads.  Cavity walls need no wrap, so any
// size works.  The host launches at least as many workgroups as the table
// has tiles, rounded up to a multiple of 8; those left without a tile return.  (A grid-stride
// loop over the table kept the tile body's addresses live from one tile to
// the next: 80 VGPRs with scratch spills against 48 without it, for 64 x 16
// tiles.)
//
// Workgroups go to the 8 XCDs round-robin (workgroup b to XCD b mod 8).
// With n tiles listed and c = ceil(n / 8), workgroup b takes tile
// (b mod 8) c + b / 8 (none when b / 8 >= c): each XCD walks one contiguous
// eighth of the table, so the neighbouring tiles of a cavity, whose halo rows
// and columns overlap, meet in the same L2.  In table order the neighbours
// land on different XCDs and every halo line comes from HBM again (2.4x the
// algorithmic reads, measured, against 1.06x in this order).  The split
// follows the current table, not the grid, so a table that shrinks as
// cavities finish still spreads over all eight XCDs.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int c = (ntiles + 7) >> 3, q = b >> 3;
    return q < c ? (b & 7) * c + q : ntiles;
}

template <typename T, int SCHEME, int TX, int TY, int NT, int S>
__device__ __forceinline__ void batch_multi(const CavityDesc* __restrict__ cav, const int2* __restrict__ tiles,
                                            const int* __restrict__ ntiles_p, T* __restrict__ base, int parity,
                                            MultiTile<T, TX, TY, S>& sh)
{
    using C = typename Storage<T>::C;
    const int ntiles = *ntiles_p;
    const int t = xcd_tile(blockIdx.x, ntiles);
    if (t >= ntiles) return;
    const int2 tt = tiles[t];
    const CavityDesc c = load_desc(cav, __builtin_amdgcn_readfirstlane(tt.x));
    const int ti = __builtin_amdgcn_readfirstlane(tt.y);
    Geom g;
    g.nx = c.nx;
    g.ny = c.ny;
    g.pitch = c.pitch;
    g.plane = c.plane;
    g.bx = TX;
    g.by = TY;
    g.rows = 1;
    g.tiles_x = c.tiles_x;
    g.panel = 0;
    const T* src = base + (parity ? c.off[1] : c.off[0]);
    T* dst = base + (parity ? c.off[0] : c.off[1]);
    const Coef<C> k = coef_of<C>(c);
    const int X0 = (ti % c.tiles_x) * TX, Y0 = (ti / c.tiles_x) * TY;
    multi_tile<T, SCHEME, CAVITY, TX, TY, NT, S>(src, dst, g, k, X0, Y0, sh);
}

template <typename T, int SCHEME, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT, NT / 128) batch_stream_collide_x2(const CavityDesc* __restrict__ cav,
                                                              const int2* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p,
                                                              T* __restrict__ base, int parity)
{
    __shared__ MultiTile<T, TX, TY, 2> sh;
    batch_multi<T, SCHEME, TX, TY, NT, 2>(cav, tiles, ntiles_p, base, parity, sh);
}

template <typename T, int SCHEME, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT, NT / 128) batch_stream_collide_x3(const CavityDesc* __restrict__ cav,
                                                              const int2* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p,
                                                              T* __restrict__ base, int parity)
{
    __shared__ MultiTile<T, TX, TY, 3> sh;
    batch_multi<T, SCHEME, TX, TY, NT, 3>(cav, tiles, ntiles_p, base, parity, sh);
}

template <typename T, int SCHEME, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT, NT / 128) batch_stream_collide_x4(const CavityDesc* __restrict__ cav,
                                                              const int2* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p,
                                                              T* __restrict__ base, int parity)
{
    __shared__ MultiTile<T, TX, TY, 4> sh;
    batch_multi<T, SCHEME, TX, TY, NT, 4>(cav, tiles, ntiles_p, base, parity, sh);
}

template <typename T, int SCHEME, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT, NT / 128) batch_stream_collide_x5(const CavityDesc* __restrict__ cav,
                                                              const int2* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p,
                                                              T* __restrict__ base, int parity)
{
    __shared__ MultiTile<T, TX, TY, 5> sh;
    batch_multi<T, SCHEME, TX, TY, NT, 5>(cav, tiles, ntiles_p, base, parity, sh);
}

// Per-tile FP64 partial sums (|u - u_snap|^2, |u|^2, rho - 1, non-finite
// nodes) of every listed tile, in a fixed order; optionally refreshes the
// snapshots.  Block: bx x by_block threads with by_block <= by and at most
// 1024 threads; thread (x, y) takes rows y, y + by_block, ... of the tile.
template <typename T>
__global__ void __launch_bounds__(1024) batch_reduce_partials(const CavityDesc* __restrict__ cav,
                                                              const int2* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p,
                                                              const T* __restrict__ base, int parity,
                                                              BatchLaunch L, double* __restrict__ snap_base,
                                                              int update, double* __restrict__ partials)
{
    __shared__ double lds[RED_VALUES][16];
    const int ntiles = *ntiles_p;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int nwaves = (blockDim.x * blockDim.y + 63) / 64;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tt = tiles[t];
        const CavityDesc c = load_desc(cav, __builtin_amdgcn_readfirstlane(tt.x));
        const int ti = __builtin_amdgcn_readfirstlane(tt.y);
        const int x = (ti % c.tiles_x) * L.bx + threadIdx.x;
        double s[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
        for (int yy = threadIdx.y; yy < L.by; yy += blockDim.y) {
            const int y = (ti / c.tiles_x) * L.by + yy;
            if (x >= c.nx || y >= c.ny) continue;
            Geom g;
            g.plane = c.plane;
            double drho, jx, jy;
            node_moments_f64(base + (parity ? c.off[1] : c.off[0]), g, (int64_t)y * c.pitch + x, drho, jx, jy);
            const double r = 1.0 + drho, vx = jx / r, vy = jy / r;
            double* sx = snap_base + c.snap + (int64_t)y * c.nx + x;
            double* sy = sx + (int64_t)c.nx * c.ny;
            const double dx = vx - *sx, dy = vy - *sy;
            s[0] += dx * dx + dy * dy;
            s[1] += vx * vx + vy * vy;
            s[2] += drho;
            s[3] += (__builtin_isfinite(r) && __builtin_isfinite(vx) && __builtin_isfinite(vy)) ? 0.0 : 1.0;
            if (update) {
                *sx = vx;
                *sy = vy;
            }
        }
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int v = 0; v < RED_VALUES; ++v) {
            const double w = wave_sum(s[v]);
            if (lane == 0) lds[v][wave] = w;
        }
        __syncthreads();
        if (tid < RED_VALUES) {
            double acc = 0.0;
            for (int w = 0; w < nwaves; ++w) acc += lds[tid][w];
            partials[(int64_t)t * RED_VALUES + tid] = acc;
        }
        __syncthreads();
    }
}

// One block per listed cavity: sums its tiles' partials (a contiguous range
// of the table, in order) into out[cavity slot].
__global__ void __launch_bounds__(RED_THREADS) batch_reduce_finish(const double* __restrict__ partials,
                                                                   const int2* __restrict__ ranges,
                                                                   double* __restrict__ out)
{
    __shared__ double lds[RED_VALUES][RED_WAVES];
    const int2 r = ranges[blockIdx.x]; // (first tile, tile count)
    double s[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < r.y; p += RED_THREADS)
#pragma unroll
        for (int v = 0; v < RED_VALUES; ++v) s[v] += partials[(int64_t)(r.x + p) * RED_VALUES + v];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < RED_VALUES; ++v) {
        const double w = wave_sum(s[v]);
        if (lane == 0) lds[v][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x < RED_VALUES) {
        double acc = 0.0;
        for (int w = 0; w < RED_WAVES; ++w) acc += lds[threadIdx.x][w];
        out[(int64_t)blockIdx.x * RED_VALUES + threadIdx.x] = acc;
    }
}

} // namespace smrt
