// smrt_api.hip -- host runtime and C ABI (include/smrt.h) of the gfx950 D2Q9
// SRT / SmrtLBM library: parameter checks, workspace layout, kernel dispatch,
// residual and mass read-back.
#include "smrt.h"

#include "host_util.hpp"
#include "lbm_kernels.hpp"
#include "moment_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <limits>
#include <mutex>
#include <new>
#include <string>

namespace smrt {

// One block: sums `nparts` partial rows in a fixed order into out[0..3].
__global__ void __launch_bounds__(RED_THREADS) reduce_finish(const double* __restrict__ partials,
                                                             int nparts, double* __restrict__ out)
{
    __shared__ double lds[RED_VALUES][RED_WAVES];
    double s[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += RED_THREADS)
#pragma unroll
        for (int v = 0; v < RED_VALUES; ++v) s[v] += partials[(int64_t)p * RED_VALUES + v];
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
        out[threadIdx.x] = t;
    }
}

// Device scratch of smrt_mass_noalloc: the reduction's per-block partial
// sums and its four totals, in a file-scope array (one copy per GPU, held
// until the process ends).  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr int SCRATCH_DOUBLES = 2048 * RED_VALUES + RED_VALUES;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

// out[0] = nodes + sum (rho - 1) (the mass), out[1] = non-finite nodes, from
// the four totals of reduce_finish.
__global__ void mass_from_sums(const double* __restrict__ sums, double nodes, double* __restrict__ out)
{
    if (threadIdx.x == 0) {
        out[0] = nodes + sums[2];
        out[1] = sums[3];
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Plain streaming copy, 16 bytes per lane per iteration.
__global__ void __launch_bounds__(256) copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                   int64_t n16)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(src[i], dst + i);
}

} // namespace smrt

namespace smrt_host {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(SMRT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int after_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return SMRT_OK;
}

} // namespace smrt_host

using smrt_host::after_launch;
using smrt_host::fail;
using smrt_host::hip_fail;

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes of the buffer's element type (moment storage: of its moment planes).
size_t elem_bytes(int storage)
{
    switch (storage) {
    case SMRT_F64:
    case SMRT_M64: return 8;
    case SMRT_F32:
    case SMRT_F32X:
    case SMRT_M16:
    case SMRT_MBF16: return 4;
    case SMRT_F16:
    case SMRT_BF16: return 2;
    default: return 0;
    }
}

bool is_moment(int storage) { return storage == SMRT_M64 || storage == SMRT_M16 || storage == SMRT_MBF16; }

// Bytes of one amplitude of the moment storage.
size_t amp_bytes(int storage) { return storage == SMRT_M64 ? 8 : 2; }

// Byte offsets of everything the context keeps in its device workspace.
struct Layout {
    int pitch = 0;       // elements per row; rows start on 256-byte boundaries
    int64_t plane = 0;   // elements per direction plane
    size_t buffer = 0;   // bytes of one population buffer (9 planes)
    size_t off_a = 0, off_b = 0, off_snap_x = 0, off_snap_y = 0, off_partials = 0, off_result = 0;
    size_t total = 0;
    int red_blocks = 0;
};

// Extra bytes between direction planes, so that the nine planes of a
// power-of-two lattice do not start on the same HBM channel.
size_t plane_pad_bytes()
{
    const char* s = std::getenv("SMRT_PLANE_PAD_BYTES");
    if (s && *s) return round_up((size_t)std::strtoull(s, nullptr, 10), kAlign);
    return 4096;
}

Layout make_layout(int nx, int ny, int storage)
{
    Layout L;
    const size_t e = elem_bytes(storage);
    L.pitch = (int)round_up((size_t)nx, kAlign / e);
    const size_t plane_bytes = round_up((size_t)L.pitch * ny * e, 65536) + plane_pad_bytes();
    L.plane = (int64_t)(plane_bytes / e);
    // populations: 9 planes; moments: 3 planes of the moment type and 2 of
    // the amplitude type with the same element count
    L.buffer = is_moment(storage) ? round_up(3 * plane_bytes + 2 * (size_t)L.plane * amp_bytes(storage), kAlign)
                                  : 9 * plane_bytes;
    const size_t n = (size_t)nx * ny;
    L.red_blocks = (int)std::min<size_t>((n + smrt::RED_THREADS - 1) / smrt::RED_THREADS, 2048);
    size_t off = 0;
    L.off_a = off;
    off += round_up(L.buffer, kAlign);
    L.off_b = off;
    off += round_up(L.buffer, kAlign);
    L.off_snap_x = off;
    off += round_up(n * sizeof(double), kAlign);
    L.off_snap_y = off;
    off += round_up(n * sizeof(double), kAlign);
    L.off_partials = off;
    off += round_up((size_t)L.red_blocks * smrt::RED_VALUES * sizeof(double), kAlign);
    L.off_result = off;
    off += kAlign;
    L.total = off;
    return L;
}

int check_params(const smrt_params* p, double* tau_out)
{
    if (!p) return fail(SMRT_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(SMRT_EINVAL, "nx and ny must be >= 3 (got %d x %d)", p->nx, p->ny);
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 34)
        return fail(SMRT_EINVAL, "lattice of %d x %d nodes is too large", p->nx, p->ny);
    if (p->scheme < SMRT_SCHEME_SRT || p->scheme > SMRT_SCHEME_TRT)
        return fail(SMRT_EINVAL, "unknown scheme %d", p->scheme);
    if (p->boundary != SMRT_CAVITY && p->boundary != SMRT_PERIODIC && p->boundary != SMRT_CAVITY_EQLID)
        return fail(SMRT_EINVAL, "unknown boundary %d", p->boundary);
    if (elem_bytes(p->storage) == 0) return fail(SMRT_EINVAL, "unknown storage type %d", p->storage);
    if ((long long)p->nx * (long long)elem_bytes(p->storage) > smrt_host::kMaxRowBytes)
        return fail(SMRT_EINVAL, "rows of %d nodes exceed %lld bytes of stored values", p->nx,
                    smrt_host::kMaxRowBytes);
    if (p->reserved0 != 0) return fail(SMRT_EINVAL, "reserved0 must be 0");
    for (int i = 0; i < 4; ++i)
        if (p->reserved[i] != 0) return fail(SMRT_EINVAL, "reserved[%d] must be 0", i);
    if (!std::isfinite(p->u_lid) || std::fabs(p->u_lid) >= 1.0 / std::sqrt(3.0))
        return fail(SMRT_EINVAL, "|u_lid| must be below the lattice sound speed 1/sqrt(3) (got %g)", p->u_lid);
    double tau = p->tau;
    if (!(tau > 0.0)) {
        // Re = U N / nu and nu = (2 tau - 1)/6 (Eq. relation-chapman-viscosity, e = dx = 1)
        if (!(p->re > 0.0) || !std::isfinite(p->re))
            return fail(SMRT_EINVAL, "tau <= 0 needs a positive Reynolds number (got re = %g)", p->re);
        if (!(std::fabs(p->u_lid) > 0.0))
            return fail(SMRT_EINVAL, "deriving tau from re needs a non-zero lid speed");
        tau = 3.0 * std::fabs(p->u_lid) * (double)p->nx / p->re + 0.5;
    }
    if (!(tau > 0.5) || !std::isfinite(tau))
        return fail(SMRT_EINVAL, "relaxation time must exceed 1/2 (got %.17g)", tau);
    if (is_moment(p->storage) && (p->scheme != SMRT_SCHEME_SMRT || p->boundary == SMRT_CAVITY_EQLID))
        return fail(SMRT_EINVAL, "moment storage holds the SmrtLBM state only, with the moving-wall cavity or periodic "
                                 "boundaries");
    if (p->scheme == SMRT_SCHEME_TRT && (!(p->tau_s > 0.5) || !std::isfinite(p->tau_s)))
        return fail(SMRT_EINVAL, "TRT needs tau_s > 1/2 (got %g)", p->tau_s);
    *tau_out = tau;
    return SMRT_OK;
}

} // namespace

struct smrt_ctx {
    smrt_params p{};
    double tau = 0.0;
    hipStream_t stream = nullptr;
    Layout L;
    char* ws = nullptr;
    bool owns_ws = false;
    double* host_result = nullptr; // pinned, RED_VALUES doubles
    int device = 0;                // HIP device current at creation
    int cur = 0;                   // 0: state in buffer A, 1: in buffer B
    int64_t steps = 0, snap_step = 0;
    int bx = 256, by = 1, rows = 1;
    int fused = 1;                 // time steps per launch (1, or 2 .. 5 with the LDS-blocked kernels)
    int fused_cols = 64, fused_rows = 8; // tile of the multi-step kernels
    int panel = 0;                 // multi-step kernels: tile order (0 = row-major)
    int mom_rows = 8;              // moment storage: tile rows (64 x 8 or 64 x 16)

    void* buffer(int which) const { return ws + (which == 0 ? L.off_a : L.off_b); }
    double* snap_x() const { return reinterpret_cast<double*>(ws + L.off_snap_x); }
    double* snap_y() const { return reinterpret_cast<double*>(ws + L.off_snap_y); }
    double* partials() const { return reinterpret_cast<double*>(ws + L.off_partials); }
    double* result() const { return reinterpret_cast<double*>(ws + L.off_result); }

    smrt::Geom geom() const
    {
        smrt::Geom g;
        g.nx = p.nx;
        g.ny = p.ny;
        g.pitch = L.pitch;
        g.plane = L.plane;
        g.bx = bx;
        g.by = by;
        g.rows = rows;
        g.tiles_x = (p.nx + bx - 1) / bx;
        g.panel = panel;
        return g;
    }
    int64_t nodes() const { return (int64_t)p.nx * p.ny; }
};

namespace {

int elementwise_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65536); }

// Address of the device scratch array on each GPU, taken once per device
// (with that device current) by scratch_setup.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch[kMaxDevices] = {};

int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(SMRT_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[device]) return SMRT_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(smrt::scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = static_cast<double*>(ptr);
    return SMRT_OK;
}

double* scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch[device];
}

template <typename T> int launch_step(smrt_ctx* c, const void* src, void* dst)
{
    using C = typename smrt::Storage<T>::C;
    const smrt::Geom g = c->geom();
    smrt::Coef<C> k;
    const double omega = 1.0 / c->tau;
    const double omega_s = c->p.scheme == SMRT_SCHEME_TRT ? 1.0 / c->p.tau_s : 1.0;
    k.omega = (C)omega;
    k.omega_s = (C)omega_s;
    k.a = (C)(1.0 - omega);
    k.b = (C)(omega_s - omega);
    k.lid = (C)(c->p.boundary == SMRT_CAVITY ? c->p.u_lid / 6.0 : 0.0);
    k.ulid = (C)(c->p.boundary == SMRT_CAVITY_EQLID ? c->p.u_lid : 0.0);
    const int tiles_y = (g.ny + g.by * g.rows - 1) / (g.by * g.rows);
    const int64_t blocks = (int64_t)g.tiles_x * tiles_y;
    if (blocks > std::numeric_limits<int>::max()) return fail(SMRT_EINVAL, "grid too large");
    dim3 grid((unsigned)blocks), block(g.bx, g.by);
    const T* s = static_cast<const T*>(src);
    T* d = static_cast<T*>(dst);
    auto go = [&](auto scheme_tag) {
        constexpr int SCHEME = decltype(scheme_tag)::value;
        switch (c->p.boundary) {
        case SMRT_PERIODIC:
            smrt::stream_collide<T, SCHEME, smrt::PERIODIC><<<grid, block, 0, c->stream>>>(s, d, g, k);
            break;
        case SMRT_CAVITY_EQLID:
            smrt::stream_collide<T, SCHEME, smrt::CAVITY_EQLID><<<grid, block, 0, c->stream>>>(s, d, g, k);
            break;
        default:
            smrt::stream_collide<T, SCHEME, smrt::CAVITY><<<grid, block, 0, c->stream>>>(s, d, g, k);
            break;
        }
    };
    switch (c->p.scheme) {
    case SMRT_SCHEME_SRT: go(std::integral_constant<int, smrt::SRT>{}); break;
    case SMRT_SCHEME_SMRT: go(std::integral_constant<int, smrt::SMRT>{}); break;
    default: go(std::integral_constant<int, smrt::TRT>{}); break;
    }
    return SMRT_OK;
}

// One SmrtLBM step on moment storage: 64 x 8 or 64 x 16 tiles, one node a
// thread.
template <typename MS, int TY> int launch_step_mom_tile(smrt_ctx* c, const void* src, void* dst)
{
    using C = typename smrt::MomPlanes<MS>::C;
    constexpr int TX = 64;
    smrt::Geom g = c->geom();
    g.tiles_x = (g.nx + TX - 1) / TX;
    const int64_t blocks = (int64_t)g.tiles_x * ((g.ny + TY - 1) / TY);
    if (blocks > std::numeric_limits<int>::max()) return fail(SMRT_EINVAL, "grid too large");
    smrt::Coef<C> k;
    k.omega = (C)(1.0 / c->tau);
    k.omega_s = (C)1;
    k.a = (C)(1.0 - 1.0 / c->tau);
    k.b = (C)0;
    k.lid = (C)(c->p.boundary == SMRT_CAVITY ? c->p.u_lid / 6.0 : 0.0);
    k.ulid = (C)0;
    const MS* s = static_cast<const MS*>(src);
    MS* d = static_cast<MS*>(dst);
    if (c->p.boundary == SMRT_PERIODIC)
        smrt::stream_collide_mom<MS, smrt::PERIODIC, TX, TY><<<(unsigned)blocks, TX * TY, 0, c->stream>>>(s, d, g, k);
    else
        smrt::stream_collide_mom<MS, smrt::CAVITY, TX, TY><<<(unsigned)blocks, TX * TY, 0, c->stream>>>(s, d, g, k);
    return SMRT_OK;
}

template <typename MS> int launch_step_mom(smrt_ctx* c, const void* src, void* dst)
{
    if (c->mom_rows == 16) return launch_step_mom_tile<MS, 16>(c, src, dst);
    return launch_step_mom_tile<MS, 8>(c, src, dst);
}

// Threads per multi-step workgroup.  Four- and five-step tiles of 512 nodes
// or more and two-step 64 x 32 tiles take 768: with two workgroups per CU
// (LDS-bound) that is 6 waves per SIMD, which hides more of the latency
// between the HBM and LDS phases (512 and 1024 measured slower, 640 and 896,
// which load the four SIMDs unevenly, much slower); other tiles of 1024
// nodes or more take 512, the rest 256.
constexpr int multi_threads(int steps, int tx, int ty)
{
    return (steps >= 4 && tx * ty >= 512) || (steps == 2 && tx * ty >= 2048) ? 768 : tx * ty >= 1024 ? 512 : 256;
}

template <typename T, int SCHEME, int BC, int TX, int TY, int STEPS>
int launch_multi(smrt_ctx* c, const T* s, T* d, const smrt::Geom& g,
                 const smrt::Coef<typename smrt::Storage<T>::C>& k, int ntiles)
{
    constexpr int NT = multi_threads(STEPS, TX, TY);
    if constexpr (STEPS == 5)
        smrt::stream_collide_x5<T, SCHEME, BC, TX, TY, NT><<<ntiles, NT, 0, c->stream>>>(s, d, g, k);
    else if constexpr (STEPS == 4)
        smrt::stream_collide_x4<T, SCHEME, BC, TX, TY, NT><<<ntiles, NT, 0, c->stream>>>(s, d, g, k);
    else if constexpr (STEPS == 3)
        smrt::stream_collide_x3<T, SCHEME, BC, TX, TY, NT><<<ntiles, NT, 0, c->stream>>>(s, d, g, k);
    else
        smrt::stream_collide_x2<T, SCHEME, BC, TX, TY, NT><<<ntiles, NT, 0, c->stream>>>(s, d, g, k);
    return SMRT_OK;
}

// One launch of the STEPS-step kernel (STEPS = 2 .. 5).
template <typename T, int STEPS, int TX, int TY> int launch_multi_tile(smrt_ctx* c, const void* src, void* dst)
{
    using C = typename smrt::Storage<T>::C;
    smrt::Geom g = c->geom();
    g.tiles_x = (g.nx + TX - 1) / TX;
    g.panel = std::min(c->panel, g.tiles_x); // a wider panel is the same order, and keeps P * tiles_y in range
    const int tiles_y = (g.ny + TY - 1) / TY;
    smrt::Coef<C> k;
    const double omega = 1.0 / c->tau;
    const double omega_s = c->p.scheme == SMRT_SCHEME_TRT ? 1.0 / c->p.tau_s : 1.0;
    k.omega = (C)omega;
    k.omega_s = (C)omega_s;
    k.a = (C)(1.0 - omega);
    k.b = (C)(omega_s - omega);
    k.lid = (C)(c->p.boundary == SMRT_CAVITY ? c->p.u_lid / 6.0 : 0.0);
    k.ulid = (C)0; // the multi-step kernels take the moving-wall lid only
    const int64_t blocks = (int64_t)g.tiles_x * tiles_y;
    if (blocks > std::numeric_limits<int>::max()) return fail(SMRT_EINVAL, "grid too large");
    const int n = (int)blocks;
    const T* s = static_cast<const T*>(src);
    T* d = static_cast<T*>(dst);
    const bool per = c->p.boundary == SMRT_PERIODIC;
    auto go = [&](auto scheme_tag, auto bc_tag) {
        constexpr int SCHEME = decltype(scheme_tag)::value, BC = decltype(bc_tag)::value;
        return launch_multi<T, SCHEME, BC, TX, TY, STEPS>(c, s, d, g, k, n);
    };
    using PER = std::integral_constant<int, smrt::PERIODIC>;
    using CAV = std::integral_constant<int, smrt::CAVITY>;
    switch (c->p.scheme) {
    case SMRT_SCHEME_SRT:
        return per ? go(std::integral_constant<int, smrt::SRT>{}, PER{}) : go(std::integral_constant<int, smrt::SRT>{}, CAV{});
    case SMRT_SCHEME_SMRT:
        return per ? go(std::integral_constant<int, smrt::SMRT>{}, PER{}) : go(std::integral_constant<int, smrt::SMRT>{}, CAV{});
    default:
        return per ? go(std::integral_constant<int, smrt::TRT>{}, PER{}) : go(std::integral_constant<int, smrt::TRT>{}, CAV{});
    }
}

// Two-step tiles offered: 64 x {4, 8, 16, 32} and 128 x {4, 8}.
template <typename T> int launch_step2(smrt_ctx* c, int cols, int rows, const void* src, void* dst)
{
    if (cols == 128) {
        if (rows == 4) return launch_multi_tile<T, 2, 128, 4>(c, src, dst);
        return launch_multi_tile<T, 2, 128, 8>(c, src, dst);
    }
    switch (rows) {
    case 4: return launch_multi_tile<T, 2, 64, 4>(c, src, dst);
    case 16: return launch_multi_tile<T, 2, 64, 16>(c, src, dst);
    case 32: return launch_multi_tile<T, 2, 64, 32>(c, src, dst);
    default: return launch_multi_tile<T, 2, 64, 8>(c, src, dst);
    }
}

// Three- and four-step tiles offered: 64 x {8, 16, 24, 26}.
template <typename T, int STEPS> int launch_step34(smrt_ctx* c, int rows, const void* src, void* dst)
{
    switch (rows) {
    case 16: return launch_multi_tile<T, STEPS, 64, 16>(c, src, dst);
    case 24: return launch_multi_tile<T, STEPS, 64, 24>(c, src, dst);
    case 26: return launch_multi_tile<T, STEPS, 64, 26>(c, src, dst);
    default: return launch_multi_tile<T, STEPS, 64, 8>(c, src, dst);
    }
}

// One launch of k = 2 .. 5 time steps with a 64 x rows tile (2: also
// cols x rows with cols = 128; 5: 64 x 16 or 64 x 22); FP32 and 16-bit
// storage only.
template <typename T> int launch_k(smrt_ctx* c, int k, int cols, int rows, const void* src, void* dst)
{
    if (k == 5)
        return rows == 22 ? launch_multi_tile<T, 5, 64, 22>(c, src, dst) : launch_multi_tile<T, 5, 64, 16>(c, src, dst);
    if (k == 4) return launch_step34<T, 4>(c, rows, src, dst);
    if (k == 3) return launch_step34<T, 3>(c, rows, src, dst);
    return launch_step2<T>(c, cols, rows, src, dst);
}

// FP64 storage: twice the LDS per node, so only 64 x 4 and 64 x 8 tiles for
// two steps and 64 x 8 for three and four.
int launch_k_f64(smrt_ctx* c, int k, int rows, const void* src, void* dst)
{
    if (k == 4) return rows == 10 ? launch_multi_tile<double, 4, 64, 10>(c, src, dst)
                                  : launch_multi_tile<double, 4, 64, 8>(c, src, dst);
    if (k == 3) return launch_multi_tile<double, 3, 64, 8>(c, src, dst);
    if (rows == 4) return launch_multi_tile<double, 2, 64, 4>(c, src, dst);
    return launch_multi_tile<double, 2, 64, 8>(c, src, dst);
}

int dispatch_multi(smrt_ctx* c, int k, int cols, int rows, const void* src, void* dst)
{
    switch (c->p.storage) {
    case SMRT_F64: return launch_k_f64(c, k, rows, src, dst);
    case SMRT_F32: return launch_k<float>(c, k, cols, rows, src, dst);
    case SMRT_F32X: return launch_k<smrt::f32x>(c, k, cols, rows, src, dst);
    case SMRT_F16: return launch_k<_Float16>(c, k, cols, rows, src, dst);
    default: return launch_k<smrt::bf16>(c, k, cols, rows, src, dst);
    }
}

int dispatch_step(smrt_ctx* c, const void* src, void* dst)
{
    switch (c->p.storage) {
    case SMRT_M64: return launch_step_mom<smrt::m64>(c, src, dst);
    case SMRT_M16: return launch_step_mom<smrt::m16>(c, src, dst);
    case SMRT_MBF16: return launch_step_mom<smrt::mbf16>(c, src, dst);
    case SMRT_F64: return launch_step<double>(c, src, dst);
    case SMRT_F32: return launch_step<float>(c, src, dst);
    case SMRT_F32X: return launch_step<smrt::f32x>(c, src, dst);
    case SMRT_F16: return launch_step<_Float16>(c, src, dst);
    default: return launch_step<smrt::bf16>(c, src, dst);
    }
}

// Calls fn(T*) with the state buffer typed by the storage type: population
// storage only (with_storage), moment storage only (with_moment_storage), or
// either (with_any_storage, for the kernels that read the moments of a node).
template <typename Fn> int with_moment_storage(smrt_ctx* c, void* buf, Fn&& fn)
{
    switch (c->p.storage) {
    case SMRT_M64: fn(static_cast<smrt::m64*>(buf)); break;
    case SMRT_M16: fn(static_cast<smrt::m16*>(buf)); break;
    default: fn(static_cast<smrt::mbf16*>(buf)); break;
    }
    return SMRT_OK;
}

template <typename Fn> int with_storage(smrt_ctx* c, void* buf, Fn&& fn);

template <typename Fn> int with_any_storage(smrt_ctx* c, void* buf, Fn&& fn)
{
    return is_moment(c->p.storage) ? with_moment_storage(c, buf, fn) : with_storage(c, buf, fn);
}

template <typename Fn> int with_storage(smrt_ctx* c, void* buf, Fn&& fn)
{
    switch (c->p.storage) {
    case SMRT_F64: fn(static_cast<double*>(buf)); break;
    case SMRT_F32: fn(static_cast<float*>(buf)); break;
    case SMRT_F32X: fn(static_cast<smrt::f32x*>(buf)); break;
    case SMRT_F16: fn(static_cast<_Float16*>(buf)); break;
    default: fn(static_cast<smrt::bf16*>(buf)); break;
    }
    return SMRT_OK;
}

int check_io_dtype(int32_t dtype)
{
    if (dtype != SMRT_F32 && dtype != SMRT_F64)
        return fail(SMRT_EINVAL, "field dtype must be SMRT_F32 or SMRT_F64 (got %d)", dtype);
    return SMRT_OK;
}

// Launches the partial sums (optionally refreshing the snapshot) and the
// finisher; copies the RED_VALUES sums to the pinned host buffer and waits.
int run_reduction(smrt_ctx* c, int update)
{
    const smrt::Geom g = c->geom();
    void* state = c->buffer(c->cur);
    with_any_storage(c, state, [&](auto* s) {
        smrt::reduce_partials<<<c->L.red_blocks, smrt::RED_THREADS, 0, c->stream>>>(
            s, g, c->snap_x(), c->snap_y(), update, c->partials());
    });
    smrt::reduce_finish<<<1, smrt::RED_THREADS, 0, c->stream>>>(c->partials(), c->L.red_blocks, c->result());
    int rc = after_launch("reduction kernels");
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->host_result, c->result(), smrt::RED_VALUES * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SMRT_OK;
}

// Snapshot := current velocity, without a host round trip.
int refresh_snapshot(smrt_ctx* c)
{
    const smrt::Geom g = c->geom();
    with_any_storage(c, c->buffer(c->cur), [&](auto* s) {
        smrt::reduce_partials<<<c->L.red_blocks, smrt::RED_THREADS, 0, c->stream>>>(
            s, g, c->snap_x(), c->snap_y(), 1, c->partials());
    });
    c->steps = 0;
    c->snap_step = 0;
    return after_launch("snapshot refresh");
}

template <typename F> int init_fields_typed(smrt_ctx* c, const void* rho, const void* ux, const void* uy)
{
    const smrt::Geom g = c->geom();
    if (is_moment(c->p.storage))
        with_moment_storage(c, c->buffer(c->cur), [&](auto* s) {
            smrt::init_moments<<<elementwise_blocks(c->nodes()), 256, 0, c->stream>>>(
                s, g, static_cast<const F*>(rho), static_cast<const F*>(ux), static_cast<const F*>(uy));
        });
    else
        with_storage(c, c->buffer(c->cur), [&](auto* s) {
            smrt::init_equilibrium<<<elementwise_blocks(c->nodes()), 256, 0, c->stream>>>(
                s, g, static_cast<const F*>(rho), static_cast<const F*>(ux), static_cast<const F*>(uy));
        });
    return after_launch("init_equilibrium");
}

} // namespace

extern "C" {

size_t smrt_workspace_bytes(const smrt_params* p)
{
    double tau;
    if (check_params(p, &tau) != SMRT_OK) return 0;
    return make_layout(p->nx, p->ny, p->storage).total;
}

int smrt_create(const smrt_params* p, void* dev_ws, size_t ws_bytes, smrt_ctx** out)
{
    try {
        if (!out) return fail(SMRT_EINVAL, "out is NULL");
        *out = nullptr;
        double tau;
        int rc = check_params(p, &tau);
        if (rc) return rc;
        Layout L = make_layout(p->nx, p->ny, p->storage);
        if (dev_ws && ws_bytes < L.total)
            return fail(SMRT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
        if (dev_ws && (reinterpret_cast<uintptr_t>(dev_ws) % kAlign))
            return fail(SMRT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
        smrt_ctx* c = new (std::nothrow) smrt_ctx;
        if (!c) return fail(SMRT_ENOMEM, "out of host memory");
        c->p = *p;
        c->tau = tau;
        c->stream = static_cast<hipStream_t>(p->stream);
        c->L = L;
        // Default block shape: one row segment per block, as wide as the
        // lattice allows (512 measured best on 4096^2, within 1-2% of 256).
        // FP32 and 16-bit storage take the LDS-blocked kernels, tiles in XCD
        // panels of 16 tile columns, or one panel up to 48 (threads per
        // workgroup by tile and step count: multi_threads).  Measured on
        // 512^2 .. 4096^2: FP32 storage five steps per launch, with 64 x 22
        // tiles while that gives >= 1024 workgroups or while 64 x 16 tiles
        // would leave a short second wave (below), else 64 x 16 while that
        // gives >= 256; 16-bit storage four steps, with 64 x 26 tiles while
        // that gives >= 1024 workgroups (the tall tile leaves fewer idle
        // lanes on the rings), else 64 x 16 while that gives >= 256; smaller
        // lattices four steps with 64 x 8 tiles; periodic lattices too small
        // for those rings two steps with 64 x 32 tiles while that gives >= 512
        // workgroups, else with 64 x 4.
        if (p->storage == SMRT_F64) {
            // FP64 (twice the LDS per node): four steps with 64 x 10 tiles
            // (80.6 KB of LDS, two workgroups per CU), measured best on
            // 512^2 .. 4096^2 (3x one step on 4096^2), in XCD panels of 32
            // tile columns (17 % faster than 8 on 4096^2).
            c->fused_cols = 64;
            c->fused_rows = 10;
            c->panel = 32;
            if (p->boundary == SMRT_CAVITY || (p->nx >= 70 && p->ny >= 16)) c->fused = 4;
        } else {
            const int64_t cols = (p->nx + 63) / 64;
            const auto tiles = [&](int rows) { return cols * ((p->ny + rows - 1) / rows); };
            const bool per = p->boundary == SMRT_PERIODIC;
            const auto fits = [&](int steps, int rows) {
                return !per || (p->nx >= 64 + 2 * (steps - 1) && p->ny >= rows + 2 * (steps - 1));
            };
            c->fused_cols = 64;
            // one XCD panel across the whole lattice up to 48 tile columns
            // (five steps: 2048^2 cavity 245.8 GLUPS against 229.8 with panels
            // of 16, 3072^2 274.5 against 268.2), where one row of tiles'
            // rings (~78 KB each) still fits an XCD's 4 MB L2 for the row
            // below; panels of 16 beyond (4096^2: 269.6 against 267.4)
            c->panel = cols <= 48 ? 48 : 16;
            const bool f32 = p->storage == SMRT_F32 || p->storage == SMRT_F32X;
            const int deep = f32 ? 5 : 4, tall = f32 ? 22 : 26;
            // Two 768-thread workgroups are resident per CU (LDS), so a launch
            // runs in waves of 2 x CUs workgroups.  Where 64 x 16 tiles need
            // more than one wave but less than two, FP32's taller tiles avoid a
            // short second wave (five steps: 768^2 cavity 154.7 GLUPS against
            // 140.1, 832^2 177.2 / 153.6, 960^2 171.1 / 165.9; at 1024^2, two
            // full waves, 64 x 16 stays ahead, 175.5 / 172.3).  16-bit storage
            // does so only while its 64 x 26 tiles fit one wave (768^2 +3 %,
            // 832^2 +5 %; 960^2, 555 tiles, -4 %).
            int cus = 256, dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
                cus = 256;
            const int64_t wave = 2 * (int64_t)cus;
            const bool short_second_wave = tiles(16) > wave && tiles(16) < 2 * wave && (f32 || tiles(tall) <= wave);
            if ((tiles(tall) >= 1024 || short_second_wave) && fits(deep, tall)) {
                c->fused = deep;
                c->fused_rows = tall;
            } else if (tiles(16) >= 256 && fits(deep, 16)) {
                c->fused = deep;
                c->fused_rows = 16;
            } else if (fits(4, 8)) {
                // Small lattices are bound by launch latency and fill few CUs:
                // four steps on 64 x 8 tiles (768 threads) beat two steps per
                // launch by 36 .. 52 % on FP32 cavities of 128^2 .. 448^2
                // (256^2: 37.4 GLUPS against 26.7; 448^2: 86.0 against 59.1).
                c->fused = 4;
                c->fused_rows = 8;
            } else {
                c->fused_rows = tiles(32) >= 512 ? 32 : 4;
                if (per && p->ny < c->fused_rows + 2) c->fused_rows = 4;
                if (fits(2, c->fused_rows)) c->fused = 2;
            }
        }
        if (p->boundary == SMRT_CAVITY_EQLID || is_moment(p->storage)) c->fused = 1; // one-step kernels only
        if (p->nx >= 512) {
            c->bx = 512; c->by = 1;
        } else if (p->nx >= 256) {
            c->bx = 256; c->by = 1;
        } else if (p->nx >= 128) {
            c->bx = 128; c->by = 2;
        } else {
            c->bx = 64; c->by = 4;
        }
        hipError_t e = hipGetDevice(&c->device);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipGetDevice");
        }
        rc = scratch_setup(c->device);
        if (rc) {
            delete c;
            return rc;
        }
        if (dev_ws) {
            c->ws = static_cast<char*>(dev_ws);
        } else {
            e = hipMalloc(reinterpret_cast<void**>(&c->ws), L.total);
            if (e != hipSuccess) {
                delete c;
                return fail(SMRT_ENOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
            }
            c->owns_ws = true;
        }
        e = hipHostMalloc(reinterpret_cast<void**>(&c->host_result), smrt::RED_VALUES * sizeof(double),
                          hipHostMallocDefault);
        if (e != hipSuccess) {
            smrt_destroy(c);
            return fail(SMRT_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        }
        rc = init_fields_typed<float>(c, nullptr, nullptr, nullptr);
        if (!rc) rc = refresh_snapshot(c);
        if (rc) {
            smrt_destroy(c);
            return rc;
        }
        *out = c;
        return SMRT_OK;
    } catch (...) {
        return fail(SMRT_ENOMEM, "unexpected host exception in smrt_create");
    }
}

int smrt_init_fields(smrt_ctx* c, const void* rho, const void* ux, const void* uy, int32_t dtype)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    int rc = check_io_dtype(dtype);
    if (rc) return rc;
    rc = dtype == SMRT_F64 ? init_fields_typed<double>(c, rho, ux, uy) : init_fields_typed<float>(c, rho, ux, uy);
    if (rc) return rc;
    return refresh_snapshot(c);
}

int smrt_set_populations(smrt_ctx* c, const void* f, int32_t dtype)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (!f) return fail(SMRT_EINVAL, "populations pointer is NULL");
    int rc = check_io_dtype(dtype);
    if (rc) return rc;
    const smrt::Geom g = c->geom();
    const int blocks = elementwise_blocks(c->nodes());
    if (is_moment(c->p.storage))
        with_moment_storage(c, c->buffer(c->cur), [&](auto* s) {
            if (dtype == SMRT_F64)
                smrt::set_populations_mom<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<const double*>(f));
            else
                smrt::set_populations_mom<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<const float*>(f));
        });
    else
        with_storage(c, c->buffer(c->cur), [&](auto* s) {
            if (dtype == SMRT_F64)
                smrt::set_populations<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<const double*>(f));
            else
                smrt::set_populations<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<const float*>(f));
        });
    rc = after_launch("set_populations");
    if (rc) return rc;
    return refresh_snapshot(c);
}

int smrt_get_populations(smrt_ctx* c, void* f, int32_t dtype)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (!f) return fail(SMRT_EINVAL, "populations pointer is NULL");
    int rc = check_io_dtype(dtype);
    if (rc) return rc;
    const smrt::Geom g = c->geom();
    const int blocks = elementwise_blocks(c->nodes());
    if (is_moment(c->p.storage))
        with_moment_storage(c, c->buffer(c->cur), [&](auto* s) {
            if (dtype == SMRT_F64)
                smrt::get_populations_mom<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<double*>(f));
            else
                smrt::get_populations_mom<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<float*>(f));
        });
    else
        with_storage(c, c->buffer(c->cur), [&](auto* s) {
            if (dtype == SMRT_F64)
                smrt::get_populations<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<double*>(f));
            else
                smrt::get_populations<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<float*>(f));
        });
    return after_launch("get_populations");
}

int smrt_step(smrt_ctx* c, int64_t n)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (n < 0) return fail(SMRT_EINVAL, "step count must be >= 0 (got %lld)", (long long)n);
    int64_t left = n;
    while (left > 0) {
        // the largest launch that fits: fused steps, then one shorter launch
        // with 64 x 16 tiles (64 x 8 after a mode with shorter tiles, and for
        // FP64 storage), whose rings need no more room on a periodic lattice
        // than the deeper mode's
        const int k = (int)std::min<int64_t>(c->fused, left);
        const void* src = c->buffer(c->cur);
        void* dst = c->buffer(c->cur ^ 1);
        int rc;
        if (k == 1)
            rc = dispatch_step(c, src, dst);
        else if (k < c->fused)
            rc = dispatch_multi(c, k, 64, c->fused_rows >= 16 ? 16 : 8, src, dst);
        else
            rc = dispatch_multi(c, k, c->fused_cols, c->fused_rows, src, dst);
        if (rc) return rc;
        c->cur ^= 1;
        c->steps += k;
        left -= k;
    }
    return n ? after_launch("stream_collide") : SMRT_OK;
}

int smrt_moments(smrt_ctx* c, void* rho, void* ux, void* uy, int32_t dtype)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    int rc = check_io_dtype(dtype);
    if (rc) return rc;
    if (!rho && !ux && !uy) return SMRT_OK;
    const smrt::Geom g = c->geom();
    const int blocks = elementwise_blocks(c->nodes());
    with_any_storage(c, c->buffer(c->cur), [&](auto* s) {
        if (dtype == SMRT_F64)
            smrt::export_moments<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<double*>(rho),
                                                                static_cast<double*>(ux), static_cast<double*>(uy));
        else
            smrt::export_moments<<<blocks, 256, 0, c->stream>>>(s, g, static_cast<float*>(rho),
                                                                static_cast<float*>(ux), static_cast<float*>(uy));
    });
    return after_launch("export_moments");
}

int smrt_residual(smrt_ctx* c, double* out)
{
    if (!c || !out) return fail(SMRT_EINVAL, "context or output is NULL");
    const int64_t window = c->steps - c->snap_step;
    if (window <= 0) return fail(SMRT_ESTATE, "no step since the last residual snapshot");
    int rc = run_reduction(c, 1);
    if (rc) return rc;
    c->snap_step = c->steps;
    const double du2 = c->host_result[0], u2 = c->host_result[1], bad = c->host_result[3];
    if (bad != 0.0 || !std::isfinite(du2) || !std::isfinite(u2)) {
        *out = std::numeric_limits<double>::quiet_NaN();
        return fail(SMRT_EUNSTABLE, "%.0f nodes hold a non-finite density or velocity", bad);
    }
    if (u2 == 0.0)
        *out = du2 == 0.0 ? 0.0 : std::numeric_limits<double>::infinity();
    else
        *out = std::sqrt(du2) / ((double)window * std::sqrt(u2));
    return SMRT_OK;
}

int smrt_mass(smrt_ctx* c, double* out)
{
    if (!c || !out) return fail(SMRT_EINVAL, "context or output is NULL");
    int rc = run_reduction(c, 0);
    if (rc) return rc;
    const double drho = c->host_result[2], bad = c->host_result[3];
    if (bad != 0.0 || !std::isfinite(drho)) {
        *out = std::numeric_limits<double>::quiet_NaN();
        return fail(SMRT_EUNSTABLE, "%.0f nodes hold a non-finite density or velocity", bad);
    }
    *out = (double)c->nodes() + drho;
    return SMRT_OK;
}

int smrt_mass_noalloc(smrt_ctx* c, double* dev_out)
{
    if (!c || !dev_out) return fail(SMRT_EINVAL, "context or output is NULL");
    const int nparts = c->L.red_blocks;
    if ((int64_t)nparts * smrt::RED_VALUES + smrt::RED_VALUES > smrt::SCRATCH_DOUBLES)
        return fail(SMRT_EINVAL, "%d reduction blocks exceed the %d doubles of device scratch", nparts,
                    smrt::SCRATCH_DOUBLES);
    double* scratch = scratch_ptr(c->device);
    if (!scratch) return fail(SMRT_ESTATE, "device scratch of device %d was not set up", c->device);
    double* partials = scratch;
    double* sums = scratch + (int64_t)nparts * smrt::RED_VALUES;
    const smrt::Geom g = c->geom();
    with_any_storage(c, c->buffer(c->cur), [&](auto* s) {
        smrt::reduce_partials<<<nparts, smrt::RED_THREADS, 0, c->stream>>>(s, g, c->snap_x(), c->snap_y(), 0,
                                                                           partials);
    });
    smrt::reduce_finish<<<1, smrt::RED_THREADS, 0, c->stream>>>(partials, nparts, sums);
    smrt::mass_from_sums<<<1, 64, 0, c->stream>>>(sums, (double)c->nodes(), dev_out);
    return after_launch("mass reduction (device scratch)");
}

int64_t smrt_steps_done(const smrt_ctx* c) { return c ? c->steps : -1; }

double smrt_tau(const smrt_ctx* c) { return c ? c->tau : std::numeric_limits<double>::quiet_NaN(); }

int smrt_set_launch(smrt_ctx* c, int32_t bx, int32_t by, int32_t rows)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (is_moment(c->p.storage)) {
        if (bx != 64 || ((int64_t)by * rows != 8 && (int64_t)by * rows != 16))
            return fail(SMRT_EINVAL, "moment storage takes 64 x 8 or 64 x 16 tiles (got %d x %d x %d)", bx, by, rows);
        c->mom_rows = by * rows;
        return SMRT_OK;
    }
    const int64_t threads = (int64_t)bx * by;
    if (bx < 16 || bx % 16 || by < 1 || (threads != 64 && threads != 128 && threads != 256 && threads != 512 &&
                                          threads != 1024))
        return fail(SMRT_EINVAL, "invalid block shape %d x %d", bx, by);
    if (rows < 1 || rows > 8) return fail(SMRT_EINVAL, "rows per thread must be in 1..8 (got %d)", rows);
    c->bx = bx;
    c->by = by;
    c->rows = rows;
    return SMRT_OK;
}

int smrt_set_steps_per_launch(smrt_ctx* c, int32_t steps, int32_t tile_cols, int32_t tile_rows)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (steps < 1 || steps > 5) return fail(SMRT_EINVAL, "steps per launch must be 1 .. 5 (got %d)", steps);
    if (steps > 1 && c->p.boundary == SMRT_CAVITY_EQLID)
        return fail(SMRT_EINVAL, "the equilibrium lid runs one time step per launch");
    if (steps > 1 && is_moment(c->p.storage))
        return fail(SMRT_EINVAL, "moment storage runs one time step per launch");
    if (steps == 1) { // one step per launch has no tile: keep the multi-step one
        c->fused = 1;
        return SMRT_OK;
    }
    if (tile_cols == 0) tile_cols = 64;
    if (tile_rows == 0) tile_rows = steps >= 3 && c->p.storage != SMRT_F64 ? 16 : 8;
    bool ok;
    if (c->p.storage == SMRT_F64)
        ok = steps <= 4 && tile_cols == 64 &&
             (tile_rows == 8 || (steps == 4 && tile_rows == 10) || (steps == 2 && tile_rows == 4));
    else if (steps == 5)
        ok = tile_cols == 64 && (tile_rows == 16 || tile_rows == 22);
    else
        ok = steps >= 3 ? tile_cols == 64 && (tile_rows == 8 || tile_rows == 16 || tile_rows == 24 || tile_rows == 26)
                        : (tile_cols == 64 && (tile_rows == 4 || tile_rows == 8 || tile_rows == 16 || tile_rows == 32)) ||
                              (tile_cols == 128 && (tile_rows == 4 || tile_rows == 8));
    if (!ok) return fail(SMRT_EINVAL, "%d-step tile %d x %d not offered", steps, tile_cols, tile_rows);
    {
        // A periodic ring wraps once, which needs the lattice wider than the tile plus its rings.
        const int ring = steps - 1;
        if (c->p.boundary == SMRT_PERIODIC && (c->p.nx < tile_cols + 2 * ring || c->p.ny < tile_rows + 2 * ring))
            return fail(SMRT_EINVAL, "periodic %d-step launches need nx >= %d and ny >= %d", steps,
                        tile_cols + 2 * ring, tile_rows + 2 * ring);
    }
    c->fused = steps;
    c->fused_cols = tile_cols;
    c->fused_rows = tile_rows;
    return SMRT_OK;
}

int32_t smrt_get_steps_per_launch(const smrt_ctx* c) { return c ? c->fused : -1; }

int smrt_set_tile_order(smrt_ctx* c, int32_t panel_cols)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    if (panel_cols < 0) return fail(SMRT_EINVAL, "panel width must be >= 0 (got %d)", panel_cols);
    c->panel = panel_cols;
    return SMRT_OK;
}

int smrt_synchronize(smrt_ctx* c)
{
    if (!c) return fail(SMRT_EINVAL, "context is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SMRT_OK;
}

void smrt_destroy(smrt_ctx* c)
{
    if (!c) return;
    if (c->host_result) (void)hipHostFree(c->host_result);
    if (c->owns_ws && c->ws) (void)hipFree(c->ws);
    delete c;
}

const char* smrt_last_error(void) { return smrt_host::g_error.c_str(); }

int smrt_copy_kernel(const void* src, void* dst, size_t bytes, void* stream)
{
    if (!src || !dst) return fail(SMRT_EINVAL, "copy pointers must not be NULL");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(SMRT_EINVAL, "copy size and pointers must be multiples of 16 bytes");
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return SMRT_OK;
    const int blocks = (int)std::min<int64_t>((n16 + 255) / 256, (int64_t)1 << 30);
    smrt::copy_kernel<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const smrt::u32x4*>(src), static_cast<smrt::u32x4*>(dst), n16);
    return after_launch("copy_kernel");
}

} // extern "C"
