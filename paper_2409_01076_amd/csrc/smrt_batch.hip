// smrt_batch.hip -- host runtime of the cavity batches (smrt_batch_* in
// include/smrt.h): workspace layout, the device tile table, graph-captured
// step windows, per-cavity residual checks with retirement, and the launch
// autotuner.
#include "smrt.h"

#include "batch_kernels.hpp"
#include "host_util.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <type_traits>
#include <vector>

using smrt_host::after_launch;
using smrt_host::fail;
using smrt_host::hip_fail;

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage)
{
    switch (storage) {
    case SMRT_F64: return 8;
    case SMRT_F32: return 4;
    case SMRT_F16:
    case SMRT_BF16: return 2;
    default: return 0;
    }
}

// Launch shapes the autotuner tries (threads per block bx * by).
const smrt::BatchLaunch kShapes[] = {{64, 4}, {128, 2}, {256, 1}, {32, 8}, {64, 8}, {128, 4}, {256, 2}, {512, 1}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
// Steps per captured graph (even, so a replay leaves the buffer parity as it was).
constexpr int kGraphSteps = 64;

int64_t tiles_of(int nx, int ny, smrt::BatchLaunch L)
{
    return (int64_t)((nx + L.bx - 1) / L.bx) * ((ny + L.by - 1) / L.by);
}

struct Plan {
    std::vector<smrt::CavityDesc> desc;
    std::vector<double> tau;
    size_t state_elems = 0;  // elements of T for all population buffers
    size_t snap_doubles = 0; // 2 per node
    int max_tiles = 0;       // largest table over all shapes
    size_t off_state = 0, off_snap = 0, off_partials = 0, off_result = 0, off_table = 0, off_ranges = 0,
           off_ntiles = 0, off_desc = 0, total = 0;
    int partial_rows = 0;
};

int make_plan(const smrt_batch_params* p, Plan* out)
{
    if (!p) return fail(SMRT_EINVAL, "batch params is NULL");
    if (p->count < 1) return fail(SMRT_EINVAL, "batch needs at least one cavity (count = %d)", p->count);
    if (!p->nx || !p->ny) return fail(SMRT_EINVAL, "nx and ny arrays are required");
    if (p->scheme < SMRT_SCHEME_SRT || p->scheme > SMRT_SCHEME_TRT)
        return fail(SMRT_EINVAL, "unknown scheme %d", p->scheme);
    const size_t e = elem_bytes(p->storage);
    if (!e) return fail(SMRT_EINVAL, "unknown storage type %d", p->storage);
    if (p->reserved0) return fail(SMRT_EINVAL, "reserved0 must be 0");
    for (int i = 0; i < 4; ++i)
        if (p->reserved[i]) return fail(SMRT_EINVAL, "reserved[%d] must be 0", i);
    if (!std::isfinite(p->u_lid) || std::fabs(p->u_lid) >= 1.0 / std::sqrt(3.0))
        return fail(SMRT_EINVAL, "|u_lid| must be below 1/sqrt(3) (got %g)", p->u_lid);
    if (p->scheme == SMRT_SCHEME_TRT && (!(p->tau_s > 0.5) || !std::isfinite(p->tau_s)))
        return fail(SMRT_EINVAL, "TRT needs tau_s > 1/2 (got %g)", p->tau_s);
    Plan P;
    P.desc.resize(p->count);
    P.tau.resize(p->count);
    size_t elems = 0, snap = 0;
    std::vector<int64_t> tiles_per_shape(kNumShapes, 0);
    for (int i = 0; i < p->count; ++i) {
        const int nx = p->nx[i], ny = p->ny[i];
        if (nx < 3 || ny < 3) return fail(SMRT_EINVAL, "cavity %d: nx and ny must be >= 3 (got %d x %d)", i, nx, ny);
        if ((int64_t)nx * ny > (int64_t)1 << 34)
            return fail(SMRT_EINVAL, "cavity %d: %d x %d nodes is too large", i, nx, ny);
        if ((long long)nx * (long long)e > smrt_host::kMaxRowBytes)
            return fail(SMRT_EINVAL, "cavity %d: rows of %d nodes exceed %lld bytes of stored values", i, nx,
                        smrt_host::kMaxRowBytes);
        double tau = p->tau ? p->tau[i] : 0.0;
        if (!(tau > 0.0)) {
            const double re = p->re ? p->re[i] : 0.0;
            if (!(re > 0.0) || !std::isfinite(re) || !(std::fabs(p->u_lid) > 0.0))
                return fail(SMRT_EINVAL, "cavity %d: give tau, or re > 0 with a moving lid", i);
            // Re = U N / nu, nu = (2 tau - 1)/6 (Eq. relation-chapman-viscosity, e = dx = 1)
            tau = 3.0 * std::fabs(p->u_lid) * (double)nx / re + 0.5;
        }
        if (!(tau > 0.5) || !std::isfinite(tau))
            return fail(SMRT_EINVAL, "cavity %d: relaxation time must exceed 1/2 (got %.17g)", i, tau);
        smrt::CavityDesc& c = P.desc[i];
        c.nx = nx;
        c.ny = ny;
        c.pitch = (int)round_up((size_t)nx, kAlign / e);
        c.plane = (int64_t)round_up((size_t)c.pitch * ny, kAlign / e);
        const size_t buffer = 9 * (size_t)c.plane;
        c.off[0] = (int64_t)elems;
        c.off[1] = (int64_t)(elems + buffer);
        elems += 2 * buffer;
        c.snap = (int64_t)snap;
        snap += 2 * (size_t)nx * ny;
        const double omega = 1.0 / tau;
        const double omega_s = p->scheme == SMRT_SCHEME_TRT ? 1.0 / p->tau_s : 1.0;
        c.omega = omega;
        c.omega_s = omega_s;
        c.a = 1.0 - omega;
        c.b = omega_s - omega;
        c.lid = p->u_lid / 6.0;
        c.tiles_x = 0; // set per launch shape
        P.tau[i] = tau;
        for (int s = 0; s < kNumShapes; ++s) tiles_per_shape[s] += tiles_of(nx, ny, kShapes[s]);
    }
    const int64_t max_tiles = *std::max_element(tiles_per_shape.begin(), tiles_per_shape.end());
    if (max_tiles > std::numeric_limits<int>::max())
        return fail(SMRT_EINVAL, "batch of %lld tiles is too large", (long long)max_tiles);
    P.max_tiles = (int)max_tiles;
    P.state_elems = elems;
    P.snap_doubles = snap;
    // partial rows: one per tile in the batch reduction, and up to 2048 blocks
    // when a single cavity's snapshot is refreshed with the lattice kernel
    P.partial_rows = std::max(P.max_tiles, 2048);
    size_t off = 0;
    P.off_state = off;
    off += round_up(elems * e, kAlign);
    P.off_snap = off;
    off += round_up(snap * sizeof(double), kAlign);
    P.off_partials = off;
    off += round_up((size_t)P.partial_rows * smrt::RED_VALUES * sizeof(double), kAlign);
    P.off_result = off;
    off += round_up((size_t)p->count * smrt::RED_VALUES * sizeof(double), kAlign);
    P.off_table = off;
    off += round_up((size_t)P.max_tiles * sizeof(int2), kAlign);
    P.off_ranges = off;
    off += round_up((size_t)p->count * sizeof(int2), kAlign);
    P.off_ntiles = off;
    off += kAlign;
    P.off_desc = off;
    off += round_up((size_t)p->count * sizeof(smrt::CavityDesc), kAlign);
    P.total = off;
    *out = std::move(P);
    return SMRT_OK;
}

} // namespace

struct smrt_batch {
    smrt_batch_params p{};
    Plan plan;
    hipStream_t stream = nullptr;   // the caller's stream
    hipStream_t capture = nullptr;  // private stream used only to capture graphs
    char* ws = nullptr;
    bool owns_ws = false;
    double* host_result = nullptr;  // pinned, count * RED_VALUES
    smrt::BatchLaunch shape{64, 4};
    int multi = 1;                  // time steps per launch (2 and 3: the LDS-blocked kernels)
    int grid = 0;                   // workgroups per step launch
    int parity = 0;                 // buffer holding the running cavities' state
    int64_t steps = 0, snap_step = 0;
    std::vector<int> status, final_parity;
    std::vector<int64_t> done_steps;
    std::vector<double> last_residual;
    std::vector<int> table_order;   // running cavities in table order
    int ntiles = 0;
    hipGraphExec_t exec[2] = {nullptr, nullptr}; // by starting parity
    hipGraph_t graph[2] = {nullptr, nullptr};

    char* state() const { return ws + plan.off_state; }
    double* snap() const { return reinterpret_cast<double*>(ws + plan.off_snap); }
    double* partials() const { return reinterpret_cast<double*>(ws + plan.off_partials); }
    double* result() const { return reinterpret_cast<double*>(ws + plan.off_result); }
    int2* table() const { return reinterpret_cast<int2*>(ws + plan.off_table); }
    int2* ranges() const { return reinterpret_cast<int2*>(ws + plan.off_ranges); }
    int* ntiles_dev() const { return reinterpret_cast<int*>(ws + plan.off_ntiles); }
    smrt::CavityDesc* desc() const { return reinterpret_cast<smrt::CavityDesc*>(ws + plan.off_desc); }
};

namespace {

void drop_graphs(smrt_batch* b)
{
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

// Uploads the per-cavity descriptors for the current shape, and the tile
// table and ranges of the running cavities; waits for the copies.
int upload_tables(smrt_batch* b)
{
    std::vector<smrt::CavityDesc> desc = b->plan.desc;
    for (auto& c : desc) c.tiles_x = (c.nx + b->shape.bx - 1) / b->shape.bx;
    std::vector<int2> table, ranges;
    b->table_order.clear();
    for (int i = 0; i < b->p.count; ++i) {
        if (b->status[i] != SMRT_RUNNING) continue;
        const int n = (int)tiles_of(desc[i].nx, desc[i].ny, b->shape); // the plan keeps the sum in int range
        ranges.push_back(make_int2((int)table.size(), n));
        for (int t = 0; t < n; ++t) table.push_back(make_int2(i, t));
        b->table_order.push_back(i);
    }
    b->ntiles = (int)table.size();
    const int n = b->ntiles;
    // The copies read these local buffers: wait for them even when one fails.
    hipError_t e = hipMemcpyAsync(b->desc(), desc.data(), desc.size() * sizeof(smrt::CavityDesc),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !table.empty())
        e = hipMemcpyAsync(b->table(), table.data(), table.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !table.empty())
        e = hipMemcpyAsync(b->ranges(), ranges.data(), ranges.size() * sizeof(int2), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ntiles_dev(), &n, sizeof(int), hipMemcpyHostToDevice, b->stream);
    const hipError_t w = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "upload_tables: hipMemcpyAsync");
    if (w != hipSuccess) return hip_fail(w, "upload_tables: hipStreamSynchronize");
    return SMRT_OK;
}

// Threads per multi-step workgroup, as for single lattices: 768 for four-
// and five-step tiles (64 x 8, 64 x 16 and 64 x 22), 512 for other 64 x 16
// and 64 x 22 tiles, 256 for smaller.
constexpr int multi_threads(int steps, int ty) { return steps >= 4 && ty >= 8 ? 768 : ty >= 16 ? 512 : 256; }

template <typename T, int SCHEME, int TY>
void launch_two_tile(smrt_batch* b, hipStream_t s, int parity, dim3 grid)
{
    constexpr int NT = multi_threads(2, TY);
    smrt::batch_stream_collide_x2<T, SCHEME, 64, TY, NT><<<grid, NT, 0, s>>>(
        b->desc(), b->table(), b->ntiles_dev(), reinterpret_cast<T*>(b->state()), parity);
}

template <typename T, int SCHEME, int TY>
void launch_three_tile(smrt_batch* b, hipStream_t s, int parity, dim3 grid)
{
    constexpr int NT = multi_threads(3, TY);
    smrt::batch_stream_collide_x3<T, SCHEME, 64, TY, NT><<<grid, NT, 0, s>>>(
        b->desc(), b->table(), b->ntiles_dev(), reinterpret_cast<T*>(b->state()), parity);
}

template <typename T, int SCHEME, int TY>
void launch_four_tile(smrt_batch* b, hipStream_t s, int parity, dim3 grid)
{
    constexpr int NT = multi_threads(4, TY);
    smrt::batch_stream_collide_x4<T, SCHEME, 64, TY, NT><<<grid, NT, 0, s>>>(
        b->desc(), b->table(), b->ntiles_dev(), reinterpret_cast<T*>(b->state()), parity);
}

template <typename T, int SCHEME, int TY>
void launch_five_tile(smrt_batch* b, hipStream_t s, int parity, dim3 grid)
{
    constexpr int NT = multi_threads(5, TY);
    smrt::batch_stream_collide_x5<T, SCHEME, 64, TY, NT><<<grid, NT, 0, s>>>(
        b->desc(), b->table(), b->ntiles_dev(), reinterpret_cast<T*>(b->state()), parity);
}

template <typename T, int SCHEME> void launch_one(smrt_batch* b, hipStream_t s, int parity, dim3 grid)
{
    dim3 block(b->shape.bx, std::min(b->shape.by, 1024 / b->shape.bx)); // 64 x 22 tiles: two row passes
    smrt::batch_stream_collide<T, SCHEME><<<grid, block, 0, s>>>(b->desc(), b->table(), b->ntiles_dev(),
                                                                reinterpret_cast<T*>(b->state()), parity, b->shape);
}

template <typename T, int SCHEME>
void launch_multi_or_one(smrt_batch* b, hipStream_t s, int parity, int k, dim3 grid)
{
    if (k == 5) {
        if (b->shape.by == 22) launch_five_tile<T, SCHEME, 22>(b, s, parity, grid);
        else if (b->shape.by == 16) launch_five_tile<T, SCHEME, 16>(b, s, parity, grid);
        else launch_five_tile<T, SCHEME, 8>(b, s, parity, grid);
        return;
    }
    if (k == 4) {
        if (b->shape.by == 22) launch_four_tile<T, SCHEME, 22>(b, s, parity, grid);
        else if (b->shape.by == 16) launch_four_tile<T, SCHEME, 16>(b, s, parity, grid);
        else launch_four_tile<T, SCHEME, 8>(b, s, parity, grid);
        return;
    }
    if (k == 3) {
        if (b->shape.by == 22) launch_three_tile<T, SCHEME, 22>(b, s, parity, grid);
        else if (b->shape.by == 16) launch_three_tile<T, SCHEME, 16>(b, s, parity, grid);
        else launch_three_tile<T, SCHEME, 8>(b, s, parity, grid);
        return;
    }
    if (k == 2) {
        if (b->shape.by == 22) launch_two_tile<T, SCHEME, 22>(b, s, parity, grid);
        else if (b->shape.by == 16) launch_two_tile<T, SCHEME, 16>(b, s, parity, grid);
        else if (b->shape.by == 8) launch_two_tile<T, SCHEME, 8>(b, s, parity, grid);
        else launch_two_tile<T, SCHEME, 4>(b, s, parity, grid);
        return;
    }
    launch_one<T, SCHEME>(b, s, parity, grid);
}

// One launch of k time steps (k = 2 .. 5: 64 x shape.by tiles, one a
// workgroup; the tile
// table is built for that shape, so a shorter remainder launch uses the same
// table).  FP64 batches take one step per launch (multi_steps), so their
// multi-step kernels are not built.
template <typename T, int SCHEME> void launch_typed_scheme(smrt_batch* b, hipStream_t s, int parity, int k)
{
    // the multi-step kernels take one tile a workgroup: never fewer
    // workgroups than tiles, and a multiple of 8 (their XCD-contiguous order)
    const int g = k > 1 ? (std::max(b->grid, b->ntiles) + 7) / 8 * 8 : b->grid;
    dim3 grid((unsigned)std::max(g, 1));
    if constexpr (!std::is_same_v<T, double>) launch_multi_or_one<T, SCHEME>(b, s, parity, k, grid);
    else launch_one<T, SCHEME>(b, s, parity, grid);
}

template <typename T> void launch_step_typed(smrt_batch* b, hipStream_t s, int parity, int k)
{
    switch (b->p.scheme) {
    case SMRT_SCHEME_SRT: launch_typed_scheme<T, smrt::SRT>(b, s, parity, k); break;
    case SMRT_SCHEME_SMRT: launch_typed_scheme<T, smrt::SMRT>(b, s, parity, k); break;
    default: launch_typed_scheme<T, smrt::TRT>(b, s, parity, k); break;
    }
}

// One launch of k = 1 .. 5 time steps (FP64 storage has only the one-step
// kernel).
void launch_step(smrt_batch* b, hipStream_t s, int parity, int k)
{
    switch (b->p.storage) {
    case SMRT_F64: launch_step_typed<double>(b, s, parity, 1); break;
    case SMRT_F32: launch_step_typed<float>(b, s, parity, k); break;
    case SMRT_F16: launch_step_typed<_Float16>(b, s, parity, k); break;
    default: launch_step_typed<smrt::bf16>(b, s, parity, k); break;
    }
}

// Time steps per launch in the current mode (FP64: always 1).
int multi_steps(const smrt_batch* b) { return b->p.storage == SMRT_F64 ? 1 : b->multi; }

// Captures kGraphSteps launches (of multi_steps(b) steps each) starting from
// `parity` on the private stream and instantiates them.
int capture_graph(smrt_batch* b, int parity)
{
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < kGraphSteps; ++i) launch_step(b, b->capture, parity ^ (i & 1), multi_steps(b));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph[parity] = g;
    b->exec[parity] = x;
    return SMRT_OK;
}

int enqueue_steps(smrt_batch* b, int64_t n)
{
    if (b->ntiles == 0 || n <= 0) return SMRT_OK;
    const int unit = multi_steps(b);
    const int64_t per_graph = (int64_t)kGraphSteps * unit;
    while (n > 0) {
        if (n >= per_graph) {
            if (!b->exec[b->parity]) {
                int rc = capture_graph(b, b->parity);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(b->exec[b->parity], b->stream));
            n -= per_graph;
            b->steps += per_graph;
        } else {
            const int k = (int)std::min<int64_t>(unit, n);
            launch_step(b, b->stream, b->parity, k);
            int rc = after_launch("batch_stream_collide");
            if (rc) return rc;
            b->parity ^= 1;
            n -= k;
            b->steps += k;
        }
    }
    return SMRT_OK;
}

// Per running cavity (table order): the four FP64 sums, copied to host_result.
template <typename T> void launch_reduce_typed(smrt_batch* b, int update)
{
    const int grid = std::min(b->ntiles, 4096);
    dim3 block(b->shape.bx, std::min(b->shape.by, 1024 / b->shape.bx)); // 64 x 22 tiles: two row passes
    smrt::batch_reduce_partials<T><<<grid, block, 0, b->stream>>>(b->desc(), b->table(), b->ntiles_dev(),
                                                                  reinterpret_cast<const T*>(b->state()), b->parity,
                                                                  b->shape, b->snap(), update, b->partials());
}

int reduce_running(smrt_batch* b, int update)
{
    if (b->ntiles == 0) return SMRT_OK;
    switch (b->p.storage) {
    case SMRT_F64: launch_reduce_typed<double>(b, update); break;
    case SMRT_F32: launch_reduce_typed<float>(b, update); break;
    case SMRT_F16: launch_reduce_typed<_Float16>(b, update); break;
    default: launch_reduce_typed<smrt::bf16>(b, update); break;
    }
    const int nrun = (int)b->table_order.size();
    smrt::batch_reduce_finish<<<nrun, smrt::RED_THREADS, 0, b->stream>>>(b->partials(), b->ranges(), b->result());
    int rc = after_launch("batch reduction");
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->host_result, b->result(), (size_t)nrun * smrt::RED_VALUES * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return SMRT_OK;
}

int check_index(const smrt_batch* b, int32_t index)
{
    if (!b) return fail(SMRT_EINVAL, "batch is NULL");
    if (index < 0 || index >= b->p.count)
        return fail(SMRT_EINVAL, "cavity index %d out of range [0, %d)", index, b->p.count);
    return SMRT_OK;
}

smrt::Geom geom_of(const smrt::CavityDesc& c)
{
    smrt::Geom g{};
    g.nx = c.nx;
    g.ny = c.ny;
    g.pitch = c.pitch;
    g.plane = c.plane;
    g.bx = 256;
    g.by = 1;
    g.rows = 1;
    g.tiles_x = (c.nx + 255) / 256;
    return g;
}

template <typename Fn> void with_storage(const smrt_batch* b, Fn&& fn)
{
    switch (b->p.storage) {
    case SMRT_F64: fn((double*)nullptr); break;
    case SMRT_F32: fn((float*)nullptr); break;
    case SMRT_F16: fn((_Float16*)nullptr); break;
    default: fn((smrt::bf16*)nullptr); break;
    }
}

} // namespace

extern "C" {

size_t smrt_batch_workspace_bytes(const smrt_batch_params* p)
{
    Plan P;
    if (make_plan(p, &P) != SMRT_OK) return 0;
    return P.total;
}

int smrt_batch_create(const smrt_batch_params* p, void* dev_ws, size_t ws_bytes, smrt_batch** out)
{
    try {
        if (!out) return fail(SMRT_EINVAL, "out is NULL");
        *out = nullptr;
        Plan P;
        int rc = make_plan(p, &P);
        if (rc) return rc;
        if (dev_ws && ws_bytes < P.total)
            return fail(SMRT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, P.total);
        if (dev_ws && (reinterpret_cast<uintptr_t>(dev_ws) % kAlign))
            return fail(SMRT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
        smrt_batch* b = new (std::nothrow) smrt_batch;
        if (!b) return fail(SMRT_ENOMEM, "out of host memory");
        b->p = *p;
        b->p.nx = b->p.ny = nullptr; // host arrays are not kept
        b->p.tau = b->p.re = nullptr;
        b->plan = std::move(P);
        b->stream = static_cast<hipStream_t>(p->stream);
        b->status.assign(p->count, SMRT_RUNNING);
        b->final_parity.assign(p->count, 0);
        b->done_steps.assign(p->count, 0);
        b->last_residual.assign(p->count, std::numeric_limits<double>::quiet_NaN());
        hipError_t e;
        if (dev_ws) {
            b->ws = static_cast<char*>(dev_ws);
        } else {
            e = hipMalloc(reinterpret_cast<void**>(&b->ws), b->plan.total);
            if (e != hipSuccess) {
                delete b;
                return fail(SMRT_ENOMEM, "hipMalloc(%zu): %s", b->plan.total, hipGetErrorString(e));
            }
            b->owns_ws = true;
        }
        e = hipHostMalloc(reinterpret_cast<void**>(&b->host_result),
                          (size_t)p->count * smrt::RED_VALUES * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            smrt_batch_destroy(b);
            return fail(SMRT_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        }
        e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            smrt_batch_destroy(b);
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        // Cold start: d = 0 (all-zero bits in every storage type) and u = 0.
        const size_t eb = elem_bytes(p->storage);
        e = hipMemsetAsync(b->state(), 0, b->plan.state_elems * eb, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->snap(), 0, b->plan.snap_doubles * sizeof(double), b->stream);
        if (e != hipSuccess) {
            smrt_batch_destroy(b);
            return hip_fail(e, "hipMemsetAsync");
        }
        // Default launch: one pass over the table per launch; FP64 one step
        // per launch with 64 x 4 tiles, FP32 64 x 22 tiles with five steps
        // per launch (the autotuner's choice for 256 cavities of 64 .. 512
        // nodes a side), 16-bit storage 64 x 16 tiles with three.
        b->shape = p->storage == SMRT_F64 ? kShapes[0]
                   : p->storage == SMRT_F32 ? smrt::BatchLaunch{64, 22}
                                            : smrt::BatchLaunch{64, 16};
        b->multi = p->storage == SMRT_F64 ? 1 : p->storage == SMRT_F32 ? 5 : 3;
        int64_t total_tiles = 0;
        for (const auto& c : b->plan.desc) total_tiles += tiles_of(c.nx, c.ny, b->shape);
        b->grid = (int)total_tiles; // at most the plan's max_tiles
        rc = upload_tables(b);
        if (rc) {
            smrt_batch_destroy(b);
            return rc;
        }
        *out = b;
        return SMRT_OK;
    } catch (...) {
        return fail(SMRT_ENOMEM, "unexpected host exception in smrt_batch_create");
    }
}

int smrt_batch_step(smrt_batch* b, int64_t n)
{
    if (!b) return fail(SMRT_EINVAL, "batch is NULL");
    if (n < 0) return fail(SMRT_EINVAL, "step count must be >= 0");
    return enqueue_steps(b, n);
}

int smrt_batch_run(smrt_batch* b, double tol, int64_t window, int64_t max_steps, int64_t* steps_out,
                   int32_t* status_out, double* residual_out)
{
    if (!b) return fail(SMRT_EINVAL, "batch is NULL");
    if (window < 1 || max_steps < 0 || !(tol >= 0.0))
        return fail(SMRT_EINVAL, "window must be >= 1, max_steps >= 0 and tol >= 0");
    try {
        int64_t done = 0;
        while (b->ntiles > 0 && done < max_steps) {
            const int64_t k = std::min(window, max_steps - done);
            int rc = enqueue_steps(b, k);
            if (rc) return rc;
            done += k;
            rc = reduce_running(b, 1);
            if (rc) return rc;
            const int64_t span = b->steps - b->snap_step;
            b->snap_step = b->steps;
            bool changed = false;
            for (size_t j = 0; j < b->table_order.size(); ++j) {
                const int i = b->table_order[j];
                const double* r = b->host_result + j * smrt::RED_VALUES;
                const double du2 = r[0], u2 = r[1], bad = r[3];
                int st = SMRT_RUNNING;
                double res;
                if (bad != 0.0 || !std::isfinite(du2) || !std::isfinite(u2)) {
                    res = std::numeric_limits<double>::quiet_NaN();
                    st = SMRT_UNSTABLE;
                } else {
                    res = u2 == 0.0 ? (du2 == 0.0 ? 0.0 : std::numeric_limits<double>::infinity())
                                    : std::sqrt(du2) / ((double)span * std::sqrt(u2));
                    if (res < tol) st = SMRT_STEADY;
                }
                b->last_residual[i] = res;
                b->done_steps[i] = b->steps;
                if (st != SMRT_RUNNING) {
                    b->status[i] = st;
                    b->final_parity[i] = b->parity;
                    changed = true;
                }
            }
            if (changed) {
                rc = upload_tables(b);
                if (rc) return rc;
            }
        }
        for (int i = 0; i < b->p.count; ++i) {
            if (b->status[i] == SMRT_RUNNING) b->done_steps[i] = b->steps;
            if (steps_out) steps_out[i] = b->done_steps[i];
            if (status_out) status_out[i] = b->status[i];
            if (residual_out) residual_out[i] = b->last_residual[i];
        }
        return SMRT_OK;
    } catch (...) {
        return fail(SMRT_ENOMEM, "unexpected host exception in smrt_batch_run");
    }
}

int smrt_batch_autotune(smrt_batch* b, int32_t steps, int32_t* chosen)
{
    if (!b) return fail(SMRT_EINVAL, "batch is NULL");
    if (steps < 2 || steps % 2) return fail(SMRT_EINVAL, "autotune steps must be even and >= 2 (got %d)", steps);
    if (b->ntiles == 0) return fail(SMRT_ESTATE, "no running cavity to tune on");
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    // timing events, destroyed on every return
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    HIP_TRY(hipEventCreate(&ev.e[0]));
    HIP_TRY(hipEventCreate(&ev.e[1]));
    hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
    float best = std::numeric_limits<float>::infinity();
    smrt::BatchLaunch best_shape = b->shape;
    int best_grid = b->grid;
    int best_multi = b->multi;
    int rc = SMRT_OK;
    // Candidates: every one-step shape (with four grid sizes), then (except
    // for FP64) the two-step kernel with 64 x 4, 64 x 8 and 64 x 16 tiles,
    // the three- and four-step kernels with 64 x 8 and 64 x 16 tiles and the
    // five-step kernel with 64 x 16 and 64 x 22 tiles (one tile a workgroup,
    // so the full grid only); times are per time step.
    static const int kMultiSteps[] = {2, 2, 2, 3, 3, 4, 4, 5, 5};
    static const int kMultiRows[] = {4, 8, 16, 8, 16, 8, 16, 16, 22};
    const int n_multi = b->p.storage == SMRT_F64 ? 0 : 9;
    for (int s = 0; s < kNumShapes + n_multi && rc == SMRT_OK; ++s) {
        const int multi = s >= kNumShapes ? kMultiSteps[s - kNumShapes] : 1;
        b->shape = multi > 1 ? smrt::BatchLaunch{64, kMultiRows[s - kNumShapes]} : kShapes[s];
        b->multi = multi;
        rc = upload_tables(b);
        if (rc) break;
        const int per_block_waves = multi > 1 ? multi_threads(multi, b->shape.by) / 64 : (b->shape.bx * b->shape.by) / 64;
        const int grids[] = {b->ntiles, cus * std::max(1, 8 / per_block_waves), cus * std::max(1, 16 / per_block_waves),
                             cus * std::max(1, 32 / per_block_waves)};
        for (int gi = 0; gi < 4; ++gi) {
            b->grid = std::min(grids[gi], b->ntiles);
            if (gi > 0 && (multi > 1 || grids[gi] >= b->ntiles)) continue; // full grid only / same as it
            const int unit = multi;
            const int launches = std::max(2, steps / unit) & ~1; // even: parity kept
            launch_step(b, b->stream, b->parity, unit); // warm-up pair
            launch_step(b, b->stream, b->parity ^ 1, unit);
            HIP_TRY(hipEventRecord(e0, b->stream));
            for (int k = 0; k < launches; ++k) launch_step(b, b->stream, b->parity ^ (k & 1), unit);
            HIP_TRY(hipEventRecord(e1, b->stream));
            rc = after_launch("batch autotune");
            if (rc) break;
            HIP_TRY(hipEventSynchronize(e1));
            b->steps += (int64_t)(launches + 2) * unit;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            const float per_step = ms / (float)(launches * unit);
            if (per_step < best) {
                best = per_step;
                best_shape = b->shape;
                best_grid = b->grid;
                best_multi = multi;
            }
        }
    }
    if (rc) return rc;
    b->shape = best_shape;
    b->multi = best_multi;
    rc = upload_tables(b);
    if (rc) return rc;
    b->grid = std::min(best_grid, b->ntiles);
    drop_graphs(b);
    if (chosen) {
        chosen[0] = b->shape.bx;
        chosen[1] = b->shape.by;
        chosen[2] = b->grid;
    }
    return SMRT_OK;
}

int smrt_batch_set_launch(smrt_batch* b, int32_t bx, int32_t by, int32_t steps)
{
    if (!b) return fail(SMRT_EINVAL, "batch is NULL");
    bool ok = false;
    if (steps == 1) {
        for (const auto& sh : kShapes) ok |= sh.bx == bx && sh.by == by;
    } else if (steps >= 2 && steps <= 5 && b->p.storage != SMRT_F64 && bx == 64) {
        ok = by == 8 || by == 16 || by == 22 || (by == 4 && steps == 2);
    }
    if (!ok)
        return fail(SMRT_EINVAL, "batch launch %d x %d with %d steps is not built for this storage", bx, by, steps);
    b->shape = smrt::BatchLaunch{bx, by};
    b->multi = steps;
    const int rc = upload_tables(b);
    if (rc) return rc;
    b->grid = std::max(b->ntiles, 1);
    drop_graphs(b);
    return SMRT_OK;
}

int smrt_batch_moments(smrt_batch* b, int32_t index, void* rho, void* ux, void* uy, int32_t dtype)
{
    int rc = check_index(b, index);
    if (rc) return rc;
    if (dtype != SMRT_F32 && dtype != SMRT_F64) return fail(SMRT_EINVAL, "field dtype must be F32 or F64");
    if (!rho && !ux && !uy) return SMRT_OK;
    const smrt::CavityDesc& c = b->plan.desc[index];
    const int buf = b->status[index] == SMRT_RUNNING ? b->parity : b->final_parity[index];
    const smrt::Geom g = geom_of(c);
    const int blocks = (int)std::min<int64_t>(((int64_t)c.nx * c.ny + 255) / 256, 65536);
    with_storage(b, [&](auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        const T* src = reinterpret_cast<const T*>(b->state()) + c.off[buf];
        if (dtype == SMRT_F64)
            smrt::export_moments<<<blocks, 256, 0, b->stream>>>(src, g, (double*)rho, (double*)ux, (double*)uy);
        else
            smrt::export_moments<<<blocks, 256, 0, b->stream>>>(src, g, (float*)rho, (float*)ux, (float*)uy);
    });
    return after_launch("batch export_moments");
}

int smrt_batch_init_fields(smrt_batch* b, int32_t index, const void* rho, const void* ux, const void* uy,
                           int32_t dtype)
{
    int rc = check_index(b, index);
    if (rc) return rc;
    if (dtype != SMRT_F32 && dtype != SMRT_F64) return fail(SMRT_EINVAL, "field dtype must be F32 or F64");
    if (b->status[index] != SMRT_RUNNING) return fail(SMRT_ESTATE, "cavity %d has finished", index);
    const smrt::CavityDesc& c = b->plan.desc[index];
    const smrt::Geom g = geom_of(c);
    const int64_t n = (int64_t)c.nx * c.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    const int red_blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
    double* sx = b->snap() + c.snap;
    with_storage(b, [&](auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        T* dst = reinterpret_cast<T*>(b->state()) + c.off[b->parity];
        if (dtype == SMRT_F64)
            smrt::init_equilibrium<<<blocks, 256, 0, b->stream>>>(dst, g, (const double*)rho, (const double*)ux,
                                                                  (const double*)uy);
        else
            smrt::init_equilibrium<<<blocks, 256, 0, b->stream>>>(dst, g, (const float*)rho, (const float*)ux,
                                                                  (const float*)uy);
        smrt::reduce_partials<<<red_blocks, smrt::RED_THREADS, 0, b->stream>>>(dst, g, sx, sx + n, 1,
                                                                               b->partials());
    });
    return after_launch("batch init_fields");
}

int64_t smrt_batch_steps_done(const smrt_batch* b) { return b ? b->steps : -1; }

int32_t smrt_batch_running(const smrt_batch* b) { return b ? (int32_t)b->table_order.size() : -1; }

void smrt_batch_destroy(smrt_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->host_result) (void)hipHostFree(b->host_result);
    if (b->owns_ws && b->ws) (void)hipFree(b->ws);
    delete b;
}

int32_t smrt_batch_steps_per_launch(const smrt_batch* b) { return b ? multi_steps(b) : -1; }

} // extern "C"
