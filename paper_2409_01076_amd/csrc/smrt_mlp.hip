// smrt_mlp.hip -- host runtime of the warm-start network (smrt_mlp_* in
// include/smrt.h): parameter layout, forward pass, backward pass, Adam.
//
// Network: features [x, y, s, sin(2 pi B p), cos(2 pi B p)] -> (layers - 1)
// SiLU layers of `width` -> linear layer of `outputs`.  Compute: bf16
// operands on MFMA with FP32 accumulation; FP32 master weights, biases and
// Adam state.  Pre-activations are not stored: the backward pass recomputes
// them (bitwise) from the stored bf16 activations.
#include "smrt.h"

#include "host_util.hpp"
#include "mlp_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <new>
#include <vector>

using smrt_host::after_launch;
using smrt_host::fail;
using smrt_host::hip_fail;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinSplitRows = 256;           // rows per weight-gradient row block, at least
constexpr size_t kPartialBytes = 512u << 20; // budget of the row-block partials
// Workgroups of a forward layer and of the input-gradient part of a
// backward grid, each looping over row tiles with the next tile's rows in
// flight.  At 65,536 rows a training step measured the same with 512, 768
// and 1024 forward groups and slower with 256.  The backward grid adds 256
// weight-gradient blocks to its input-gradient groups; 256 of these (one of
// each kind a CU) measured 0.179 ms a step, 384 0.194, 512 0.200, 128 0.200.
constexpr int kForwardGroups = 512;
constexpr int kBackwardGroups = 256;
// The one-launch forward pass: one workgroup of 12 waves a CU (its weights fill the LDS).
constexpr int kFusedGroups = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct MlpLayout {
    int layers = 0, width = 0, nf = 0, outputs = 0, max_batch = 0;
    int k0 = 0, k0_real = 0, n_last = 0;
    std::vector<int> in, out, in_real, out_real; // padded and real sizes per layer
    std::vector<size_t> w_off, b_off;             // offsets (floats) in the padded parameter block
    size_t padded_params = 0, real_params = 0;
    int max_splits = 256;
    smrt::mlp::LayerTable table;
    // byte offsets in the workspace
    size_t off_params = 0, off_wbf = 0, off_wbf_t = 0, off_grad = 0, off_m = 0, off_v = 0, off_fourier = 0,
           off_x0 = 0, off_a = 0, off_y = 0, off_dy = 0, off_dz0 = 0, off_dz1 = 0, off_wpart = 0, off_loss = 0,
           total = 0;
    size_t a_stride = 0; // elements between hidden layers' activation arrays
    int loss_blocks = 0;
};

int make_layout(const smrt_mlp_params* p, MlpLayout* out)
{
    if (!p) return fail(SMRT_EINVAL, "mlp params is NULL");
    if (p->inputs != 3) return fail(SMRT_EINVAL, "the network takes 3 inputs (x, y, s), got %d", p->inputs);
    if (p->fourier < 0 || p->fourier > 64) return fail(SMRT_EINVAL, "fourier features must be in 0..64");
    if (p->width < 64 || p->width % 64 || p->width > 1024)
        return fail(SMRT_EINVAL, "width must be a multiple of 64 in 64..1024 (got %d)", p->width);
    if (p->layers < 2 || p->layers > smrt::mlp::kMaxLayers)
        return fail(SMRT_EINVAL, "layers must be in 2..%d (got %d)", smrt::mlp::kMaxLayers, p->layers);
    if (p->outputs < 1 || p->outputs > 64) return fail(SMRT_EINVAL, "outputs must be in 1..64");
    if (p->max_batch < 64 || p->max_batch % 64 || p->max_batch > (1 << 24))
        return fail(SMRT_EINVAL, "max_batch must be a positive multiple of 64 up to 2^24 (got %d)", p->max_batch);
    for (int i = 0; i < 4; ++i)
        if (p->reserved[i]) return fail(SMRT_EINVAL, "reserved[%d] must be 0", i);
    MlpLayout L;
    L.layers = p->layers;
    L.width = p->width;
    L.nf = p->fourier;
    L.outputs = p->outputs;
    L.max_batch = p->max_batch;
    L.k0_real = 3 + 2 * p->fourier;
    L.k0 = (int)round_up((size_t)L.k0_real, 64);
    if (L.k0 > smrt::mlp::kMaxFeatureWidth) return fail(SMRT_EINVAL, "too many input features (%d)", L.k0);
    L.n_last = 64;
    for (int l = 0; l < L.layers; ++l) {
        L.in.push_back(l == 0 ? L.k0 : L.width);
        L.in_real.push_back(l == 0 ? L.k0_real : L.width);
        L.out.push_back(l == L.layers - 1 ? L.n_last : L.width);
        L.out_real.push_back(l == L.layers - 1 ? L.outputs : L.width);
    }
    size_t pp = 0, rp = 0;
    L.table.layers = L.layers;
    for (int l = 0; l < L.layers; ++l) {
        L.w_off.push_back(pp);
        L.table.off[l] = (int64_t)pp;
        L.table.in[l] = L.in[l];
        L.table.out[l] = L.out[l];
        pp += (size_t)L.in[l] * L.out[l];
        L.b_off.push_back(pp);
        pp += L.out[l];
        rp += (size_t)L.in_real[l] * L.out_real[l] + L.out_real[l];
    }
    L.table.off[L.layers] = (int64_t)pp;
    L.padded_params = pp;
    L.real_params = rp;
    // every layer's row-block partials are kept until one pass sums them all
    while (L.max_splits > 1 && (size_t)L.max_splits * pp * 4 > kPartialBytes) L.max_splits >>= 1;
    const size_t mb = (size_t)L.max_batch;
    L.loss_blocks = kForwardGroups;
    const int hidden = L.layers - 1;
    L.a_stride = mb * L.width;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round_up(bytes, kAlign);
        return o;
    };
    L.off_params = take(pp * 4);
    L.off_wbf = take(pp * 2);
    L.off_wbf_t = take(pp * 2);
    L.off_grad = take(pp * 4);
    L.off_m = take(pp * 4);
    L.off_v = take(pp * 4);
    L.off_fourier = take((size_t)std::max(1, L.nf) * 3 * 4);
    L.off_x0 = take(mb * L.k0 * 2);
    L.off_a = take((size_t)hidden * L.a_stride * 2);
    L.off_y = take(mb * L.outputs * 4);
    L.off_dy = take(mb * L.n_last * 2);
    L.off_dz0 = take(mb * L.width * 2);
    L.off_dz1 = take(mb * L.width * 2);
    // per layer and row block: the weight-gradient partial (in x out) and the
    // bias-gradient partial (out) after it, laid out as the layer's W and b
    L.off_wpart = take((size_t)L.max_splits * pp * 4);
    L.off_loss = take((size_t)L.loss_blocks * 8);
    L.total = off;
    *out = std::move(L);
    return SMRT_OK;
}

} // namespace

struct smrt_mlp {
    MlpLayout L;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    bool owns_ws = false;
    int64_t adam_steps = 0;
    int loss_parts = 0; // squared-error partials written by the last forward pass with a target
    bool fused = true;  // one launch for the whole forward pass where the network fits
    bool dz_ready = false; // the last forward pass also wrote dZ_{L-2} into dz(0)
    bool has_params = false;
    std::vector<double> loss_host;

    float* params() const { return reinterpret_cast<float*>(ws + L.off_params); }
    uint16_t* wbf() const { return reinterpret_cast<uint16_t*>(ws + L.off_wbf); }
    uint16_t* wbf_t() const { return reinterpret_cast<uint16_t*>(ws + L.off_wbf_t); }
    float* grad() const { return reinterpret_cast<float*>(ws + L.off_grad); }
    float* adam_m() const { return reinterpret_cast<float*>(ws + L.off_m); }
    float* adam_v() const { return reinterpret_cast<float*>(ws + L.off_v); }
    float* fourier() const { return reinterpret_cast<float*>(ws + L.off_fourier); }
    uint16_t* x0() const { return reinterpret_cast<uint16_t*>(ws + L.off_x0); }
    uint16_t* a(int l) const { return reinterpret_cast<uint16_t*>(ws + L.off_a) + (size_t)l * L.a_stride; }
    float* y() const { return reinterpret_cast<float*>(ws + L.off_y); }
    uint16_t* dy() const { return reinterpret_cast<uint16_t*>(ws + L.off_dy); }
    uint16_t* dz(int i) const { return reinterpret_cast<uint16_t*>(ws + (i ? L.off_dz1 : L.off_dz0)); }
    float* wpart() const { return reinterpret_cast<float*>(ws + L.off_wpart); }
    double* loss_part() const { return reinterpret_cast<double*>(ws + L.off_loss); }
};

namespace {

int blocks_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65536); }

// C (+ split offset) = opA x opB through the general MFMA product kernel.
int gemm(hipStream_t s, bool ta, bool tb, const uint16_t* A, const uint16_t* B, float* C, int M, int N, int K,
         int lda, int ldb, int ldc, int splits)
{
    if (M % smrt::mlp::TM || N % smrt::mlp::TN || K % (smrt::mlp::TK * splits))
        return fail(SMRT_EINVAL, "gemm shape %d x %d x %d (splits %d) not tile-aligned", M, N, K, splits);
    // operand slices are staged 8 elements (16 bytes) at a time
    if (lda % 8 || ldb % 8 || reinterpret_cast<uintptr_t>(A) % 16 || reinterpret_cast<uintptr_t>(B) % 16)
        return fail(SMRT_EINVAL, "gemm operands need 16-byte alignment and leading dimensions that are multiples of 8 "
                                 "(lda %d, ldb %d)", lda, ldb);
    dim3 grid(N / smrt::mlp::TN, M / smrt::mlp::TM, splits);
    const int ks = K / splits;
    const int64_t ss = (int64_t)M * ldc;
    using namespace smrt::mlp;
    constexpr int T = GEMM_THREADS;
    if (!ta && !tb) gemm_bf16<false, false><<<grid, T, 0, s>>>(A, B, C, M, N, lda, ldb, ldc, ks, ss);
    else if (ta && !tb) gemm_bf16<true, false><<<grid, T, 0, s>>>(A, B, C, M, N, lda, ldb, ldc, ks, ss);
    else if (!ta && tb) gemm_bf16<false, true><<<grid, T, 0, s>>>(A, B, C, M, N, lda, ldb, ldc, ks, ss);
    else gemm_bf16<true, true><<<grid, T, 0, s>>>(A, B, C, M, N, lda, ldb, ldc, ks, ss);
    return after_launch("gemm_bf16");
}

int check_batch(const smrt_mlp* m, int32_t n)
{
    if (n < 64 || n % 64 || n > m->L.max_batch)
        return fail(SMRT_EINVAL, "rows must be a multiple of 64 in 64..%d (got %d)", m->L.max_batch, n);
    if (!m->has_params) return fail(SMRT_ESTATE, "parameters not set (smrt_mlp_set_params)");
    return SMRT_OK;
}

// Output-column tile of the row-tile kernels: 128 where the width allows.
int column_tile(int n) { return n % 128 == 0 ? 128 : 64; }

// Whether the network's transposed weights fit the one-launch forward pass.
bool fused_fits(const MlpLayout& L)
{
    using namespace smrt::mlp;
    return (L.k0 == 64 || L.k0 == 128) && (L.width == 64 || L.width == 128) && L.layers <= kFusedMaxLayers &&
           fused_weight_elems(L.k0, L.width, L.layers) <= kFusedWeightElems;
}

int forward_fused_launch(smrt_mlp* m, int n, float* out, const float* target)
{
    using namespace smrt::mlp;
    const MlpLayout& L = m->L;
    FusedArgs a{};
    a.X0 = m->x0();
    a.layers = L.layers;
    for (int l = 0; l < L.layers; ++l) {
        a.wt[l] = m->wbf_t() + L.w_off[l];
        a.bias[l] = m->params() + L.b_off[l];
        if (l < L.layers - 1) a.act[l] = m->a(l);
    }
    a.blocks = n / 16;
    a.o.y = out;
    a.o.keep = L.outputs;
    const int waves = FUSED_THREADS / 64;
    const int groups = std::min(kFusedGroups, (a.blocks + waves - 1) / waves);
    if (target) {
        a.o.target = target;
        a.o.dy = m->dy();
        a.o.scale = 2.0f / ((float)n * L.outputs);
        a.o.loss = m->loss_part();
        m->loss_parts = groups;
        // the output layer's input gradient in the same launch
        a.w_last = m->wbf() + L.w_off[L.layers - 1];
        a.dz_last = m->dz(0);
    }
    const int mse = target != nullptr;
    hipStream_t s = m->stream;
#define SMRT_FUSED(K0, H)                                                                    \
    if (L.k0 == K0 && L.width == H) {                                                        \
        if (mse) forward_fused<K0, H, FWD_OUT_MSE><<<groups, FUSED_THREADS, 0, s>>>(a);        \
        else forward_fused<K0, H, FWD_OUT><<<groups, FUSED_THREADS, 0, s>>>(a);                \
        m->dz_ready = mse;                                                                   \
        return after_launch("forward_fused");                                                \
    }
    SMRT_FUSED(64, 128)
    SMRT_FUSED(64, 64)
    SMRT_FUSED(128, 128)
    SMRT_FUSED(128, 64)
#undef SMRT_FUSED
    return fail(SMRT_ESTATE, "no fused forward kernel for %d features, width %d", L.k0, L.width);
}

// Forward pass over n rows of points.  Hidden activations go to m->a(l); the
// output layer writes `out` ([n][outputs]) and, given a target, also the MSE
// gradient m->dy() and the squared-error partials m->loss_part().
int forward(smrt_mlp* m, const float* pts, int n, float* out, const float* target)
{
    using namespace smrt::mlp;
    const MlpLayout& L = m->L;
    hipStream_t s = m->stream;
    m->dz_ready = false;
    features<<<n / 64, 256, 0, s>>>(pts, m->fourier(), L.nf, n, L.k0, m->x0());
    int rc = after_launch("features");
    if (rc) return rc;
    if (m->fused && fused_fits(L)) return forward_fused_launch(m, n, out, target);
    const int tiles = n / RT;
    const int groups = std::min(tiles, kForwardGroups);
    for (int l = 0; l < L.layers; ++l) {
        const uint16_t* in = l == 0 ? m->x0() : m->a(l - 1);
        const int K = L.in[l], N = L.out[l];
        const uint16_t* wt = m->wbf_t() + L.w_off[l];
        const float* bias = m->params() + L.b_off[l];
        FwdOut o;
        if (l < L.layers - 1) {
            o.act = m->a(l);
            const int bn = column_tile(N);
            dim3 grid(groups, N / bn);
            if (bn == 128) layer_forward<128, FWD_HIDDEN><<<grid, ROW_THREADS, 0, s>>>(in, K, wt, bias, N, tiles, o);
            else layer_forward<64, FWD_HIDDEN><<<grid, ROW_THREADS, 0, s>>>(in, K, wt, bias, N, tiles, o);
        } else {
            // the output layer is one 64-column tile (N == n_last == 64)
            o.y = out;
            o.keep = L.outputs;
            dim3 grid(groups, 1);
            if (target) {
                o.target = target;
                o.dy = m->dy();
                o.scale = 2.0f / ((float)n * L.outputs);
                o.loss = m->loss_part();
                m->loss_parts = groups;
                layer_forward<64, FWD_OUT_MSE><<<grid, ROW_THREADS, 0, s>>>(in, K, wt, bias, N, tiles, o);
            } else {
                layer_forward<64, FWD_OUT><<<grid, ROW_THREADS, 0, s>>>(in, K, wt, bias, N, tiles, o);
            }
        }
        rc = after_launch("layer_forward");
        if (rc) return rc;
    }
    return SMRT_OK;
}

// Row blocks of the weight-gradient products: as many as keep at least
// kMinSplitRows rows (a multiple of 64) per block, at most L.max_splits.
int splits_for(const MlpLayout& L, int n)
{
    int s = L.max_splits;
    while (s > 1 && (n % (smrt::mlp::WG_ROWS * s) || n / s < kMinSplitRows)) s >>= 1;
    return s;
}

int launch_weight_grad(hipStream_t s, const smrt::mlp::GradArgs& a, int splits)
{
    using namespace smrt::mlp;
    const int bm = column_tile(a.M), bn = column_tile(a.N);
    dim3 grid(a.N / bn, a.M / bm, splits);
    if (bm == 128 && bn == 128) weight_grad<128, 128><<<grid, ROW_THREADS, 0, s>>>(a);
    else if (bm == 128) weight_grad<128, 64><<<grid, ROW_THREADS, 0, s>>>(a);
    else if (bn == 128) weight_grad<64, 128><<<grid, ROW_THREADS, 0, s>>>(a);
    else weight_grad<64, 64><<<grid, ROW_THREADS, 0, s>>>(a);
    return after_launch("weight_grad");
}

// Input gradient of layer l and its weight-gradient partials in one grid.
int launch_backward_and_grad(hipStream_t s, const smrt::mlp::BackArgs& ba, int groups,
                             const smrt::mlp::GradArgs& ga, int splits)
{
    using namespace smrt::mlp;
    const int bn = column_tile(ba.K), bn2 = column_tile(ga.N); // ga.M == ba.K
    const int gy_back = ba.K / bn, gx = ga.N / bn2, gy = ga.M / bn;
    const int64_t total = (int64_t)groups * gy_back + (int64_t)gx * gy * splits;
    if (total > std::numeric_limits<int>::max()) return fail(SMRT_EINVAL, "grid too large");
    const dim3 grid((unsigned)total);
    if (bn == 128 && bn2 == 128)
        backward_and_grad<128, 128, 128><<<grid, ROW_THREADS, 0, s>>>(ba, groups, gy_back, ga, gx, gy, splits);
    else if (bn == 128)
        backward_and_grad<128, 128, 64><<<grid, ROW_THREADS, 0, s>>>(ba, groups, gy_back, ga, gx, gy, splits);
    else if (bn2 == 128)
        backward_and_grad<64, 64, 128><<<grid, ROW_THREADS, 0, s>>>(ba, groups, gy_back, ga, gx, gy, splits);
    else
        backward_and_grad<64, 64, 64><<<grid, ROW_THREADS, 0, s>>>(ba, groups, gy_back, ga, gx, gy, splits);
    return after_launch("backward_and_grad");
}

// Backward pass after forward() with a target: the row-block partials of
// every layer's W and b gradient in m->wpart(), then one pass that sums them
// into m->grad() (adam null) or applies Adam; with loss != NULL also the mean
// squared error (synchronizes).
int backward(smrt_mlp* m, int n, const smrt::mlp::AdamArgs* adam, double* loss)
{
    using namespace smrt::mlp;
    const MlpLayout& L = m->L;
    hipStream_t s = m->stream;
    const int splits = splits_for(L, n);
    const int tiles = n / RT;
    const int groups = std::min(tiles, kBackwardGroups);
    const uint16_t* dcur = m->dy();
    int flip = 0;
    int rc = SMRT_OK;
    for (int l = L.layers - 1; l >= 0; --l) {
        const uint16_t* in = l == 0 ? m->x0() : m->a(l - 1);
        const int K = L.in[l], N = L.out[l];
        GradArgs ga;
        ga.X = in;
        ga.dZ = dcur;
        ga.M = K;
        ga.N = N;
        ga.rps = n / splits;
        ga.part = m->wpart() + (size_t)splits * L.w_off[l];
        ga.split_stride = (int64_t)K * N + N;
        if (l == 0) {
            rc = launch_weight_grad(s, ga, splits);
            if (rc) return rc;
            break;
        }
        if (l == L.layers - 1 && m->dz_ready) {
            // the fused forward pass already wrote dZ_{l-1} into dz(0)
            rc = launch_weight_grad(s, ga, splits);
            if (rc) return rc;
            dcur = m->dz(0);
            flip = 1;
            continue;
        }
        // dZ_{l-1} = (dZ_l W_l^T) silu'(Z_{l-1}), Z_{l-1} = A_{l-2} W_{l-1} + b_{l-1},
        // beside the row-block partials of layer l's W and b gradient
        BackArgs ba;
        ba.dZ = dcur;
        ba.N = N;
        ba.W = m->wbf() + L.w_off[l];
        ba.Xp = l == 1 ? m->x0() : m->a(l - 2);
        ba.Kp = L.in[l - 1];
        ba.Wpt = m->wbf_t() + L.w_off[l - 1];
        ba.bp = m->params() + L.b_off[l - 1];
        ba.K = K;
        ba.tiles = tiles;
        ba.dZout = m->dz(flip);
        flip ^= 1;
        rc = launch_backward_and_grad(s, ba, groups, ga, splits);
        if (rc) return rc;
        dcur = ba.dZout;
    }
    ReduceArgs r;
    r.part = m->wpart();
    r.S = splits;
    r.T = L.table;
    r.grad = m->grad();
    if (adam) r.a = *adam;
    r.i0 = 0;
    r.i1 = (int64_t)L.padded_params;
    reduce_adam<<<(int)((r.i1 + RED_PARAMS - 1) / RED_PARAMS), REDUCE_THREADS, 0, s>>>(r);
    rc = after_launch("reduce_adam");
    if (rc) return rc;
    if (loss) {
        m->loss_host.resize(m->loss_parts);
        HIP_TRY(hipMemcpyAsync(m->loss_host.data(), m->loss_part(), m->loss_parts * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double acc = 0.0;
        for (double v : m->loss_host) acc += v;
        *loss = acc / ((double)n * L.outputs);
    }
    return SMRT_OK;
}

// Real (dense) <-> padded parameter layout, one layer at a time.
int convert_params(smrt_mlp* m, const float* src, float* dst, int to_padded)
{
    const MlpLayout& L = m->L;
    size_t real = 0;
    for (int l = 0; l < L.layers; ++l) {
        const int rows = L.in_real[l], cols = L.out_real[l];
        const float* s_w = to_padded ? src + real : src + L.w_off[l];
        float* d_w = to_padded ? dst + L.w_off[l] : dst + real;
        smrt::mlp::pad_copy<<<blocks_for((int64_t)rows * cols), 256, 0, m->stream>>>(s_w, d_w, rows, cols, L.out[l],
                                                                                    to_padded);
        real += (size_t)rows * cols;
        const float* s_b = to_padded ? src + real : src + L.b_off[l];
        float* d_b = to_padded ? dst + L.b_off[l] : dst + real;
        smrt::mlp::pad_copy<<<blocks_for(cols), 256, 0, m->stream>>>(s_b, d_b, 1, cols, cols, to_padded);
        real += cols;
    }
    return after_launch("pad_copy");
}

} // namespace

extern "C" {

size_t smrt_mlp_param_count(const smrt_mlp_params* p)
{
    MlpLayout L;
    if (make_layout(p, &L) != SMRT_OK) return 0;
    return L.real_params;
}

size_t smrt_mlp_workspace_bytes(const smrt_mlp_params* p)
{
    MlpLayout L;
    if (make_layout(p, &L) != SMRT_OK) return 0;
    return L.total;
}

int smrt_mlp_create(const smrt_mlp_params* p, void* dev_ws, size_t ws_bytes, smrt_mlp** out)
{
    try {
        if (!out) return fail(SMRT_EINVAL, "out is NULL");
        *out = nullptr;
        MlpLayout L;
        int rc = make_layout(p, &L);
        if (rc) return rc;
        if (dev_ws && ws_bytes < L.total)
            return fail(SMRT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
        if (dev_ws && (reinterpret_cast<uintptr_t>(dev_ws) % kAlign))
            return fail(SMRT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
        smrt_mlp* m = new (std::nothrow) smrt_mlp;
        if (!m) return fail(SMRT_ENOMEM, "out of host memory");
        m->L = std::move(L);
        m->stream = static_cast<hipStream_t>(p->stream);
        if (dev_ws) {
            m->ws = static_cast<char*>(dev_ws);
        } else {
            hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->ws), m->L.total);
            if (e != hipSuccess) {
                const size_t total = m->L.total;
                smrt_mlp_destroy(m);
                return fail(SMRT_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
            }
            m->owns_ws = true;
        }
        *out = m;
        return SMRT_OK;
    } catch (...) {
        return fail(SMRT_ENOMEM, "unexpected host exception in smrt_mlp_create");
    }
}

int smrt_mlp_set_params(smrt_mlp* m, const float* params, const float* fourier)
{
    if (!m || !params) return fail(SMRT_EINVAL, "network or parameters is NULL");
    if (m->L.nf > 0 && !fourier) return fail(SMRT_EINVAL, "Fourier frequencies are required");
    const MlpLayout& L = m->L;
    const size_t pb = L.padded_params * sizeof(float);
    HIP_TRY(hipMemsetAsync(m->params(), 0, pb, m->stream));
    HIP_TRY(hipMemsetAsync(m->adam_m(), 0, pb, m->stream));
    HIP_TRY(hipMemsetAsync(m->adam_v(), 0, pb, m->stream));
    HIP_TRY(hipMemsetAsync(m->grad(), 0, pb, m->stream));
    if (L.nf > 0)
        HIP_TRY(hipMemcpyAsync(m->fourier(), fourier, (size_t)L.nf * 3 * sizeof(float), hipMemcpyDeviceToDevice,
                               m->stream));
    int rc = convert_params(m, params, m->params(), 1);
    if (rc) return rc;
    smrt::mlp::weights_to_bf16<<<blocks_for((int64_t)L.padded_params), 256, 0, m->stream>>>(
        m->params(), L.table, m->wbf(), m->wbf_t());
    rc = after_launch("weights_to_bf16");
    if (rc) return rc;
    m->adam_steps = 0;
    m->has_params = true;
    return SMRT_OK;
}

int smrt_mlp_get_params(smrt_mlp* m, float* params)
{
    if (!m || !params) return fail(SMRT_EINVAL, "network or output is NULL");
    if (!m->has_params) return fail(SMRT_ESTATE, "parameters not set");
    return convert_params(m, m->params(), params, 0);
}

int smrt_mlp_forward(smrt_mlp* m, const float* points, int32_t n, float* out)
{
    if (!m || !points || !out) return fail(SMRT_EINVAL, "network, points or output is NULL");
    int rc = check_batch(m, n);
    if (rc) return rc;
    return forward(m, points, n, out, nullptr);
}

int smrt_mlp_set_fused_forward(smrt_mlp* m, int32_t enable)
{
    if (!m) return fail(SMRT_EINVAL, "network is NULL");
    m->fused = enable != 0;
    return SMRT_OK;
}

int smrt_mlp_uses_fused_forward(const smrt_mlp* m)
{
    if (!m) return fail(SMRT_EINVAL, "network is NULL");
    return m->fused && fused_fits(m->L) ? 1 : 0;
}

int smrt_mlp_gradient(smrt_mlp* m, const float* points, const float* target, int32_t n, float* grad,
                      double* loss)
{
    if (!m || !points || !target || !grad) return fail(SMRT_EINVAL, "network, points, target or grad is NULL");
    int rc = check_batch(m, n);
    if (rc) return rc;
    rc = forward(m, points, n, m->y(), target);
    if (!rc) rc = backward(m, n, nullptr, loss);
    if (!rc) rc = convert_params(m, m->grad(), grad, 0);
    return rc;
}

int smrt_mlp_train_step(smrt_mlp* m, const float* points, const float* target, int32_t n, float lr, double* loss)
{
    if (!m || !points || !target) return fail(SMRT_EINVAL, "network, points or target is NULL");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(SMRT_EINVAL, "learning rate must be positive");
    int rc = check_batch(m, n);
    if (rc) return rc;
    m->adam_steps += 1;
    const double t = (double)m->adam_steps;
    smrt::mlp::AdamArgs a;
    a.w = m->params();
    a.m = m->adam_m();
    a.v = m->adam_v();
    a.lr_t = (float)(lr * std::sqrt(1.0 - std::pow(0.999, t)) / (1.0 - std::pow(0.9, t)));
    a.wbf = m->wbf();
    a.wbf_t = m->wbf_t();
    rc = forward(m, points, n, m->y(), target);
    if (!rc) rc = backward(m, n, &a, loss);
    return rc;
}

int smrt_gemm_bf16(const uint16_t* A, const uint16_t* B, float* C, int32_t M, int32_t N, int32_t K, int32_t lda,
                   int32_t ldb, int32_t ldc, int32_t trans_a, int32_t trans_b, int32_t splits, void* stream)
{
    if (!A || !B || !C) return fail(SMRT_EINVAL, "gemm operands must not be NULL");
    if (M <= 0 || N <= 0 || K <= 0 || splits < 1 || splits > 4096)
        return fail(SMRT_EINVAL, "gemm sizes must be positive (M %d N %d K %d splits %d)", M, N, K, splits);
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N) || ldc < N)
        return fail(SMRT_EINVAL, "gemm leading dimensions too small");
    return gemm(static_cast<hipStream_t>(stream), trans_a != 0, trans_b != 0, A, B, C, M, N, K, lda, ldb, ldc, splits);
}

void smrt_mlp_destroy(smrt_mlp* m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    if (m->owns_ws && m->ws) (void)hipFree(m->ws);
    delete m;
}

} // extern "C"
