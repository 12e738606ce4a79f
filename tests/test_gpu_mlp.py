"""The warm-start network's GPU kernels: the bf16 MFMA product against an FP64
product of the same bf16 values; the forward pass and every gradient entry
element by element against the bfloat16/binary32 model of the network in the
CPU oracle (oracle/mlp_oracle.py), each within its own tolerance; and training
that reduces the loss."""
import ctypes

import numpy as np
import pytest

from gpu_util import require_gpu, torch
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smrt():
    return require_gpu()


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def make_net(rng, fourier=16, width=128, layers=5, outputs=3):
    dims = M.layer_dims(fourier, width, layers, outputs)
    params = []
    for i, o in dims:
        params.append(rng.normal(0, np.sqrt(2.0 / i), size=(i, o)).ravel())
        params.append(rng.normal(0, 0.05, size=o))
    return dims, np.concatenate(params), rng.normal(0, 2.0, size=(fourier, 3))


def gradient_depth(n, max_splits=256):
    """Longest chain of binary32 additions in the library's sums over n rows
    (weight and bias gradients).  The library splits the rows into S blocks
    (S = max_splits, halved until S divides n into blocks of at least 256
    rows, a multiple of 64 each), accumulates each block on the matrix cores
    (n / S additions), then sums the S partials in one pass in sixteen
    consecutive groups (at most S / 16 + 1 additions, then 15 to join the
    groups)."""
    sp = max_splits
    while sp > 1 and (n % (64 * sp) or n // sp < 256):
        sp //= 2
    return n // sp + sp // 16 + 16


def test_forward_matches_oracle(smrt):
    """Every output element within its tolerance of the bfloat16/binary32
    model of the network (oracle/mlp_oracle.py forward_tolerance)."""
    rng = np.random.default_rng(1)
    dims, params, B = make_net(rng)
    params, B = params.astype(np.float32), B.astype(np.float32)
    pts = rng.uniform(0, 1, size=(512, 3)).astype(np.float32)
    with smrt.MLP(max_batch=1024) as net:
        net.set_params(torch.tensor(params, device="cuda:0"), torch.tensor(B, device="cuda:0"))
        assert np.array_equal(net.get_params().cpu().numpy(), params)
        y = net.forward(torch.tensor(pts, device="cuda:0")).cpu().numpy().astype(np.float64)
    want, tol = M.forward_tolerance(params, B, pts, dims)
    used = np.abs(y - want) / tol
    plain, _ = M.forward(params, B, pts, dims)
    print("forward: largest fraction of the tolerance used %.3f; median |dy|/|y| %.2e "
          "(FP64 network: %.2e)" % (used.max(), np.median(np.abs(y - want) / np.abs(want)),
                                    np.median(np.abs(y - plain) / np.abs(plain))))
    assert np.all(used <= 1.0), np.argwhere(used > 1.0)[:10]


@pytest.mark.parametrize("n", [1024, 8192, 65536])   # 4, 32 and 256 row blocks of the weight gradients
def test_gradient_matches_oracle(smrt, n):
    """All 54,531 gradient entries and the loss within their tolerances of the
    bfloat16/binary32 model (oracle/mlp_oracle.py gradient_tolerance)."""
    rng = np.random.default_rng(2)
    dims, params, B = make_net(rng)
    params, B = params.astype(np.float32), B.astype(np.float32)
    pts = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    tgt = rng.normal(0, 0.5, size=(n, 3)).astype(np.float32)
    with smrt.MLP(max_batch=n) as net:
        net.set_params(torch.tensor(params, device="cuda:0"), torch.tensor(B, device="cuda:0"))
        loss, g = net.gradient(torch.tensor(pts, device="cuda:0"), torch.tensor(tgt, device="cuda:0"))
        g = g.cpu().numpy().astype(np.float64)
    want_loss, loss_tol, want, tol = M.gradient_tolerance(params, B, pts, tgt, dims, gradient_depth(n))
    assert g.shape == want.shape == (54531,)
    used = np.abs(g - want) / tol
    scale = np.abs(want) + 1e-3 * np.abs(want).max()
    print("gradient: largest fraction of the tolerance used %.3f, median tolerance / |g| %.2e; "
          "loss %.8f vs %.8f (tolerance %.1e)" % (used.max(), np.median(tol / scale), loss, want_loss, loss_tol))
    assert np.all(used <= 1.0), np.argwhere(used > 1.0)[:10]
    # the loss is summed in FP64 from binary32 errors in a block order
    assert abs(loss - want_loss) <= loss_tol + 1e-12 * want_loss


@pytest.mark.parametrize("fourier,width,layers,outputs,n", [
    (4, 64, 3, 2, 512),      # 64-column tiles everywhere
    (40, 256, 3, 3, 1024),   # 83 features padded to 128, two 128-column chunks, weights restaged per tile
    (8, 192, 2, 1, 320),     # three 64-column tiles; one hidden layer; 320 rows: 5 row tiles, 1 block
])
def test_gradient_other_shapes(smrt, fourier, width, layers, outputs, n):
    """Forward pass and every gradient entry within tolerance for networks
    whose sizes take the other tile shapes and contraction chunkings."""
    rng = np.random.default_rng(fourier + width + layers)
    dims, params, B = make_net(rng, fourier=fourier, width=width, layers=layers, outputs=outputs)
    params, B = params.astype(np.float32), B.astype(np.float32)
    pts = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    tgt = rng.normal(0, 0.5, size=(n, outputs)).astype(np.float32)
    with smrt.MLP(fourier=fourier, width=width, layers=layers, outputs=outputs, max_batch=n) as net:
        net.set_params(torch.tensor(params, device="cuda:0"), torch.tensor(B, device="cuda:0"))
        y = net.forward(torch.tensor(pts, device="cuda:0")).cpu().numpy().astype(np.float64)
        loss, g = net.gradient(torch.tensor(pts, device="cuda:0"), torch.tensor(tgt, device="cuda:0"))
        g = g.cpu().numpy().astype(np.float64)
    want_y, tol_y = M.forward_tolerance(params, B, pts, dims)
    assert np.all(np.abs(y - want_y) <= tol_y)
    want_loss, loss_tol, want, tol = M.gradient_tolerance(params, B, pts, tgt, dims, gradient_depth(n))
    assert g.shape == want.shape
    used = np.abs(g - want) / tol
    print("%s: largest fraction of the tolerance used %.3f (forward %.3f)"
          % (dims, used.max(), (np.abs(y - want_y) / tol_y).max()))
    assert np.all(used <= 1.0), np.argwhere(used > 1.0)[:10]
    assert abs(loss - want_loss) <= loss_tol + 1e-12 * want_loss


@pytest.mark.parametrize("fourier,width,layers,outputs,n", [
    (16, 128, 5, 3, 65536),  # the warm-start network: 35 features padded to 64, LDS full
    (16, 128, 5, 3, 320),    # 20 blocks of 16 rows: 5 workgroups, one block a wave
    (30, 128, 5, 3, 1024),   # 63 features, the widest first layer that still fits
    (4, 64, 3, 2, 512),      # width 64
    (40, 64, 3, 3, 1024),    # 83 features padded to 128, width 64
    (40, 128, 4, 1, 2048),   # 128 features, width 128, four layers
    (8, 128, 2, 1, 320),     # one hidden layer
    (8, 64, 2, 2, 192),      # one hidden layer of width 64; 12 row blocks, fewer than a workgroup's waves
])
def test_fused_forward_bitwise_equals_per_layer(smrt, fourier, width, layers, outputs, n):
    """The one-launch forward pass against one launch per layer: outputs and
    every gradient entry bitwise equal (same operands, same MFMA order), the
    loss equal up to the order of its FP64 block sums."""
    rng = np.random.default_rng(fourier * 7 + width + layers + n)
    dims, params, B = make_net(rng, fourier=fourier, width=width, layers=layers, outputs=outputs)
    params, B = params.astype(np.float32), B.astype(np.float32)
    pts = torch.tensor(rng.uniform(0, 1, size=(n, 3)).astype(np.float32), device="cuda:0")
    tgt = torch.tensor(rng.normal(0, 0.5, size=(n, outputs)).astype(np.float32), device="cuda:0")
    res = {}
    with smrt.MLP(fourier=fourier, width=width, layers=layers, outputs=outputs, max_batch=n) as net:
        net.set_params(torch.tensor(params, device="cuda:0"), torch.tensor(B, device="cuda:0"))
        assert net.fused_forward
        for fused in (True, False):
            net.fused_forward = fused
            assert net.fused_forward == fused
            y = net.forward(pts).clone()
            loss, g = net.gradient(pts, tgt)
            res[fused] = (y, loss, g.clone())
    print("n %d: loss fused %.17g, per layer %.17g" % (n, res[True][1], res[False][1]))
    assert torch.equal(res[True][0], res[False][0])
    assert torch.equal(res[True][2], res[False][2])
    assert abs(res[True][1] - res[False][1]) <= 1e-12 * abs(res[False][1])


def test_fused_forward_only_where_it_fits(smrt):
    """Width 192 or 256, or a 128-feature input with four 128-wide hidden
    layers, exceed the LDS-resident form: those networks run layer by layer."""
    for fourier, width, layers in [(8, 192, 2), (40, 256, 3), (40, 128, 5)]:
        with smrt.MLP(fourier=fourier, width=width, layers=layers, outputs=3, max_batch=256) as net:
            assert not net.fused_forward


def to_bf16_bits(a):
    """float array of bf16-exact values -> int16 tensor of their bit patterns."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32)
    assert np.all((u & 0xFFFF) == 0), "values must be exact in bfloat16"
    return torch.tensor((u >> 16).astype(np.uint16).view(np.int16), device="cuda:0")


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("m,n,k,splits", [(64, 64, 32, 1), (128, 192, 96, 1), (192, 128, 512, 4),
                                          (64, 64, 2048, 64)])
def test_gemm_bf16_exact(smrt, ta, tb, m, n, k, splits):
    """Integer-valued bf16 operands: every FP32 partial sum is exact, so the
    matrix-core product must equal the FP64 product bit for bit (all four
    transposition cases, split-K, ragged leading dimensions)."""
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.integers(-8, 9, size=(m, k)).astype(np.float64)
    Bm = rng.integers(-8, 9, size=(k, n)).astype(np.float64)
    lda = (m if ta else k) + 16
    ldb = (k if tb else n) + 32
    a_store = np.zeros(((k if ta else m), lda))
    b_store = np.zeros(((n if tb else k), ldb))
    if ta:
        a_store[:, :m] = A.T
    else:
        a_store[:, :k] = A
    if tb:
        b_store[:, :k] = Bm.T
    else:
        b_store[:, :n] = Bm
    C = smrt.gemm_bf16(to_bf16_bits(a_store), to_bf16_bits(b_store), m, n, k, lda, ldb, n + 64,
                       trans_a=ta, trans_b=tb, splits=splits).cpu().numpy()
    ks = k // splits
    for sidx in range(splits):
        want = A[:, sidx * ks:(sidx + 1) * ks] @ Bm[sidx * ks:(sidx + 1) * ks, :]
        assert np.array_equal(C[sidx][:, :n], want)


def test_gemm_bf16_rejects_unaligned(smrt):
    z = torch.zeros(64 * 64, dtype=torch.int16, device="cuda:0")
    with pytest.raises(smrt.SmrtError):
        smrt.gemm_bf16(z, z, 64, 64, 48, 64, 64, 64)      # K not a multiple of 32
    with pytest.raises(smrt.SmrtError):
        smrt.gemm_bf16(z, z, 32, 64, 32, 64, 64, 64)      # M not a multiple of 64
    with pytest.raises(smrt.SmrtError):
        smrt.gemm_bf16(z, z, 64, 64, 32, 68, 64, 64)      # lda not a multiple of 8


def test_training_reduces_loss(smrt):
    rng = np.random.default_rng(5)
    dims, params, B = make_net(rng)
    n = 4096
    pts = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    x, y, s = pts[:, 0], pts[:, 1], pts[:, 2]
    tgt = np.stack([np.sin(np.pi * x) * np.sin(np.pi * y) * (1 + s), np.cos(2 * x) * y, x * y - s],
                   axis=1).astype(np.float32)
    P, T = torch.tensor(pts, device="cuda:0"), torch.tensor(tgt, device="cuda:0")
    with smrt.MLP(max_batch=n) as net:
        net.set_params(torch.tensor(params * 0.5, dtype=torch.float32, device="cuda:0"),
                       torch.tensor(B * 0.5, dtype=torch.float32, device="cuda:0"))
        first = net.train_step(P, T, 2e-3, want_loss=True)
        for _ in range(400):
            net.train_step(P, T, 2e-3)
        last = net.train_step(P, T, 2e-3, want_loss=True)
    print("training loss %.4e -> %.4e" % (first, last))
    assert last < first / 20


def test_mlp_rejects_bad_shapes(smrt):
    with smrt.MLP(max_batch=256) as net:
        with pytest.raises(smrt.SmrtError):
            net.forward(torch.zeros((64, 3), device="cuda:0"))      # parameters not set
        net.set_params(torch.zeros(net.param_count, device="cuda:0"),
                       torch.zeros((16, 3), device="cuda:0"))
        with pytest.raises(smrt.SmrtError):
            net.forward(torch.zeros((100, 3), device="cuda:0"))     # not a multiple of 64
        with pytest.raises(smrt.SmrtError):
            net.forward(torch.zeros((512, 3), device="cuda:0"))     # above max_batch
