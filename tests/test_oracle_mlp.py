"""Pins of the FP64 network reference (oracle/mlp_oracle.py).

* Hand-worked values: a 2-layer and a 3-layer network on points where every
  pre-activation is 1, -2 or 0, so the outputs and gradients are closed forms
  in e (silu(1) = e/(1+e), silu(-2) = -2/(1+e^2), silu'(z) = s(z)(1 + z(1 - s(z))),
  s the logistic function).  A tanh or ReLU activation, an activation on the
  output layer, a dropped bias or swapped hidden layers all change them.
* The gradient against central finite differences of the loss.
* The features on hand-computable points.
* The bfloat16/binary32 model: its rounding against an independent bit-level
  round-to-nearest-even, and its element bounds against a binary32 emulation
  of the network (numpy float32, a different summation order): every element
  inside its bound, the bounds small, and planted indexing mistakes outside.
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

E = math.e
SILU1 = 0.7310585786300049        # e / (1 + e)
SILU_M2 = -0.23840584404423515    # -2 / (1 + e^2)
DSILU1 = 0.9276705118714869       # s(1) (1 + (1 - s(1))),  s(1) = e / (1 + e)
DSILU_M2 = -0.0907842487848955    # s(-2) (1 - 2 (1 - s(-2))),  s(-2) = 1 / (1 + e^2)


def test_closed_forms_of_the_constants():
    # the literals above are the closed forms (typed as decimals)
    assert SILU1 == pytest.approx(E / (1 + E), abs=1e-16)
    assert SILU_M2 == pytest.approx(-2 / (1 + E * E), abs=1e-16)
    assert DSILU1 == pytest.approx(E / (1 + E) * (2 - E / (1 + E)), abs=1e-16)
    assert DSILU_M2 == pytest.approx(1 / (1 + E * E) * (1 - 2 * (E * E / (1 + E * E))), abs=1e-16)


def two_layer():
    # features (x, y, s) with no Fourier terms; hidden width 2, one output
    dims = M.layer_dims(0, 2, 2, 1)
    W0 = np.array([[1.0, -2.0], [0.0, 0.0], [0.0, 0.0]])
    b0 = np.array([0.0, 0.0])
    W1 = np.array([[1.0], [1.0]])
    b1 = np.array([0.25])
    params = np.concatenate([W0.ravel(), b0, W1.ravel(), b1])
    return dims, params


def test_two_layer_forward_by_hand():
    dims, params = two_layer()
    y, _ = M.forward(params, np.zeros((0, 3)), np.array([[1.0, 0.0, 0.0]]), dims)
    # z = (1, -2), y = silu(1) + silu(-2) + 0.25
    assert y[0, 0] == pytest.approx(SILU1 + SILU_M2 + 0.25, abs=1e-15)


def test_two_layer_gradient_by_hand():
    dims, params = two_layer()
    pts, tgt = np.array([[1.0, 0.0, 0.0]]), np.array([[0.0]])
    loss, g = M.loss_and_grad(params, np.zeros((0, 3)), pts, tgt, dims)
    y = SILU1 + SILU_M2 + 0.25
    assert loss == pytest.approx(y * y, abs=1e-15)
    r = 2 * y                       # d loss / d y (one output, one row)
    # layout: W0 (3 x 2) row-major, b0 (2), W1 (2 x 1), b1 (1)
    want = np.zeros(11)
    want[0], want[1] = r * DSILU1, r * DSILU_M2   # d/dW0[0, j] = r W1[j] silu'(z_j) x
    want[6], want[7] = r * DSILU1, r * DSILU_M2   # d/db0[j]
    want[8], want[9] = r * SILU1, r * SILU_M2     # d/dW1[j] = r silu(z_j)
    want[10] = r                                  # d/db1
    assert np.allclose(g, want, atol=1e-15, rtol=0)


def test_three_layer_forward_by_hand():
    # two hidden layers of width 3: swapping them changes the output
    dims = M.layer_dims(0, 3, 3, 1)
    W0 = np.array([[1.0, -2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    W1 = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    W2 = np.array([[1.0], [0.0], [0.0]])
    z3 = np.zeros(3)
    params = np.concatenate([W0.ravel(), z3, W1.ravel(), z3, W2.ravel(), [0.0]])
    y, _ = M.forward(params, np.zeros((0, 3)), np.array([[1.0, 0.0, 0.0]]), dims)
    c = SILU1 + SILU_M2            # second pre-activation, z = (c, 0, 0)
    assert y[0, 0] == pytest.approx(c / (1 + math.exp(-c)), abs=1e-15)
    swapped = np.concatenate([W1.ravel(), z3, W0.ravel(), z3, W2.ravel(), [0.0]])
    ys, _ = M.forward(swapped, np.zeros((0, 3)), np.array([[1.0, 0.0, 0.0]]), dims)
    assert abs(ys[0, 0] - y[0, 0]) > 0.1


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    fourier, width, layers, outputs = 4, 8, 3, 3
    dims = M.layer_dims(fourier, width, layers, outputs)
    n = M.param_count(fourier, width, layers, outputs)
    params = rng.normal(0, 0.5, size=n)
    B = rng.normal(0, 1.0, size=(fourier, 3))
    pts = rng.uniform(0, 1, size=(7, 3))
    tgt = rng.normal(0, 1, size=(7, outputs))
    loss, g = M.loss_and_grad(params, B, pts, tgt, dims)
    h = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd[i] = (M.loss_and_grad(params + e, B, pts, tgt, dims)[0] -
                 M.loss_and_grad(params - e, B, pts, tgt, dims)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8 * max(1.0, np.abs(g).max())
    assert loss > 0


def test_features_definition():
    B = np.array([[1.0, 0.0, 0.0], [0.0, 0.5, 0.0]])
    p = np.array([[0.25, 0.5, 0.0]])
    f = M.features(p, B)
    assert np.allclose(f, [[0.25, 0.5, 0.0, 1.0, np.sin(np.pi / 2), 0.0, np.cos(np.pi / 2)]], atol=1e-15)


def test_zero_network_outputs_bias():
    dims = M.layer_dims(2, 4, 3, 3)
    n = M.param_count(2, 4, 3, 3)
    params = np.zeros(n)
    params[-3:] = [1.0, -2.0, 0.5]
    y, _ = M.forward(params, np.ones((2, 3)), np.ones((5, 3)), dims)
    assert np.array_equal(y, np.tile([1.0, -2.0, 0.5], (5, 1)))


# --- the bfloat16 / binary32 model ------------------------------------------

def bf16_bits_rne(a32):
    """Round-to-nearest-even binary32 -> bfloat16 on the bit patterns
    (integer arithmetic), returned as float64."""
    u = np.ascontiguousarray(a32, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_round_matches_bit_level_rounding():
    rng = np.random.default_rng(11)
    v = np.concatenate([rng.normal(0, 1, 100000) * 10.0 ** rng.integers(-6, 6, 100000),
                        [0.0, 1.0, -1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 255.5, 2 ** -100]])
    v32 = v.astype(np.float32)
    assert np.array_equal(M.bf16_round(v32.astype(np.float64)), bf16_bits_rne(v32))


def emulate_f32(params, B, pts, tgt, dims):
    """The network in binary32 (numpy float32, its own summation order) with
    bfloat16 rounding at the library's points: outputs, loss and gradient."""
    f32 = np.float32
    bf = lambda a: bf16_bits_rne(np.asarray(a, f32)).astype(f32)
    layers = M.unpack(np.asarray(params, np.float64), dims)
    p = np.asarray(pts, f32)
    arg = f32(2 * np.pi) * (p @ np.asarray(B, f32).T)
    x = bf(np.concatenate([p, np.sin(arg), np.cos(arg)], axis=1))
    acts, zs = [x], []
    for li, (W, b) in enumerate(layers):
        z = x @ bf(W) + np.asarray(b, f32)
        zs.append(z)
        if li < len(layers) - 1:
            x = bf(z * (f32(1) / (f32(1) + np.exp(-z))))
            acts.append(x)
    y = z
    t = np.asarray(tgt, f32)
    e = y - t
    loss = float((e.astype(np.float64) ** 2).sum() / y.size)
    dz = bf((f32(2.0) / f32(y.size)) * e)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        grads[li] = (acts[li].T @ dz, dz.sum(axis=0, dtype=f32))
        if li == 0:
            break
        dA = dz @ bf(layers[li][0]).T
        zz = zs[li - 1]
        sg = f32(1) / (f32(1) + np.exp(-zz))
        dz = bf(dA * (sg * (f32(1) + zz * (f32(1) - sg))))
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads]).astype(np.float64)
    return y.astype(np.float64), loss, flat


def random_net(rng, fourier=16, width=128, layers=5, outputs=3):
    dims = M.layer_dims(fourier, width, layers, outputs)
    params = []
    for i, o in dims:
        params.append(rng.normal(0, np.sqrt(2.0 / i), size=(i, o)).ravel())
        params.append(rng.normal(0, 0.05, size=o))
    p = np.concatenate(params).astype(np.float32).astype(np.float64)
    B = rng.normal(0, 2.0, size=(fourier, 3)).astype(np.float32).astype(np.float64)
    return dims, p, B


@pytest.fixture(scope="module")
def bounded_case():
    rng = np.random.default_rng(2)
    dims, params, B = random_net(rng)
    n = 1024
    pts = rng.uniform(0, 1, size=(n, 3)).astype(np.float32).astype(np.float64)
    tgt = rng.normal(0, 0.5, size=(n, 3)).astype(np.float32).astype(np.float64)
    y, ey = M.forward_tolerance(params, B, pts, dims)
    loss, eloss, g, eg = M.gradient_tolerance(params, B, pts, tgt, dims, depth=n)
    ye, loss_e, ge = emulate_f32(params, B, pts, tgt, dims)
    return dict(dims=dims, y=y, ey=ey, loss=loss, eloss=eloss, g=g, eg=eg, ye=ye, loss_e=loss_e, ge=ge,
                plain=M.loss_and_grad(params, B, pts, tgt, dims), plain_args=(params, B, pts, dims))


def test_tolerances_hold_for_a_binary32_evaluation(bounded_case):
    """Every element of the emulation within its tolerance, with room to
    spare (the library's evaluation differs from the emulation's in order and
    in its own rounding flips)."""
    c = bounded_case
    fwd = np.abs(c["ye"] - c["y"]) / c["ey"]
    grad = np.abs(c["ge"] - c["g"]) / c["eg"]
    print("largest fraction of the tolerance used: outputs %.3f, gradients %.3f" % (fwd.max(), grad.max()))
    assert fwd.max() < 0.5 and grad.max() < 0.5
    assert abs(c["loss_e"] - c["loss"]) <= c["eloss"]


def test_model_is_the_right_reference(bounded_case):
    """The bfloat16 model sits far closer to a binary32 evaluation than the
    plain FP64 network does (most rows see no rounding flip at all), and its
    tolerances stay well below the size of the values."""
    c = bounded_case
    loss_plain, g_plain = c["plain"]
    y_plain = M.forward(*c["plain_args"])[0]
    med_model = np.median(np.abs(c["ye"] - c["y"]) / np.abs(c["y"]))
    med_plain = np.median(np.abs(c["ye"] - y_plain) / np.abs(y_plain))
    print("median relative distance of the emulation: bf16 model %.2e, FP64 network %.2e"
          % (med_model, med_plain))
    assert med_model < 1e-3 * med_plain
    scale = np.abs(c["g"]) + 1e-3 * np.abs(c["g"]).max()
    rel_y = np.median(c["ey"] / np.abs(c["y"]))
    rel_g = np.median(c["eg"] / scale)
    print("median relative tolerance: outputs %.2e, gradients %.2e" % (rel_y, rel_g))
    assert rel_y < 0.3 and rel_g < 0.1
    assert abs(c["loss"] / loss_plain - 1) < 1e-2


def test_planted_gradient_mistakes_exceed_the_bounds(bounded_case):
    c = bounded_case
    dims = c["dims"]
    g = c["ge"]
    off, layer_offsets = 0, []
    for i, o in dims:
        layer_offsets.append((off, i, o))
        off += i * o + o
    # a bias gradient written to the neighbouring column
    w0, i0, o0 = layer_offsets[2]
    bad = g.copy()
    b = w0 + i0 * o0
    bad[b:b + o0] = np.roll(bad[b:b + o0], 1)
    assert np.any(np.abs(bad - c["g"]) > c["eg"])
    # one weight-gradient row taken from the next input feature
    bad = g.copy()
    bad[w0:w0 + o0] = g[w0 + o0:w0 + 2 * o0]
    assert np.any(np.abs(bad - c["g"]) > c["eg"])
    # a forward output from the wrong row
    yb = c["ye"].copy()
    yb[[0, 1]] = yb[[1, 0]]
    assert np.any(np.abs(yb - c["y"]) > c["ey"])
