"""FP64 numpy reference of the warm-start coordinate network.

TEST INFRASTRUCTURE ONLY: checks the GPU network's forward pass and
gradients.  Plain, unblocked numpy; no code shared with the GPU path.

Network (the same definition the GPU library implements): features
[x, y, s, sin(2 pi B p), cos(2 pi B p)] of a point p = (x, y, s), then SiLU
layers z -> z sigmoid(z), then a linear output; loss = mean squared error
over all outputs.  Parameters are one flat vector: for each layer W_l
([in][out], row-major) then b_l.

forward / loss_and_grad are the plain FP64 definition, pinned by hand-worked
closed forms (silu(1) = e/(1+e), silu(-2) = -2/(1+e^2) and their
derivatives), central finite differences and hand-computed features
(tests/test_oracle_mlp.py).  forward_tolerance / gradient_tolerance evaluate
the same network with the library's bfloat16 roundings and give every
element a tolerance for a binary32 evaluation (see the section below); they
are pinned against a numpy binary32 emulation and by planted indexing
mistakes that must fall outside the tolerances.
"""
import numpy as np


def layer_dims(fourier, width, layers, outputs):
    dims = [3 + 2 * fourier] + [width] * (layers - 1) + [outputs]
    return list(zip(dims[:-1], dims[1:]))


def param_count(fourier, width, layers, outputs):
    return sum(i * o + o for i, o in layer_dims(fourier, width, layers, outputs))


def unpack(params, dims):
    out, k = [], 0
    for i, o in dims:
        W = params[k:k + i * o].reshape(i, o)
        k += i * o
        b = params[k:k + o]
        k += o
        out.append((W, b))
    return out


def features(points, B):
    arg = 2.0 * np.pi * points @ B.T
    return np.concatenate([points, np.sin(arg), np.cos(arg)], axis=1)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, B, points, dims):
    """Returns (outputs, cache)."""
    layers = unpack(np.asarray(params, np.float64), dims)
    a = features(np.asarray(points, np.float64), np.asarray(B, np.float64))
    cache = [a]
    for li, (W, b) in enumerate(layers):
        z = a @ W + b
        if li < len(layers) - 1:
            cache.append(z)
            a = z * sigmoid(z)
            cache.append(a)
        else:
            a = z
    return a, cache


def loss_and_grad(params, B, points, target, dims):
    """Mean squared error and its gradient (flat, same layout as params)."""
    params = np.asarray(params, np.float64)
    layers = unpack(params, dims)
    y, cache = forward(params, B, points, dims)
    t = np.asarray(target, np.float64)
    n_el = y.size
    loss = float(((y - t) ** 2).sum() / n_el)
    dz = 2.0 * (y - t) / n_el
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        a_in = cache[0] if li == 0 else cache[2 * li]
        W, _ = layers[li]
        grads[li] = (a_in.T @ dz, dz.sum(axis=0))
        if li == 0:
            break
        da = dz @ W.T
        z = cache[2 * li - 1]
        sg = sigmoid(z)
        dz = da * sg * (1.0 + z * (1.0 - sg))
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


# ---------------------------------------------------------------------------
# The network as the GPU library evaluates it, with a tolerance on every
# element.
#
# The library's precision contract: bfloat16 operands on the matrix cores
# (input features, weights, hidden activations, the output gradient and the
# hidden-layer gradients are rounded to bfloat16, nearest-even), products
# accumulated in binary32, pre-activations, biases, outputs and gradients held
# in binary32.  The functions below evaluate the network in float64 with the
# bfloat16 roundings at those points and carry, for every value, how far the
# library's binary32 evaluation can lie from it, in two parts:
#   L  binary32 arithmetic, bounded in the worst case: a binary32 sum of m
#      exact products (a bfloat16 x bfloat16 product is exact in binary32)
#      differs from the exact sum by at most 2 m u sum|terms|, u = 2^-24 (at
#      most one ulp per addition, any order; m is the longest chain of
#      additions a term passes through); sin/cos, exp, the reciprocal and
#      each multiply or add are charged a few ulp of their result (generous
#      multiples below); errors pass through the activation with its
#      derivative bounds (|silu'| <= 1.1, |silu''| <= 0.5);
#   S  bfloat16 rounding flips, as a standard deviation.  Rounding is
#      monotone and absorbs small differences: a binary32 value that differs
#      from the model's v by less than v's distance to the nearest rounding
#      boundary rounds to the same bfloat16 value.  Where the difference can
#      reach the boundary (L + 7 S, a Gaussian tail below 1e-12, against the
#      distance) the rounded values may differ by one spacing; with p the
#      probability of crossing, that flip is charged an rms of
#      spacing * max(sqrt(p), 1/6), so that a single flip always lies inside
#      the 6-sigma tolerance below.  Flips of different values have
#      independent signs and combine in quadrature: a worst-case (linear) sum
#      over five layers of 128 would carry every possible flip into every
#      later value and bound nothing.
# The tolerance of a value is L + KAPPA S with KAPPA = 6.
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24
KAPPA = 6.0
TAIL = 7.0
FLIP_FLOOR = 1.0 / 6.0


def bf16_round(v):
    """Nearest bfloat16 (8 significant bits, ties to even) of float64 values,
    as float64 (exact: scaling by a power of two)."""
    v = np.asarray(v, np.float64)
    _, ex = np.frexp(v)
    scale = np.ldexp(1.0, ex - 8)
    return np.round(v / scale) * scale


def _tail(x):
    """P(N(0, 1) > x)."""
    from scipy.special import erfc
    return 0.5 * erfc(x / np.sqrt(2.0))


def round_tracked(v, L, S):
    """bfloat16 rounding of a tracked value (v, L, S): returns (bf16(v), 0, S')
    with S' the rms of the flip it may cause (0 where no flip is possible)."""
    v = np.asarray(v, np.float64)
    L = np.broadcast_to(L, v.shape)
    S = np.broadcast_to(S, v.shape)
    r = bf16_round(v)
    a, ar = np.abs(v), np.abs(r)
    m, ex = np.frexp(ar)
    up = np.ldexp(1.0, ex - 8)                             # spacing above |r|
    down = np.where(m == 0.5, up / 2, up)                  # spacing below |r|
    up = np.where(ar == 0, 2.0 ** -133, up)
    down = np.where(ar == 0, 2.0 ** -133, down)
    d_up = ar + up / 2 - a                                 # distance to the boundary above
    d_dn = a - (ar - down / 2)                             # and below
    e = L + TAIL * S
    possible = (d_up <= e) | (d_dn <= e)
    with np.errstate(divide="ignore", invalid="ignore"):
        z_up = np.where(S > 0, (d_up - L) / S, np.where(d_up <= L, -np.inf, np.inf))
        z_dn = np.where(S > 0, (d_dn - L) / S, np.where(d_dn <= L, -np.inf, np.inf))
    p = np.minimum(1.0, _tail(z_up) + _tail(z_dn))
    flip = np.maximum(up, down) * np.maximum(np.sqrt(p), FLIP_FLOOR)
    # below one spacing the rounding absorbs the difference unless it
    # crosses (the flip); above, the difference itself passes through
    pre = S + L
    S_post = np.where(possible, np.where(pre < np.maximum(up, down), flip, np.sqrt(pre ** 2 + flip ** 2)), 0.0)
    return r, np.zeros_like(r), S_post


def features_tracked(points, B):
    """bfloat16 input features.  The raw coordinates are binary32 inputs
    rounded once (no error); the angle 2 pi B p is formed in binary32 (a few
    roundings of the dot product and of 2 pi), then sin/cos."""
    p = np.asarray(points, np.float64)
    Bm = np.asarray(B, np.float64)
    arg = 2.0 * np.pi * (p @ Bm.T)
    e_trig = 2.0 * np.pi * 4 * U32 * (np.abs(p) @ np.abs(Bm).T) + 4 * U32 * np.abs(arg) + 8 * U32
    xs, _, ss = round_tracked(np.sin(arg), e_trig, 0.0)
    xc, _, sc = round_tracked(np.cos(arg), e_trig, 0.0)
    x = np.concatenate([bf16_round(p), xs, xc], axis=1)
    s = np.concatenate([np.zeros_like(p), ss, sc], axis=1)
    return x, np.zeros_like(x), s


def _dense_tracked(x, Lx, Sx, W, b):
    """z = x bf16(W) + b, binary32 accumulation of K products and the bias."""
    Wb = bf16_round(W)
    aW = np.abs(Wb)
    z = x @ Wb + b
    prop = Lx @ aW
    terms = np.abs(x) @ aW + prop + KAPPA * (Sx @ aW) + np.abs(b)
    L = prop + 2 * U32 * (W.shape[0] + 1) * terms
    S = np.sqrt((Sx * Sx) @ (Wb * Wb))
    return z, L, S


def forward_tracked(params, B, points, dims):
    """(y, L_y, S_y, cache) of the bfloat16/binary32 network; cache holds each
    layer's input and pre-activation with their L and S."""
    layers = unpack(np.asarray(params, np.float64), dims)
    x, Lx, Sx = features_tracked(points, B)
    cache = []
    for li, (W, b) in enumerate(layers):
        z, Lz, Sz = _dense_tracked(x, Lx, Sx, W, b)
        cache.append((x, Lx, Sx, z, Lz, Sz))
        if li < len(layers) - 1:
            a = z * sigmoid(z)
            # exp, 1 + exp, the reciprocal and z * sigmoid in binary32
            La = 1.1 * Lz + np.abs(a) * (2.0 * np.abs(z) + 20.0) * U32
            x, Lx, Sx = round_tracked(a, La, 1.1 * Sz)
    return z, Lz, Sz, cache


def forward_tolerance(params, B, points, dims):
    """Outputs of the bfloat16/binary32 network and their element tolerances."""
    y, L, S, _ = forward_tracked(params, B, points, dims)
    return y, L + KAPPA * S


def gradient_tolerance(params, B, points, target, dims, depth):
    """Mean squared error and its parameter gradient (flat, the layout of
    params) for the bfloat16/binary32 network, with tolerances.  depth: the
    longest chain of binary32 additions in the library's sums over rows
    (weight and bias gradients).  Returns (loss, loss_tol, grad, grad_tol)."""
    params = np.asarray(params, np.float64)
    layers = unpack(params, dims)
    y, Ly, Sy, cache = forward_tracked(params, B, points, dims)
    t = np.asarray(target, np.float64)
    n_el = y.size
    diff = y - t
    loss = float((diff ** 2).sum() / n_el)
    # loss error: sum 2 diff dy + dy^2 over the outputs; the flip parts of dy
    # have independent signs (quadrature), the binary32 parts add up
    ed = Ly + np.abs(diff) * U32
    loss_tol = float(((2 * np.abs(diff) * ed + (ed + KAPPA * Sy) ** 2).sum()
                      + KAPPA * np.sqrt(((2 * diff * Sy) ** 2).sum())) / n_el + 1e-12 * loss)
    g = 2.0 * diff / n_el
    dz, Ldz, Sdz = round_tracked(g, 2.0 / n_el * Ly + np.abs(g) * 3 * U32, 2.0 / n_el * Sy)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        x, Lx, Sx = cache[li][0], cache[li][1], cache[li][2]
        ax, adz = np.abs(x), np.abs(dz)
        gW = x.T @ dz
        LgW = (ax.T @ Ldz + Lx.T @ adz + Lx.T @ Ldz
               + 2 * U32 * depth * (ax.T @ adz + Lx.T @ adz + ax.T @ Ldz + KAPPA * (Sx.T @ adz + ax.T @ Sdz)))
        SgW = np.sqrt((x * x).T @ (Sdz * Sdz) + (Sx * Sx).T @ (dz * dz) + (Sx * Sx).T @ (Sdz * Sdz))
        gb = dz.sum(axis=0)
        Lgb = Ldz.sum(axis=0) + 2 * U32 * depth * (adz + Ldz + KAPPA * Sdz).sum(axis=0)
        Sgb = np.sqrt((Sdz * Sdz).sum(axis=0))
        grads[li] = (gW, gb, LgW + KAPPA * SgW, Lgb + KAPPA * Sgb)
        if li == 0:
            break
        Wb = bf16_round(layers[li][0])
        aW = np.abs(Wb)
        dA = dz @ Wb.T
        LdA = Ldz @ aW.T + 2 * U32 * (Wb.shape[1] + 1) * ((adz + Ldz + KAPPA * Sdz) @ aW.T)
        SdA = np.sqrt((Sdz * Sdz) @ (Wb * Wb).T)
        z, Lz, Sz = cache[li - 1][3], cache[li - 1][4], cache[li - 1][5]
        sg = sigmoid(z)
        sp = sg * (1.0 + z * (1.0 - sg))
        Lsp = 0.5 * Lz + (2.0 * np.abs(z) + 20.0) * (1.0 + np.abs(z)) * U32
        Ssp = 0.5 * Sz
        gz = dA * sp
        Lgz = np.abs(sp) * LdA + np.abs(dA) * Lsp + LdA * Lsp + np.abs(gz) * 2 * U32
        Sgz = np.sqrt((sp * SdA) ** 2 + (dA * Ssp) ** 2)
        dz, Ldz, Sdz = round_tracked(gz, Lgz, Sgz)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb, _, _ in grads])
    tol = np.concatenate([np.concatenate([tW.ravel(), tb]) for _, _, tW, tb in grads])
    return loss, loss_tol, flat, tol
