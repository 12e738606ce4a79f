"""FP64 numpy reference of the warm-start coordinate network.

TEST INFRASTRUCTURE ONLY: checks the GPU network's forward pass and
gradients.  Plain, unblocked numpy; no code shared with the GPU path.

Network (the same definition the GPU library implements): features
[x, y, s, sin(2 pi B p), cos(2 pi B p)] of a point p = (x, y, s), then SiLU
layers z -> z sigmoid(z), then a linear output; loss = mean squared error
over all outputs.  Parameters are one flat vector: for each layer W_l
([in][out], row-major) then b_l.  Pinned by central finite differences
(tests/test_oracle_mlp.py).
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
