"""Pins of the FP64 network reference: its gradient matches central finite
differences of its own loss (a check independent of the backward formulas),
and its features follow the stated definition on hand-computable points."""
import numpy as np

from oracle import mlp_oracle as M


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
