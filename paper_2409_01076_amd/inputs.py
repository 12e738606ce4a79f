"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws initial fields; it holds none of the lattice
Boltzmann arithmetic.  Fields are generated in FP64 on the host and rounded
to FP32 once, so the GPU library and the CPU oracle start from identical
values (the oracle receives the FP32 values widened back to FP64).

Recipes (lattice units, arrays indexed [y, x]):
  taylor_green  u_x = -u0 cos(k x) sin(k y), u_y = u0 sin(k x) cos(k y),
                k = 2 pi / N, rho = 1 + xi with xi ~ U(-amp, amp) i.i.d.
  shear_wave    u_x = u0 sin(k y), u_y = 0, rho = 1 + xi
  perturbed     a non-equilibrium population field f = f_w (1 + eps), for
                collision checks from states that are not equilibria
"""
import numpy as np

DEFAULT_SEED = 2409010760


def _noise(rng, shape, amp):
    return rng.uniform(-amp, amp, size=shape) if amp else np.zeros(shape)


def taylor_green(nx, ny, u0=0.05, noise=1e-3, seed=DEFAULT_SEED):
    """(rho, ux, uy) float32 arrays of shape (ny, nx)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    ux = -u0 * np.cos(kx * x) * np.sin(ky * y)
    uy = u0 * np.sin(kx * x) * np.cos(ky * y)
    rho = 1.0 + _noise(rng, (ny, nx), noise)
    return tuple(a.astype(np.float32) for a in (rho, ux, uy))


def shear_wave(nx, ny, u0=0.05, noise=1e-3, seed=DEFAULT_SEED):
    """(rho, ux, uy) float32 arrays of shape (ny, nx)."""
    rng = np.random.default_rng(seed)
    y = np.mgrid[0:ny, 0:nx][0].astype(np.float64)
    ux = u0 * np.sin(2 * np.pi / ny * y)
    uy = np.zeros((ny, nx))
    rho = 1.0 + _noise(rng, (ny, nx), noise)
    return tuple(a.astype(np.float32) for a in (rho, ux, uy))


def perturbed_populations(nx, ny, eps=0.05, seed=DEFAULT_SEED):
    """float64 array (9, ny, nx): rest-state weights times (1 + U(-eps, eps)) with
    a random drift added to the axis and diagonal directions, so that the
    field has non-zero velocity and is far from equilibrium."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    f = w * (1.0 + rng.uniform(-eps, eps, size=(9, ny, nx)))
    tilt = rng.uniform(-eps, eps, size=(2, ny, nx))
    f[1] *= 1 + tilt[0]
    f[5] *= 1 + tilt[1]
    return f


def cavity_batch(count, n_lo=64, n_hi=512, re_lo=100.0, re_hi=10000.0, seed=DEFAULT_SEED):
    """Side lengths and Reynolds numbers drawn log-uniformly: (n[int], re[float])."""
    rng = np.random.default_rng(seed)
    u, v = rng.uniform(size=count), rng.uniform(size=count)
    n = np.round(n_lo * (n_hi / n_lo) ** u).astype(np.int64)
    re = re_lo * (re_hi / re_lo) ** v
    return n, re
