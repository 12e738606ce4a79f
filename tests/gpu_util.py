"""Helpers shared by the GPU parity tests: run the HIP library and the CPU
oracle on the same seeded inputs and compare them.

The GPU state after n steps holds the post-collision populations f*(n); the
oracle, which follows the paper's collide-then-stream order, holds the
pre-collision f(n).  Moments agree because the collision conserves density and
momentum; populations are compared as f*(n) against collide(f(n)).
"""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_01076_amd import smrt
    smrt.load()   # raises if the HIP library is missing: no silent fallback
    return smrt


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def gpu_fields(solver):
    rho, ux, uy = solver.moments(torch.float64)
    return rho.cpu().numpy(), ux.cpu().numpy(), uy.cpu().numpy()


def gpu_populations(solver):
    """(ny, nx, 9) float64, oracle node-major layout."""
    return np.moveaxis(solver.populations(torch.float64).cpu().numpy(), 0, -1)


def oracle_lattice(nx, ny, scheme, boundary, tau, u_lid=0.0, tau_s=1.0):
    """The oracle lattice for a library boundary name ('cavity_eqlid': the
    cavity under the equilibrium-lid reading)."""
    if boundary == "cavity_eqlid":
        return O.Lattice(nx, ny, scheme, tau=tau, u_lid=u_lid, boundary="cavity", tau_s=tau_s,
                         lid="equilibrium")
    return O.Lattice(nx, ny, scheme, tau=tau, u_lid=u_lid, boundary=boundary, tau_s=tau_s)


def oracle_from_fields(L, rho, ux, uy, steps):
    """Oracle populations f(steps) from f(0) = f^eq(rho, u)."""
    f = L.init_equilibrium(np.asarray(rho, np.float64), np.asarray(ux, np.float64),
                           np.asarray(uy, np.float64))
    return L.run(f, steps)


def oracle_from_post_collision(L, fstar0, steps):
    """Oracle f(steps) when the state at step 0 is the post-collision field fstar0
    (what the GPU stores): stream once, then steps-1 collide-stream steps."""
    f = L.stream(fstar0)
    return L.run(f, steps - 1)


def max_vel_err(a, b):
    return max(np.max(np.abs(a[1] - b[1])), np.max(np.abs(a[2] - b[2])))


def window_indices(n, c, h):
    """Indices c-h .. c+h wrapped onto 0..n-1."""
    return np.arange(c - h, c + h + 1) % n


def oracle_sample_periodic(L_params, rho, ux, uy, cells, steps, chunk=None):
    """Oracle velocity at `cells` [(y, x), ...] after `steps` on a periodic
    lattice, computed on shrinking windows: information moves one node per step,
    so a (2h+1)^2 window wrapped on itself is exact at distance > s from its
    edge after s steps; the window loses `chunk` nodes per side every `chunk`
    steps and ends as the single sampled node."""
    ny, nx = rho.shape
    scheme, tau, tau_s = L_params
    chunk = chunk or max(1, steps // 20)
    out = []
    for (cy, cx) in cells:
        h = steps
        iy, ix = window_indices(ny, cy, h), window_indices(nx, cx, h)
        sub = [np.asarray(a, np.float64)[np.ix_(iy, ix)] for a in (rho, ux, uy)]
        L = O.Lattice(2 * h + 1, 2 * h + 1, scheme, tau=tau, tau_s=tau_s, boundary="periodic")
        f = L.init_equilibrium(*sub)
        done = 0
        while done < steps:
            s = min(chunk, steps - done)
            f = L.run(f, s)
            done += s
            h -= s
            f = np.ascontiguousarray(f[s:-s, s:-s]) if s else f
            L = O.Lattice(2 * h + 1, 2 * h + 1, scheme, tau=tau, tau_s=tau_s, boundary="periodic")
        r, vx, vy = L.fields(f)
        out.append((r[0, 0], vx[0, 0], vy[0, 0]))
    return np.array(out)
