"""smrt_mass_noalloc (the allocation-free variant of smrt_mass, its partial
sums in the library's static device scratch) against smrt_mass, through the
C ABI: bitwise the same mass on two calls in a row, the second on a smaller
lattice, and the same non-finite verdict."""
import ctypes

import numpy as np
import pytest

from gpu_util import require_gpu, to_dev, torch
from paper_2409_01076_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smrt():
    return require_gpu()


def both_masses(smrt, solver):
    lib = smrt.load()
    host = ctypes.c_double()
    rc_host = lib.smrt_mass(solver._ctx, ctypes.byref(host))
    dev = torch.full((2,), -1.0, dtype=torch.float64, device="cuda:0")
    rc_dev = lib.smrt_mass_noalloc(solver._ctx, ctypes.c_void_p(dev.data_ptr()))
    assert rc_dev == smrt.OK, lib.smrt_last_error()
    assert lib.smrt_synchronize(solver._ctx) == smrt.OK
    return rc_host, host.value, dev.cpu().numpy()


def test_noalloc_mass_equals_mass_large_then_small(smrt):
    print("case: 300x157 cavity f32 smrt, then 48x40 periodic f64 srt", flush=True)
    with smrt.Solver(300, 157, scheme="smrt", boundary="cavity", storage="f32", re=200.0, u_lid=0.1) as big:
        big.step(137)
        rc, m_host, m_dev = both_masses(smrt, big)
        assert rc == smrt.OK
        assert m_dev[0] == m_host and m_dev[1] == 0.0
        assert abs(m_host / (300 * 157) - 1) < 1e-6
    rho, ux, uy = inputs.taylor_green(48, 40, u0=0.05, noise=1e-3)
    with smrt.Solver(48, 40, scheme="srt", boundary="periodic", storage="f64", tau=0.7) as small:
        small.init_fields(to_dev(rho, torch.float64), to_dev(ux, torch.float64), to_dev(uy, torch.float64))
        small.step(23)
        rc, m_host, m_dev = both_masses(smrt, small)
        assert rc == smrt.OK
        assert m_dev[0] == m_host and m_dev[1] == 0.0
        assert m_host == pytest.approx(float(np.sum(rho.astype(np.float64))), rel=1e-12)


def test_noalloc_mass_reports_non_finite_nodes(smrt):
    print("case: 64x64 cavity f32 with one NaN population", flush=True)
    with smrt.Solver(64, 64, scheme="smrt", boundary="cavity", storage="f32", re=100.0, u_lid=0.1) as s:
        f = s.populations(torch.float64)
        f[3, 10, 20] = float("nan")
        s.set_populations(f)
        rc, m_host, m_dev = both_masses(smrt, s)
        assert rc == smrt.EUNSTABLE and np.isnan(m_host)
        assert np.isnan(m_dev[0]) and m_dev[1] == 1.0


def test_noalloc_mass_rejects_null(smrt):
    lib = smrt.load()
    assert lib.smrt_mass_noalloc(None, None) == smrt.EINVAL
    with smrt.Solver(16, 16, storage="f32", re=10.0, u_lid=0.1) as s:
        assert lib.smrt_mass_noalloc(s._ctx, None) == smrt.EINVAL
