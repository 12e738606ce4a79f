"""Cavity batches (smrt_batch_*): every cavity of a batch must be bitwise
identical to the same cavity run alone through smrt_step, across graph
replays, autotuned launch shapes and retirement; one cavity is also checked
against the CPU oracle."""
import numpy as np
import pytest

import oracle as O
from gpu_util import max_vel_err, require_gpu, torch

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (100, 77), (130, 130), (37, 200), (256, 64), (3, 3)]
RES = [100.0, 400.0, 1000.0, 250.0, 2000.0, 50.0]


@pytest.fixture(scope="module")
def smrt():
    return require_gpu()


def single_run(smrt, nx, ny, re, steps, scheme="smrt", storage="f32"):
    with smrt.Solver(nx, ny, scheme=scheme, boundary="cavity", storage=storage, re=re,
                     u_lid=0.1) as s:
        s.step(steps)
        return [t.cpu().numpy() for t in s.moments(torch.float64)]


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("scheme", ["smrt", "srt"])
def test_batch_matches_single_lattice_bitwise(smrt, scheme, storage):
    nx, ny = zip(*SIZES)
    with smrt.Batch(nx, ny, scheme=scheme, storage=storage, re=RES, u_lid=0.1) as b:
        # two replays of a 64-launch graph, then a few single launches with a
        # shorter remainder launch at the end
        steps = 2 * 64 * b.steps_per_launch + 7
        b.step(steps)
        assert b.steps_done == steps and b.running == len(SIZES)
        got = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(SIZES))]
    for i, ((x, y), re) in enumerate(zip(SIZES, RES)):
        want = single_run(smrt, x, y, re, steps, scheme, storage)
        for g, w in zip(got[i], want):
            assert np.array_equal(g, w), (i, x, y)


def test_autotune_keeps_results_bitwise(smrt):
    nx, ny = zip(*SIZES)
    with smrt.Batch(nx, ny, scheme="smrt", storage="f32", re=RES, u_lid=0.1) as b:
        bx, by, grid = b.autotune(steps=6)
        assert bx * by in (256, 512, 1024, 1408) and grid >= 1 and b.steps_per_launch in (1, 2, 3, 4, 5)
        done = b.steps_done
        b.step(130 - done if done < 130 else 0)
        steps = b.steps_done
        got = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(SIZES))]
    for i, ((x, y), re) in enumerate(zip(SIZES, RES)):
        want = single_run(smrt, x, y, re, steps)
        for g, w in zip(got[i], want):
            assert np.array_equal(g, w), i


@pytest.mark.parametrize("bx,by,steps", [(64, 22, 5), (64, 22, 4), (64, 22, 3), (64, 22, 2), (64, 16, 5),
                                          (64, 8, 4), (64, 4, 2), (128, 2, 1)])
def test_set_launch_keeps_results_bitwise(smrt, bx, by, steps):
    """Every tile shape, with graph replays and shorter remainder launches
    (one-step remainders on 64 x 22 tables take two row passes a block)."""
    nx, ny = zip(*SIZES)
    with smrt.Batch(nx, ny, scheme="smrt", storage="f32", re=RES, u_lid=0.1) as b:
        b.set_launch(bx, by, steps)
        assert b.steps_per_launch == steps
        n = 64 * steps + steps + 1 if steps > 1 else 70   # one graph, one full launch, remainders
        for chunk in (n, 1, steps - 1 if steps > 1 else 1):
            b.step(chunk)
        total = b.steps_done
        got = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(SIZES))]
    for i, ((x, y), re) in enumerate(zip(SIZES, RES)):
        want = single_run(smrt, x, y, re, total)
        for g, w in zip(got[i], want):
            assert np.array_equal(g, w), (i, bx, by, steps)


def test_set_launch_rejects_unbuilt_shapes(smrt):
    with smrt.Batch([64], [64], scheme="smrt", storage="f32", re=[100.0], u_lid=0.1) as b:
        for bx, by, steps in [(64, 22, 1), (64, 12, 5), (32, 22, 5), (64, 4, 3), (64, 16, 6)]:
            with pytest.raises(smrt.SmrtError):
                b.set_launch(bx, by, steps)
    with smrt.Batch([64], [64], scheme="smrt", storage="f64", re=[100.0], u_lid=0.1) as b:
        with pytest.raises(smrt.SmrtError):
            b.set_launch(64, 16, 5)
        b.set_launch(64, 8, 1)


def test_batch_cavity_against_oracle(smrt):
    n, steps = 48, 600
    with smrt.Batch([n, 32], [n, 40], scheme="smrt", storage="f32", re=[150.0, 80.0],
                    u_lid=0.1) as b:
        b.step(steps)
        g = [t.cpu().numpy() for t in b.moments(0)]
    L = O.Lattice(n, n, "smrt", re=150.0, u_lid=0.1)
    o = L.fields(L.run(L.init_equilibrium(), steps))
    assert max_vel_err(g, o) / 0.1 <= 1e-5


def test_run_retires_steady_and_unstable_cavities(smrt):
    """Two small cavities converge; an SRT-unstable one (tau barely above 1/2 with a
    fast lid) is flagged; results equal the single-lattice runs at the reported steps."""
    nx, ny = [24, 32, 100], [24, 30, 100]
    tau = [0.8, 0.7, 0.51]
    with smrt.Batch(nx, ny, scheme="srt", storage="f32", tau=tau, u_lid=0.1667) as b:
        steps, status, res = b.run(tol=1e-6, window=500, max_steps=200_000)
        assert b.running == 0
        fields = [[t.cpu().numpy() for t in b.moments(i)] for i in range(2)]
    assert status[:2] == [smrt.STEADY, smrt.STEADY] and status[2] == smrt.UNSTABLE
    assert all(r < 1e-6 for r in res[:2]) and np.isnan(res[2])
    for i in range(2):
        with smrt.Solver(nx[i], ny[i], scheme="srt", boundary="cavity", storage="f32", tau=tau[i],
                         u_lid=0.1667) as s:
            k, r, ok = s.run_to_steady(1e-6, 500, 200_000)
            assert ok and k == steps[i]
            want = [t.cpu().numpy() for t in s.moments(torch.float64)]
        for g, w in zip(fields[i], want):
            assert np.array_equal(g, w)


def test_init_fields_in_a_batch(smrt):
    n = 40
    rho = torch.ones((n, n), dtype=torch.float32, device="cuda:0")
    ux = torch.full((n, n), 0.01, dtype=torch.float32, device="cuda:0")
    with smrt.Batch([n, n], [n, n], scheme="smrt", storage="f32", tau=[0.7, 0.7], u_lid=0.0) as b:
        b.init_fields(1, rho, ux, None)
        _, gx0, _ = b.moments(0)
        _, gx1, _ = b.moments(1)
        assert float(gx0.abs().max()) == 0.0
        assert abs(float(gx1.mean()) - 0.01) < 1e-7
    with pytest.raises(smrt.SmrtError):
        smrt.Batch([2], [5], tau=[0.7])
