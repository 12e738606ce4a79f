"""What the learned warm start gains: a network trained (on the GPU, by the
library's kernels) on steady cavity fields from the solver reaches the steady
residual in fewer steps than the uniform cold start on held-out Reynolds
numbers, and both runs end on the same field."""
import numpy as np
import pytest

from gpu_util import require_gpu, torch

pytestmark = pytest.mark.gpu

N, U, TOL, WINDOW = 48, 0.1, 1e-7, 500


@pytest.fixture(scope="module")
def smrt():
    return require_gpu()


def steady_fields(smrt, res):
    with smrt.Batch([N] * len(res), [N] * len(res), scheme="smrt", storage="f32", re=res,
                    u_lid=U) as b:
        steps, status, _ = b.run(TOL, WINDOW, 400_000)
        fields = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(res))]
    return np.array(steps), np.array(status), fields


def test_warm_start_cuts_steps_to_steady(smrt):
    from paper_2409_01076_amd import warmstart as W
    rng = np.random.default_rng(11)
    train_re = 100.0 * 10.0 ** rng.uniform(0, 1, size=16)
    test_re = np.array([130.0, 270.0, 480.0, 850.0])
    steps, status, fields = steady_fields(smrt, train_re)
    assert (status == smrt.STEADY).all()
    pts = np.concatenate([W.cavity_points(N, r) for r in train_re])
    tgt = np.concatenate([W.targets(*f, U) for f in fields])
    ws = W.WarmStart(fourier=16, width=128, layers=5, batch=4096)
    hist = ws.fit(pts, tgt, epochs=150, lr=3e-3)
    assert hist[-1][1] < hist[0][1] / 10

    cold_steps, cold_status, cold = steady_fields(smrt, test_re)
    with smrt.Batch([N] * 4, [N] * 4, scheme="smrt", storage="f32", re=test_re, u_lid=U) as b:
        for i, r in enumerate(test_re):
            b.init_fields(i, *ws.predict(N, r, U))
        warm_steps, warm_status, _ = b.run(TOL, WINDOW, 400_000)
        warm = [[t.cpu().numpy() for t in b.moments(i)] for i in range(4)]
    ws.close()
    assert (np.array(cold_status) == smrt.STEADY).all() and (np.array(warm_status) == smrt.STEADY).all()
    err = max(max(np.abs(w[1] - c[1]).max(), np.abs(w[2] - c[2]).max()) for w, c in zip(warm, cold)) / U
    print("cold steps %s, warm steps %s, final-field max|du|/U %.2e" % (list(cold_steps), list(warm_steps), err))
    assert np.mean(warm_steps) < 0.8 * np.mean(cold_steps)
    assert err < 1e-2
