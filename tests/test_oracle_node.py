"""Pins of the oracle's per-node arithmetic against what the paper fixes.

Equilibrium, moments and the three collisions (SRT, SmrtLBM, the
two-relaxation-time form) are checked against: the paper's own constants
(tests/golden/d2q9_paper.txt), the closed-form moments of the D2Q9
equilibrium, the MRT matrix form of the appendix (Eq. lb.1 with the printed M
and S), and the special cases the paper states (tau_s = tau gives SRT,
tau_s = 1 gives SmrtLBM).
"""
import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(2409010760)


def random_state(rng, scale=0.05):
    """A positive, non-equilibrium population vector near rest."""
    _, _, w, _ = O.constants()
    rho = 1.0 + 0.02 * rng.uniform(-1, 1)
    u = rng.uniform(-0.08, 0.08, size=2)
    feq = O.equilibrium(rho, u[0], u[1])
    return feq * (1.0 + scale * rng.uniform(-1, 1, size=9))


def test_constants_match_paper(paper_constants):
    vel, w, M, _ = paper_constants
    ex, ey, ow, opp = O.constants()
    assert np.array_equal(ex, vel[:, 0]) and np.array_equal(ey, vel[:, 1])
    assert np.allclose(ow, w, rtol=0, atol=1e-16)
    for a in range(9):
        assert ex[opp[a]] == -ex[a] and ey[opp[a]] == -ey[a]
    # The printed M and the printed velocity set agree: rows 3 and 5 of M are
    # the x and y momentum, row 0 the density.
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], vel[:, 0]) and np.array_equal(M[5], vel[:, 1])
    # M's rows are mutually orthogonal, so M is invertible.
    G = M @ M.T
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0


@pytest.mark.parametrize("seed", range(20))
def test_equilibrium_moments_closed_form(seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.2, 0.2, size=2)
    ex, ey, _, _ = O.constants()
    feq = O.equilibrium(rho, u[0], u[1])
    e = np.stack([ex, ey], axis=1).astype(float)
    assert abs(feq.sum() - rho) < 1e-14
    assert np.allclose(e.T @ feq, rho * u, rtol=0, atol=1e-15)
    # second moment of the D2Q9 equilibrium: rho/3 I + rho u u
    P = np.einsum("ai,aj,a->ij", e, e, feq)
    assert np.allclose(P, rho / 3.0 * np.eye(2) + rho * np.outer(u, u), rtol=0, atol=1e-15)
    # the rest weight multiplies rho (1 - 3/2 u.u)
    assert abs(feq[0] - 4.0 / 9.0 * rho * (1 - 1.5 * u @ u)) < 1e-15


def test_node_moments_brute_force():
    ex, ey, _, _ = O.constants()
    for a in range(9):
        f = np.zeros(9)
        f[a] = 2.0
        r, ux, uy = O.node_moments(f)
        assert r == 2.0 and ux == ex[a] and uy == ey[a]
    f = np.arange(1.0, 10.0)
    r, ux, uy = O.node_moments(f)
    assert r == 45.0
    assert abs(ux - (2 - 4 + 6 - 7 - 8 + 9) / 45.0) < 1e-16
    assert abs(uy - (3 - 5 + 6 + 7 - 8 - 9) / 45.0) < 1e-16


@pytest.mark.parametrize("scheme", ["srt", "smrt", "trt"])
@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0, 1.7])
def test_equilibrium_is_fixed_point(scheme, tau):
    feq = O.equilibrium(1.01, 0.04, -0.03)
    out = O.node_collide(feq, scheme, tau, tau_s=0.8)
    assert np.allclose(out, feq, rtol=0, atol=1e-16)


@pytest.mark.parametrize("scheme", ["srt", "smrt", "trt"])
def test_collision_conserves_mass_and_momentum(scheme):
    ex, ey, _, _ = O.constants()
    for _ in range(50):
        f = random_state(RNG)
        out = O.node_collide(f, scheme, 0.57, tau_s=0.9)
        assert abs(out.sum() - f.sum()) < 1e-15
        assert abs(ex @ out - ex @ f) < 1e-15 and abs(ey @ out - ey @ f) < 1e-15


def mrt_collide(M, f, tau, tau_s, relaxed):
    """Eq. (lb.1) right-hand side with the paper's M and S = diag(1/tau_s.., 1/tau, 1/tau)."""
    r, ux, uy = O.node_moments(f)
    feq = O.equilibrium(r, ux, uy)
    s = np.full(9, 1.0 / tau_s)
    s[relaxed] = 1.0 / tau
    return f - np.linalg.solve(M, s * (M @ (f - feq)))


@pytest.mark.parametrize("tau", [0.502, 0.51, 0.6, 0.8072, 1.0, 1.5])
def test_smrt_equals_mrt_matrix_form(paper_constants, tau):
    """SmrtLBM is MRT with every rate 1 except the two stress rates 1/tau."""
    _, _, M, relaxed = paper_constants
    for _ in range(200):
        f = random_state(RNG)
        a = O.node_collide(f, "smrt", tau)
        b = mrt_collide(M, f, tau, 1.0, relaxed)
        assert np.max(np.abs(a - b)) < 2e-16 * 16


@pytest.mark.parametrize("tau,tau_s", [(0.51, 0.9), (0.6, 1.3), (1.2, 0.55)])
def test_trt_equals_mrt_matrix_form(paper_constants, tau, tau_s):
    _, _, M, relaxed = paper_constants
    for _ in range(200):
        f = random_state(RNG)
        a = O.node_collide(f, "trt", tau, tau_s=tau_s)
        b = mrt_collide(M, f, tau, tau_s, relaxed)
        assert np.max(np.abs(a - b)) < 2e-16 * 32


@pytest.mark.parametrize("tau", [0.51, 0.6, 0.9, 1.4])
def test_trt_special_cases(tau):
    """tau_s = tau gives SRT and tau_s = 1 gives SmrtLBM (paper, after Eq. SmrtLBM-lb.1.5)."""
    for _ in range(100):
        f = random_state(RNG)
        assert np.max(np.abs(O.node_collide(f, "trt", tau, tau_s=tau) -
                             O.node_collide(f, "srt", tau))) < 1e-16
        assert np.max(np.abs(O.node_collide(f, "trt", tau, tau_s=1.0) -
                             O.node_collide(f, "smrt", tau))) < 1e-16


def test_tau_one_all_schemes_give_equilibrium():
    for _ in range(50):
        f = random_state(RNG)
        r, ux, uy = O.node_moments(f)
        feq = O.equilibrium(r, ux, uy)
        for scheme in ("srt", "smrt"):
            assert np.max(np.abs(O.node_collide(f, scheme, 1.0) - feq)) < 1e-16


def test_smrt_sign_pattern_is_stress_moments(paper_constants):
    """f*_a - f^eq_a = (-1)^a (1 - 1/tau) C_g(a), with C_1 = -m_7/4, C_2 = -m_8/4
    where m = M (f - f^eq) are the paper's moments (Eq. sigma1-2-0, Eq. M-matrix)."""
    _, _, M, _ = paper_constants
    tau = 0.55
    for _ in range(100):
        f = random_state(RNG)
        r, ux, uy = O.node_moments(f)
        feq = O.equilibrium(r, ux, uy)
        m = M @ (f - feq)
        c1, c2 = -m[7] / 4.0, -m[8] / 4.0
        want = feq.copy()
        for a in range(1, 9):
            want[a] += (-1) ** a * (1 - 1 / tau) * (c1 if a <= 4 else c2)
        assert np.max(np.abs(O.node_collide(f, "smrt", tau) - want)) < 1e-16 * 8


def test_collide_rejects_bad_tau():
    f = random_state(RNG)
    with pytest.raises(ValueError):
        O.node_collide(f, "smrt", 0.5)
    with pytest.raises(ValueError):
        O.node_collide(f, "trt", 0.6, tau_s=0.4)


def test_tau_from_re_viscosity_relation():
    # nu = U N / Re and nu = (2 tau - 1)/6 (Eq. relation-chapman-viscosity, e = dx = 1)
    assert abs(O.tau_from_re(100, 0.1, 64) - (0.5 + 3 * 0.064)) < 1e-15
    assert abs(O.tau_from_re(1000, 0.1, 1024) - 0.8072) < 1e-15
    tau = O.tau_from_re(7000, 0.1, 300)
    assert abs((2 * tau - 1) / 6 - 0.1 * 300 / 7000) < 1e-15
