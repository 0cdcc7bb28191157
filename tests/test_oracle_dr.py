"""Pins of the oracle's Douglas-Rachford solver (CPU only)."""
import numpy as np

import synth
from oracle import dr, metrics, solver, wavelet, wproj
from oracle.wproj import Setup


def test_projection_with_identity_operator_is_the_ball_projection():
    """Phi = I (a tight frame, ||Phi||^2 = 1): one dual step gives P_C(z) = P_B(z) exactly."""
    rng = np.random.default_rng(81)
    y = rng.normal(size=(8, 8))
    z = y + 3.0 * rng.normal(size=(8, 8))
    eps = 2.0
    A = lambda t: np.asarray(t, dtype=np.complex128)
    AH = lambda r: np.asarray(r)
    got, _ = dr.project_constraint(z, y.astype(np.complex128), A, AH, eps, 1.0, 1)
    r = z - y
    want = y + r * min(1.0, eps / np.linalg.norm(r))
    assert np.abs(got - want).max() < 1e-13
    inside = y + 0.1 * (z - y) / np.linalg.norm(z - y)
    got, _ = dr.project_constraint(inside, y.astype(np.complex128), A, AH, eps, 1.0, 3)
    assert np.abs(got - inside).max() < 1e-13


def test_douglas_rachford_and_primal_dual_reach_the_same_solution():
    """Eq. 7 without positivity: two different splittings converge to one minimiser."""
    N, M = 16, 400
    s = Setup(N=N, L=synth.fov_L())
    u, v, w = synth.uvw(N, M, s.L, "uniform", 0.0, N / (2 * s.L ** 2), np.random.default_rng(71))
    G = wproj.build_rows(u, v, w, 0.99, s)
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    x = synth.sky(N, 2, 3, np.random.default_rng(72))
    y0 = A(x)
    sig = metrics.noise_sigma(y0, 30.0)
    y = y0 + synth.noise(M, sig, np.random.default_rng(73))
    eps = metrics.l2_ball_radius(sig, M)
    nu = solver.power_norm2(A, AH, np.ones((N, N)), 60)
    gamma = 0.01 * np.abs(wavelet.dwt2(np.real(AH(y)) / nu, 2)).max()
    xd = dr.solve(y, A, AH, (N, N), eps, nu, 400, 5, gamma, levels=2)
    xp = solver.solve(y, A, AH, (N, N), eps, nu, 3000, levels=2, positive=False)
    assert np.linalg.norm(A(xd) - y) <= eps * (1 + 1e-9)              # feasible
    l1 = lambda z: np.abs(wavelet.dwt2(z, 2)).sum()
    # the primal-dual run is still 1e-5 from feasibility after 3000 iterations (4000 bring the two
    # within 6e-7)
    assert abs(l1(xd) - l1(xp)) < 1e-4 * l1(xp)
    assert np.linalg.norm(xd - xp) < 5e-4 * np.linalg.norm(xp)
