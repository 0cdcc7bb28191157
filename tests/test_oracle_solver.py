"""Pins of the oracle's l1 solver (CPU only).  Parity unpinned against the paper's printed SNRs."""
import numpy as np

import synth
from oracle import metrics, solver, wavelet, wproj
from oracle.wproj import Setup

L = synth.fov_L()


def test_noiseless_full_coverage_converges():
    N, M = 16, 1200
    s = Setup(N=N, L=L)
    rng = np.random.default_rng(7)
    u, v, w = synth.uvw(N, M, L, "uniform", 0.0, N / (2 * L * L), rng)
    G = wproj.build_rows(u, v, w, 1.0, s)
    x = synth.sky(N, 3, 4, np.random.default_rng(8))
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    y = A(x)
    nu = solver.power_norm2(A, AH, np.random.default_rng(9).normal(size=(N, N)), 60)
    eps = 1e-6 * np.linalg.norm(y)
    xr, hist = solver.solve(y, A, AH, (N, N), eps, nu, 600, levels=2, history=True, x_true=x)
    assert hist[-1] > 40.0
    assert np.mean(hist[-50:]) > np.mean(hist[100:150])


def test_constraint_met_when_ball_is_loose():
    """With eps above ||y||, x = 0 is feasible and optimal: the solver must return ~0."""
    N, M = 16, 200
    s = Setup(N=N, L=L)
    u, v, w = synth.uvw(N, M, L, "uniform", 0.0, 1000.0, np.random.default_rng(3))
    G = wproj.build_rows(u, v, w, 0.99, s)
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    x = synth.sky(N, 2, 2, np.random.default_rng(4))
    y = A(x)
    nu = solver.power_norm2(A, AH, np.ones((N, N)), 40)
    xr = solver.solve(y, A, AH, (N, N), 1.01 * np.linalg.norm(y), nu, 200, levels=2)
    assert np.abs(xr).max() < 1e-6 * np.abs(x).max() + 1e-9


def test_power_iteration_matches_dense_norm():
    N, M = 8, 50
    s = Setup(N=N, L=L)
    u, v, w = synth.uvw(N, M, L, "uniform", 0.0, 500.0, np.random.default_rng(5))
    G = wproj.build_rows(u, v, w, 0.9, s)
    cols = []
    for i in range(N * N):
        e = np.zeros(N * N); e[i] = 1
        cols.append(wproj.phi(G, e.reshape(N, N), s))
    A = np.array(cols).T
    Ar = np.vstack([A.real, A.imag])      # real image domain
    want = np.linalg.norm(Ar, 2) ** 2
    got = solver.power_norm2(lambda z: wproj.phi(G, z, s), lambda r: wproj.phi_adjoint(G, r, s),
                             np.random.default_rng(6).normal(size=(N, N)), 300)
    assert abs(got - want) < 1e-6 * want


def test_snr_definition():
    x = np.arange(16.0).reshape(4, 4)
    assert metrics.snr_out(x, x + 0.01 * np.std(x) * np.sign(np.arange(16).reshape(4, 4) % 2 - 0.5)) > 39.9


def _soft_threshold_level(y, eps):
    """lambda >= 0 with ||min(y, lambda)||_2 = eps (y >= 0, ||y|| > eps), by bisection."""
    lo, hi = 0.0, float(y.max())
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.norm(np.minimum(y, mid)) < eps:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_dirac_basis_identity_operator_closed_form():
    """Psi = I, Phi = I: min ||x||_1 s.t. ||y - x|| <= eps, x >= 0 is soft thresholding of y."""
    N = 16
    y = np.abs(np.random.default_rng(11).normal(size=(N, N))) ** 2
    eps = 0.3 * np.linalg.norm(y)
    A = lambda z: np.asarray(z, dtype=np.complex128)
    AH = lambda r: np.asarray(r)
    lam = _soft_threshold_level(y, eps)
    want = np.maximum(0.0, y - lam)
    nu = solver.power_norm2(A, AH, np.random.default_rng(12).normal(size=(N, N)), 5)
    assert abs(nu - 1.0) < 1e-12
    got = solver.solve(y.astype(np.complex128), A, AH, (N, N), eps, nu, 3000, levels=0)
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max()
    # the same problem in the wavelet basis has a different (non-thresholded) solution
    got_db = solver.solve(y.astype(np.complex128), A, AH, (N, N), eps, nu, 3000, levels=2)
    assert np.abs(got_db - want).max() > 1e-3 * np.abs(want).max()


def test_dirac_transform_is_identity():
    x = np.random.default_rng(13).normal(size=(8, 8))
    assert np.array_equal(wavelet.dwt2(x, 0), x) and np.array_equal(wavelet.idwt2(x, 0), x)


def test_residual_image_against_dense_normal_matrix():
    """x_res = Re(A^H A)(x_rec - x) with A the dense matrix whose columns are Phi of unit images."""
    N, M = 8, 60
    s = Setup(N=N, L=L)
    u, v, w = synth.uvw(N, M, L, "uniform", 0.0, 500.0, np.random.default_rng(14))
    G = wproj.build_rows(u, v, w, 0.9, s)
    cols = []
    for i in range(N * N):
        e = np.zeros(N * N); e[i] = 1
        cols.append(wproj.phi(G, e.reshape(N, N), s))
    A = np.array(cols).T
    rng = np.random.default_rng(15)
    x, xr = rng.normal(size=(N, N)), rng.normal(size=(N, N))
    want = np.real(A.conj().T @ (A @ (xr - x).ravel())).reshape(N, N)
    got = solver.residual_image(lambda z: wproj.phi(G, z, s), lambda r: wproj.phi_adjoint(G, r, s), xr, x)
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    assert np.abs(solver.residual_image(lambda z: wproj.phi(G, z, s), lambda r: wproj.phi_adjoint(G, r, s),
                                        x, x)).max() == 0.0
