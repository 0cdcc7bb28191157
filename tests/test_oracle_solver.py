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
