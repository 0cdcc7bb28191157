"""Pins of the oracle's SARA dictionary and weighted solver (CPU only).  Parity unpinned against the
paper's printed SARA SNRs (they need its test images)."""
import numpy as np
import pytest

import synth
from oracle import metrics, sara, solver, wavelet, wproj
from oracle.wproj import Setup


def test_haar_closed_form():
    assert np.abs(wavelet.daubechies_lowpass(1) - np.array([1.0, 1.0]) / np.sqrt(2.0)).max() < 1e-15


@pytest.mark.parametrize("p", [1, 3, 5, 6, 7])
def test_every_sara_basis_is_orthonormal(p):
    N, levels = 32, 2
    x = np.random.default_rng(p).normal(size=(N, N))
    c = wavelet.dwt2(x, levels, p)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-11 * np.linalg.norm(x)
    assert np.abs(wavelet.idwt2(c, levels, p) - x).max() < 1e-11


def test_dictionary_is_a_normalised_tight_frame():
    N, levels = 32, 3
    rng = np.random.default_rng(31)
    x = rng.normal(size=(N, N))
    c = sara.analysis(x, levels)
    assert c.shape == (9, N, N)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-11 * np.linalg.norm(x)   # isometry
    assert np.abs(sara.synthesis(c, levels) - x).max() < 1e-11                       # Psi Psi^T = I
    d = rng.normal(size=(9, N, N))
    assert abs(np.sum(sara.analysis(x, levels) * d) - np.sum(x * sara.synthesis(d, levels))) < 1e-9 * N * N


def test_unit_weights_and_one_basis_equal_the_plain_solver():
    N, M = 16, 300
    s = Setup(N=N, L=synth.fov_L())
    u, v, w = synth.uvw(N, M, s.L, "uniform", 0.0, 500.0, np.random.default_rng(32))
    G = wproj.build_rows(u, v, w, 0.99, s)
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    x = synth.sky(N, 2, 3, np.random.default_rng(33))
    y = A(x)
    nu = solver.power_norm2(A, AH, np.ones((N, N)), 40)
    eps = 0.05 * np.linalg.norm(y)
    want = solver.solve(y, A, AH, (N, N), eps, nu, 60, levels=2)
    dic = (lambda z: wavelet.dwt2(z, 2), lambda c: wavelet.idwt2(c, 2))
    got = solver.solve(y, A, AH, (N, N), eps, nu, 60, dictionary=dic, weights=np.ones((N, N)))
    assert np.abs(got - want).max() == 0.0


def test_weighted_soft_thresholding_closed_form():
    """Psi = I, Phi = I, weights w: x_i = max(0, y_i - lambda w_i) with ||y - x|| = eps."""
    N = 16
    rng = np.random.default_rng(34)
    y = np.abs(rng.normal(size=(N, N))) ** 2
    wts = rng.uniform(0.2, 2.0, size=(N, N))
    eps = 0.3 * np.linalg.norm(y)
    lo, hi = 0.0, float((y / wts).max())
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        if np.linalg.norm(y - np.maximum(0.0, y - lam * wts)) < eps:
            lo = lam
        else:
            hi = lam
    want = np.maximum(0.0, y - 0.5 * (lo + hi) * wts)
    A = lambda z: np.asarray(z, dtype=np.complex128)
    AH = lambda r: np.asarray(r)
    dic = (lambda z: np.array(z, dtype=np.float64), lambda c: np.array(c, dtype=np.float64))
    got = solver.solve(y.astype(np.complex128), A, AH, (N, N), eps, 1.0, 4000, dictionary=dic, weights=wts)
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max()


def test_reweighting_improves_a_sparse_reconstruction():
    """Property, not a printed value: reweighted SARA beats a single unweighted round."""
    N, M = 32, 700
    s = Setup(N=N, L=synth.fov_L())
    rng = np.random.default_rng(35)
    u, v, w = synth.uvw(N, M, s.L, "uniform", 0.0, N / (2 * s.L ** 2), rng)
    G = wproj.build_rows(u, v, w, 0.99, s)
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    x = synth.sky(N, 3, 6, np.random.default_rng(36))
    y0 = A(x)
    sig = metrics.noise_sigma(y0, 30.0)
    y = y0 + synth.noise(M, sig, np.random.default_rng(37))
    eps = metrics.l2_ball_radius(sig, M)
    nu = solver.power_norm2(A, AH, np.random.default_rng(38).normal(size=(N, N)), 40)
    x1, w1 = sara.solve(y, A, AH, (N, N), eps, nu, 150, rounds=1, levels=3)
    x3, w3 = sara.solve(y, A, AH, (N, N), eps, nu, 150, rounds=3, levels=3)
    assert w1 is None and w3.shape == (9, N, N) and np.all((w3 > 0) & (w3 <= 1))
    assert metrics.snr_out(x, x3) > metrics.snr_out(x, x1)
