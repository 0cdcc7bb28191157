"""Pins of the oracle's Daubechies wavelets (CPU only)."""
import numpy as np
import pytest

from oracle import wavelet


def test_db2_matches_closed_form():
    s3 = np.sqrt(3.0)
    closed = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    assert np.abs(wavelet.daubechies_lowpass(2) - closed).max() < 1e-14


@pytest.mark.parametrize("p", [2, 4, 8])
def test_filter_conditions(p):
    h = wavelet.daubechies_lowpass(p)
    g = wavelet.highpass(h)
    assert h.size == 2 * p
    assert abs(h.sum() - np.sqrt(2)) < 1e-13 and abs(np.dot(h, h) - 1) < 1e-13
    for k in range(1, p):
        assert abs(np.dot(h[2 * k:], h[:-2 * k])) < 1e-13
    n = np.arange(h.size, dtype=float)
    n /= n.max()
    for k in range(p):
        assert abs(np.sum(g * n ** k)) < 1e-10
    assert abs(np.sum(g * n ** p)) > 1e-8       # exactly p vanishing moments


def test_minimum_phase():
    h = wavelet.daubechies_lowpass(8)
    z = np.roots(h)
    near = np.abs(z + 1) < 0.1            # the 8-fold zero at -1 (numerically split)
    assert np.count_nonzero(near) == 8
    assert np.all(np.abs(z[~near]) < 1)


@pytest.mark.parametrize("N,levels", [(64, 4), (32, 2), (256, 4)])
def test_perfect_reconstruction_and_orthonormality(N, levels):
    x = np.random.default_rng(N).normal(size=(N, N))
    c = wavelet.dwt2(x, levels)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-11 * np.linalg.norm(x)
    assert np.abs(wavelet.idwt2(c, levels) - x).max() < 1e-12
    y = np.random.default_rng(N + 1).normal(size=(N, N))
    assert abs(np.sum(wavelet.dwt2(y, levels) * c) - np.sum(y * x)) < 1e-10 * N * N


def test_smooth_image_is_compressible():
    N = 64
    i, j = np.mgrid[0:N, 0:N]
    x = np.exp(-((i - 30.3) ** 2 + (j - 20.7) ** 2) / 50.0)
    c = np.sort(np.abs(wavelet.dwt2(x, 4)).ravel())[::-1]
    assert np.sum(c[:400] ** 2) > (1 - 1e-7) * np.sum(c ** 2)      # 10 % of the coefficients
