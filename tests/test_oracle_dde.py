"""Pins of the oracle's direction-dependent effect (a Gaussian power pattern per visibility) through
the sparse w-projection rows (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import dft, geometry, wproj
from oracle.wproj import Setup

L = synth.fov_L()


def _beams(M, seed, L):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-0.2, 0.2, M) * L, rng.uniform(-0.2, 0.2, M) * L,
                     rng.uniform(0.3, 0.8, M) * L], axis=1)


@pytest.mark.parametrize("kind", ["linear", "exact"])
def test_phi_with_beam_converges_to_direct_sum(kind):
    N, M = 16, 20
    u, v, w = synth.uvw(N, M, L, "uniform", 0.25, N / (2 * L * L), np.random.default_rng(41))
    beam = _beams(M, 42, L)
    x = synth.random_complex((N, N), np.random.default_rng(43))
    yd = dft.measure(x, u, v, w, N, L, kind=kind, beam=beam)
    errs = []
    for W in (4, 6, 8):
        s = Setup(N=N, L=L, W=W, kind=kind)
        G = wproj.build_rows(u, v, w, 1.0, s, beam=beam)
        errs.append(np.linalg.norm(wproj.phi(G, x, s) - yd) / np.linalg.norm(yd))
    assert errs[0] < 3e-3
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20
    assert errs[2] < 1e-6
    # the beam matters: without it the operator misses the direct sum by far more
    G0 = wproj.build_rows(u, v, w, 1.0, Setup(N=N, L=L, W=8, kind=kind))
    assert np.linalg.norm(wproj.phi(G0, x, Setup(N=N, L=L, W=8, kind=kind)) - yd) / np.linalg.norm(yd) > 0.1


def test_beam_spectrum_at_w_zero_is_a_product_of_sampled_gaussian_spectra():
    """w = 0: H is the 2-D DFT of the sampled Gaussian, by Poisson summation
    Ng^-1 sum_t exp(-(t delta - a)^2 / (2 s^2)) e^(-2 pi i t d / Ng)
      = (s sqrt(2 pi) / (Ng delta)) exp(-2 pi^2 s^2 f^2) exp(-2 pi i a f),  f = d / (Ng delta),
    up to terms below 1e-12 here (the pattern is 7 sigma inside the padded field)."""
    N = 32
    s = Setup(N=N, L=L)
    l0, m0, sg = 0.05 * L, -0.04 * L, L / 8
    H = wproj.chirp_spectrum_2d(0.0, s, beam=(l0, m0, sg))
    d = np.fft.fftfreq(s.Ng, 1.0 / s.Ng)          # d mod Ng as signed integers
    f = d / (s.Ng * s.delta)
    g = lambda a: sg * np.sqrt(2 * np.pi) / (s.Ng * s.delta) * np.exp(-2 * np.pi ** 2 * sg ** 2 * f ** 2) \
        * np.exp(-2j * np.pi * a * f)
    want = np.outer(g(m0), g(l0))
    assert np.abs(H - want).max() < 1e-12 * np.abs(want).max()


def test_wide_beam_gives_back_the_plain_rows():
    N, M = 16, 12
    s = Setup(N=N, L=L, kind="exact")
    u, v, w = synth.uvw(N, M, L, "uniform", 0.25, N / (2 * L * L), np.random.default_rng(44))
    beam = np.tile([0.0, 0.0, 1e6], (M, 1))
    G1 = wproj.build_rows(u, v, w, 0.99, s, beam=beam)
    G0 = wproj.build_rows(u, v, w, 0.99, s)
    assert np.array_equal(G1.indices, G0.indices)
    assert np.abs(G1.data - G0.data).max() < 1e-9 * np.abs(G0.data).max()
