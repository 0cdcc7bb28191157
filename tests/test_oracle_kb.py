"""Pins of the oracle's Kaiser-Bessel window (CPU only)."""
import warnings

import numpy as np
import pytest
from scipy import integrate

from oracle import kb


@pytest.mark.parametrize("W", [4, 6, 8])
@pytest.mark.parametrize("xi", [0.0, 0.05, 0.13, 0.25, 0.37, 0.5, 0.9, 1.3])
@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_kb_ft_closed_form_matches_quadrature(W, xi):
    beta = kb.beatty_beta(W, 2.0)
    f = lambda t: kb.kb(np.array([t]), W, beta)[0] * np.cos(2 * np.pi * xi * t)
    val, err = integrate.quad(f, -W / 2, W / 2, limit=400, epsabs=1e-13, epsrel=1e-13, points=[0.0])
    scale = kb.kb_ft(np.array([0.0]), W, beta)[0]       # integral of |KB|: the cancellation scale
    assert abs(kb.kb_ft(np.array([xi]), W, beta)[0] - val) <= 1e-12 * scale


def test_kb_window_support_and_edges():
    W, beta = 4, kb.beatty_beta(4)
    t = np.array([-2.0, -1.0, 0.0, 1.0, 2.0, 2.0001])
    v = kb.kb(t, W, beta)
    assert v[-1] == 0.0
    assert v[0] == pytest.approx(1.0) and v[4] == pytest.approx(1.0)   # I0(0) at the edge
    assert np.all(np.diff(v[:3]) > 0) and v[2] == v.max()


@pytest.mark.parametrize("ut", [-3.0, -2.5, 0.0, 0.3, 17.999, -255.2])
def test_kb_taps_cover_the_window(ut):
    W = 4
    q, wt = kb.kb_taps(ut, W, kb.beatty_beta(W))
    d = ut - q
    assert q.size == W and np.all(np.diff(q) == 1)
    assert np.all(d >= -W / 2) and np.all(d < W / 2)
    assert np.all(wt > 0)


def test_beta_increases_with_support():
    b = [kb.beatty_beta(W) for W in (4, 6, 8, 10)]
    assert all(x < y for x, y in zip(b, b[1:]))
