"""CPU check of the separable expansion behind the exact chirp's rows on large grids.

On the padded grid the exact chirp (Eq. 4) is the linear chirp times q(l^2 + m^2),
q(s) = exp(-2 pi i w (sqrt(1 - s) - 1 + s / 2)).  The GPU builder replaces x -> q(x + y) by its
interpolation at 8 Chebyshev points of [0, L^2] (x = l^2, y = m^2).  This test evaluates the
interpolation error at every pair of padded-grid samples (exhaustively, not on a sample) for the grids
and w ranges the builder serves, and asserts it below 1e-9; since |c| = 1, a row's relative error is at
most W (= 4, the gridding window's width) times that by Parseval, far inside the 1e-5 tolerance of the
FP32 operator.  Written from the construction's definition, independently of the GPU code.
"""
import numpy as np
import pytest

import synth

R = 8


def q(s, w):
    return np.exp(1j * np.pi * w * s * s / (1.0 + np.sqrt(1.0 - s)) ** 2)


def max_error(Ng, w, L):
    delta = 2.0 * L / Ng
    t = np.arange(0, Ng // 2 + 1)                 # |t| takes these values on [-Ng/2, Ng/2)
    x = (t * delta) ** 2
    xmax = L * L
    nodes = 0.5 * xmax * (1.0 - np.cos((2 * np.arange(R) + 1) * np.pi / (2 * R)))
    ell = np.ones((R, x.size))
    for i in range(R):
        for j in range(R):
            if j != i:
                ell[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    approx = ell.T @ q(nodes[:, None] + x[None, :], w)           # [x, y]
    exact = q(x[:, None] + x[None, :], w)
    # the linear chirp factors and the identity exp(-2 pi i w (sqrt(1 - s) - 1)) = e^{i pi w s} q(s)
    s = x[:, None] + x[None, :]
    lhs = np.exp(-2j * np.pi * w * (-s / (1.0 + np.sqrt(1.0 - s))))
    assert np.max(np.abs(lhs - np.exp(1j * np.pi * w * s) * exact)) < 1e-9
    return float(np.max(np.abs(approx - exact)))


@pytest.mark.parametrize("N,support", [(512, 64), (1024, 64), (2048, 32), (2048, 64)])
def test_expansion_error_over_every_sample_pair(N, support):
    L = synth.fov_L()
    w = synth.configs.w_for_support(support, 4, L)
    err = max_error(2 * N, w, L)
    assert err < 1e-9, err
    assert 4 * err < 1e-5


def test_expansion_error_up_to_the_widest_window():
    """The builder's window holds rows spreading over up to 88 - 2 (W/2 + 8) - 1 = 67 cells, i.e.
    4 w L^2 / sqrt(1 - 2 L^2) <= 67: the largest w it accepts."""
    L = synth.fov_L()
    w = 67.0 * np.sqrt(1.0 - 2.0 * L * L) / (4.0 * L * L)
    assert max_error(4096, w, L) < 1e-9
