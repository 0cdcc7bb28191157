"""The paper's own on-grid operator Phi' = C-hat F U (Eq. 8), for the sparsity check.

Test infrastructure (see the package header).

Section 3.1 / 3.2 discretisation: visibilities lie on the 2N x 2N uv grid
(no gridding kernel), the image is upsampled twice (U) so the grid of pixels
is Ng = 2N per side over the field L, and each row of C-hat is the shifted,
2-D Fourier transform of the chirp sampled on that grid.  Here the chirp is
sampled at half-pixel-centred positions l_j = (j - Ng/2 + 1/2) L / Ng, and the
transform is divided by Ng^2 (the number of pixels) so that a full row has unit
energy (the w-modulation is a norm-preserving convolution, Section 2.3).

The modulation strength is given as w_d = w L^2 / N (Section 4.1), w_d = 1
being the maximal case.  The non-zero fraction of the sparsified C-hat is
reported in Section 3.2 for w_d ~ U(0, 1): about 20 % at E = 0.999, 7 % at
E = 0.9 and 0.6 % at E = 0.1 of the M x (2N)^2 entries.
"""
from __future__ import annotations

import numpy as np

from .chirp import chirp
from .wproj import energy_threshold


def chirp_row(w_d: float, N: int, L: float, kind: str = "linear") -> np.ndarray:
    """Unit-energy Ng x Ng row (unshifted) of C-hat for modulation w_d."""
    Ng = 2 * N
    l = (np.arange(Ng) - Ng / 2 + 0.5) * (L / Ng)
    w = w_d * N / (L * L)
    c = chirp(l[None, :], l[:, None], w, kind)
    return np.fft.fft2(c) / (Ng * Ng)


def shifted_row(w_d: float, qv: int, qu: int, N: int, L: float, kind: str = "linear") -> np.ndarray:
    """Row of C-hat for a visibility on grid cell (qv, qu): the kernel rolled to that cell."""
    return np.roll(np.roll(chirp_row(w_d, N, L, kind), qv, axis=0), qu, axis=1)


def row_nnz(w_d: float, E: float, N: int, L: float) -> int:
    g = chirp_row(w_d, N, L)
    m = (g * g.conj()).real.ravel()
    tau, _ = energy_threshold(m, E)
    return int(np.count_nonzero(m >= tau))


def nnz_fraction(w_d_samples, E: float, N: int, L: float) -> float:
    Ng = 2 * N
    tot = sum(row_nnz(wd, E, N, L) for wd in w_d_samples)
    return tot / (len(w_d_samples) * Ng * Ng)
