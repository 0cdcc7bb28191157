"""Coordinates of the image, the padded image and the oversampled uv grid.

Test infrastructure (see the package header).

Discretisation (Section 2.2 recast for continuous visibilities):

* the N x N image covers the planar field of view L (Section 4.1), pixel
  size delta = L / N, pixel p in [0, N) sits at l_p = (p - N/2) delta;
* the image is zero-padded to Ng = sigma N pixels (sigma = 2) with the same
  pixel size; padded pixel j sits at l_j = (j - Ng/2) delta, so image pixel p
  is padded pixel j = p + (Ng - N)/2;
* the uv grid is the centred DFT of the padded image: cell q in [0, Ng) sits
  at u = (q - Ng/2) du with du = 1 / (Ng delta);
* a visibility at u (wavelengths) has grid coordinate u~ = u / du, and the
  grid spans u~ in [-Ng/2, Ng/2), i.e. u in [-B, B) with B = N / (2L).

Arrays are indexed [m, l] (first axis along v / m, second along u / l); a
flattened grid index is q_v * Ng + q_u.
"""
from __future__ import annotations

import numpy as np


def pixel_size(N: int, L: float) -> float:
    return L / N


def padded_size(N: int, sigma: float = 2.0) -> int:
    Ng = int(round(sigma * N))
    if Ng % 2:
        raise ValueError("padded grid size must be even")
    return Ng


def cell_size(N: int, L: float, sigma: float = 2.0) -> float:
    """du = 1 / (Ng delta) in wavelengths."""
    return 1.0 / (padded_size(N, sigma) * pixel_size(N, L))


def image_coords(N: int, L: float) -> np.ndarray:
    """l_p = (p - N/2) delta for p in [0, N)."""
    return (np.arange(N) - N / 2) * pixel_size(N, L)


def padded_coords(N: int, L: float, sigma: float = 2.0) -> np.ndarray:
    """l_j = (j - Ng/2) delta for j in [0, Ng)."""
    Ng = padded_size(N, sigma)
    return (np.arange(Ng) - Ng / 2) * pixel_size(N, L)


def grid_coord(u: np.ndarray, N: int, L: float, sigma: float = 2.0) -> np.ndarray:
    """u~ = u / du (centred grid units, in [-Ng/2, Ng/2) inside the band)."""
    return np.asarray(u, dtype=np.float64) / cell_size(N, L, sigma)


def pad_offset(N: int, sigma: float = 2.0) -> int:
    return (padded_size(N, sigma) - N) // 2
