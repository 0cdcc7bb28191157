"""Brute-force evaluation of the discretised measurement equation.

Test infrastructure (see the package header).

Eq. 1 / Eq. 3 on the pixel grid, with the primary beam absorbed into the sky
(Section 2.1):

    y_k = sum_p x_p a_phys(p) exp(-2 pi i (u_k l_p + v_k m_p)) C(l_p, m_p; w_k)

where C is the exact w-modulation (Eq. 4) or the linear chirp (Eq. 5), and
a_phys is 1 or 1/n(l, m); with a direction-dependent effect (oracle.dde) C is
multiplied by the visibility's beam A_k(l, m).  Cost O(M N^2) (Section 3.2's complexity of the
direct approach).  This is the definition the sparse operator approaches at
E = 1 as the KB support W grows.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from .chirp import chirp
from .dde import gaussian_beam


def _phys(l, m, a_phys):
    if a_phys == "one":
        return np.ones_like(l)
    if a_phys == "inv_n":
        return 1.0 / np.sqrt(1.0 - l * l - m * m)
    raise ValueError(a_phys)


def measure(x, u, v, w, N: int, L: float, kind: str = "linear", a_phys: str = "one",
            chunk: int = 64, beam=None) -> np.ndarray:
    """beam: optional [M, 3] per-visibility Gaussian power patterns (l0, m0, sigma), oracle.dde."""
    x = np.asarray(x, dtype=np.complex128)
    lp = geo.image_coords(N, L)
    l = np.broadcast_to(lp[None, :], (N, N)).ravel()
    m = np.broadcast_to(lp[:, None], (N, N)).ravel()
    xa = x.ravel() * _phys(l, m, a_phys)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    y = np.empty(u.size, dtype=np.complex128)
    for s in range(0, u.size, chunk):
        e = slice(s, s + chunk)
        ph = np.exp(-2j * np.pi * (u[e, None] * l[None, :] + v[e, None] * m[None, :]))
        C = np.stack([chirp(l, m, wk, kind) for wk in w[e]])
        if beam is not None:
            C = C * np.stack([gaussian_beam(l, m, *b) for b in np.asarray(beam)[e]])
        y[e] = (ph * C) @ xa
    return y


def measure_adjoint(y, u, v, w, N: int, L: float, kind: str = "linear", a_phys: str = "one",
                    chunk: int = 64) -> np.ndarray:
    lp = geo.image_coords(N, L)
    l = np.broadcast_to(lp[None, :], (N, N)).ravel()
    m = np.broadcast_to(lp[:, None], (N, N)).ravel()
    y = np.asarray(y, dtype=np.complex128)
    out = np.zeros(N * N, dtype=np.complex128)
    for s in range(0, y.size, chunk):
        e = slice(s, s + chunk)
        ph = np.exp(-2j * np.pi * (np.asarray(u)[e, None] * l[None, :] + np.asarray(v)[e, None] * m[None, :]))
        C = np.stack([chirp(l, m, wk, kind) for wk in np.asarray(w)[e]])
        out += (ph * C).conj().T @ y[e]
    return (out * _phys(l, m, a_phys)).reshape(N, N)
