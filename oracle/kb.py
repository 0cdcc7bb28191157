"""Kaiser-Bessel gridding window and its Fourier transform.

Test infrastructure (see the package header).

The paper leaves out the gridding operator for continuous visibilities
(Section 2.2, and the conclusions defer continuous (u, v) to later work).  The
continuous-(u, v) operator Phi = G F Z A interpolates the oversampled grid
with a Kaiser-Bessel window of W cells and corrects the taper in the image
(the apodisation A).  Definitions used here:

* window   KB(t) = I0(beta sqrt(1 - (2t/W)^2)) for |t| <= W/2, else 0
* shape    beta = pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8)
           (Beatty, Nishimura & Pauly 2005, for oversampling sigma)
* FT       g(xi) = int KB(t) exp(-2 pi i xi t) dt
                 = W sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(beta^2 - (pi W xi)^2)
           (sin form when the radicand is negative)
* taps     a visibility at grid coordinate u~ uses the W cells q' (centred
           integers) with u~ - q' in [-W/2, W/2): q' = floor(u~) - W/2 + 1 + i,
           i = 0 .. W-1.

Pins: the FT closed form is checked against numerical quadrature of the window
(tests/test_oracle_kb.py); I0 is SciPy's.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def beatty_beta(W: int, sigma: float = 2.0) -> float:
    return float(np.pi * np.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8))


def kb(t, W: int, beta: float) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    r = 1.0 - (2.0 * t / W) ** 2
    out = np.zeros_like(t)
    inside = r >= 0.0
    out[inside] = special.i0(beta * np.sqrt(r[inside]))
    return out


def kb_ft(xi, W: int, beta: float) -> np.ndarray:
    xi = np.asarray(xi, dtype=np.float64)
    z = beta ** 2 - (np.pi * W * xi) ** 2
    out = np.empty_like(xi)
    pos = z > 0
    s = np.sqrt(z[pos])
    out[pos] = W * np.sinh(s) / s
    neg = z < 0
    s = np.sqrt(-z[neg])
    out[neg] = W * np.sin(s) / s
    out[z == 0] = W
    return out


def kb_taps(ut: float, W: int, beta: float):
    """Centred cell indices q' and weights KB(u~ - q') of one visibility."""
    base = int(np.floor(ut)) - W // 2 + 1
    q = base + np.arange(W)
    return q, kb(ut - q, W, beta)
