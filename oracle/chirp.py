"""The w-modulation of the measurement equation.

Test infrastructure (see the package header).

* Exact form (Eq. 4): C(l, m; w) = exp(-2 pi i w (sqrt(1 - l^2 - m^2) - 1)).
* Linear chirp (Eq. 5), the paper's working approximation: first order of
  Eq. 4 in r^2 = l^2 + m^2.  Since sqrt(1 - r^2) - 1 = -r^2/2 + O(r^4), the
  first-order term is exp(+i pi w r^2).  Eq. 5 prints the opposite sign; we
  take the sign of the expansion (reading recorded with the design notes) so
  that the linear and exact forms agree to first order.  Kernel magnitudes,
  and therefore the sparsity pattern, are the same under either sign.

Pins: the 1-D discrete chirp spectrum matches the quadratic Gauss sum in closed
form at w delta^2 Ng = 1; the linear and exact forms differ by O(w r^4);
constant-w modulation in the image equals convolution by the chirp spectrum
in uv (tests/test_oracle_wproj.py).
"""
from __future__ import annotations

import numpy as np

LINEAR = "linear"
EXACT = "exact"


def chirp(l, m, w: float, kind: str = LINEAR) -> np.ndarray:
    l = np.asarray(l, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    r2 = l * l + m * m
    if kind == LINEAR:
        return np.exp(1j * np.pi * w * r2)
    if kind == EXACT:
        # sqrt(1 - r^2) - 1 written as -r^2 / (1 + sqrt(1 - r^2)) to avoid cancellation
        return np.exp(-2j * np.pi * w * (-r2 / (1.0 + np.sqrt(1.0 - r2))))
    raise ValueError(kind)


def chirp_1d(l, w: float) -> np.ndarray:
    """One separable factor of the linear chirp: exp(i pi w l^2)."""
    l = np.asarray(l, dtype=np.float64)
    return np.exp(1j * np.pi * w * l * l)
