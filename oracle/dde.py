"""A direction-dependent effect beside w, through the same sparsifier (Section 3.2).

Test infrastructure (see the package header).

Section 3.2 notes that the per-row energy threshold assumes nothing about a
row's structure, so any direction-dependent effect (DDE) multiplied into the
w-modulation kernel is sparsified the same way.  The DDE taken here (a reading,
recorded with the design notes) is a per-visibility Gaussian antenna power
pattern with a pointing offset,

    A_k(l, m) = exp(-((l - l0_k)^2 + (m - m0_k)^2) / (2 sigma_k^2)),

so visibility k measures sum_p x_p A_k(l_p, m_p) C(l_p, m_p; w_k) exp(-2 pi i (u_k l_p + v_k m_p))
and row k of G is built from the modulation A_k C instead of C.

Pins (tests/test_oracle_dde.py): the operator approaches this direct sum as the
KB support grows; at w = 0 the row spectrum is the product of two sampled
Gaussians' spectra in closed form (Poisson summation); a very wide beam gives
back the rows without it.
"""
from __future__ import annotations

import numpy as np


def gaussian_beam(l, m, l0: float, m0: float, sigma: float) -> np.ndarray:
    l = np.asarray(l, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    return np.exp(-((l - l0) ** 2 + (m - m0) ** 2) / (2.0 * sigma * sigma))
