"""SARA: sparsity averaging over several wavelet bases with reweighted l1 (Section 4.2).

Test infrastructure (see the package header).

Section 4.2 reconstructs with a third dictionary beside Dirac and Daubechies 8:
SARA (Carrillo, McEwen & Wiaux 2012), which the paper cites without restating.
Reading taken here (recorded with the design notes):

* dictionary: the concatenation of q = 9 orthonormal bases, the Dirac basis and
  the Daubechies wavelets with 1 to 8 vanishing moments (periodic, `levels`
  levels each), scaled by 1 / sqrt(q):
      Psi^T x = (x, W_1 x, ..., W_8 x) / 3,   Psi c = (c_0 + sum_p W_p^T c_p) / 3,
  a tight frame with Psi Psi^T = I, so ||Psi|| = 1 and the solver's step sizes
  stay valid;
* reweighting: `rounds` solves of Eq. 7 with the weighted analysis norm
  ||W Psi^T x||_1 (same constraint and positivity).  Round 0 has unit weights;
  before round r >= 1 the weights are w_i = delta_r / (delta_r + |alpha_i|),
  alpha = Psi^T x of the previous round, delta_1 = the standard deviation of
  alpha and delta_(r+1) = delta_r / 10.  Each round starts from the previous
  estimate with its dual variables at zero.

Pins (tests/test_oracle_sara.py): Psi Psi^T = I and Psi^T is an isometry; Haar
against its closed form; with one basis and unit weights the solve equals the
plain solver; weighted soft thresholding (Phi = I, Dirac basis) against its
closed form.
"""
from __future__ import annotations

import numpy as np

from . import solver
from .wavelet import dwt2, idwt2

Q = 9                      # Dirac + Daubechies 1..8
SCALE = 1.0 / 3.0          # 1 / sqrt(Q)


def analysis(x: np.ndarray, levels: int = 4) -> np.ndarray:
    """Coefficients [Q, N, N] of Psi^T x."""
    x = np.asarray(x, dtype=np.float64)
    return SCALE * np.stack([x] + [dwt2(x, levels, p) for p in range(1, 9)])


def synthesis(c: np.ndarray, levels: int = 4) -> np.ndarray:
    """Image Psi c of coefficients [Q, N, N]."""
    c = np.asarray(c, dtype=np.float64)
    return SCALE * (c[0] + sum(idwt2(c[p], levels, p) for p in range(1, 9)))


def weights(alpha: np.ndarray, delta: float) -> np.ndarray:
    return delta / (delta + np.abs(alpha))


def solve(y, apply, apply_adj, shape, eps: float, nu: float, iters: int, rounds: int,
          levels: int = 4, tau: float = 0.49):
    """Reweighted analysis over the SARA dictionary; returns (x, the weights of the last round)."""
    dic = (lambda z: analysis(z, levels), lambda c: synthesis(c, levels))
    x = np.zeros(shape)
    w = None
    delta = None
    for r in range(rounds):
        if r >= 1:
            alpha = analysis(x, levels)
            delta = float(np.std(alpha)) if r == 1 else delta / 10.0
            w = weights(alpha, delta)
        x = solver.solve(y, apply, apply_adj, shape, eps, nu, iters, tau=tau, dictionary=dic,
                         weights=w, x0=x)
    return x, w
