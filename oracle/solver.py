"""Constrained l1 reconstruction (Eq. 7) by a primal-dual splitting.

Test infrastructure (see the package header).

Problem (Eq. 7 in its analysis form, which equals the synthesis form for the
orthonormal Daubechies basis; positivity added since skies are non-negative):

    min_x ||Psi^T x||_1   subject to   ||y - Phi x||_2 <= eps,   x >= 0 (real).

The paper names Douglas-Rachford splitting (Section 2.3); any convergent
splitting solves the same problem.  Here: the primal-dual method of Condat
(2013) / Vu (2013) with two dual variables, one per term,

    x+   = max(0, x - tau (Psi v1 + Re Phi^H v2))
    xb   = 2 x+ - x
    v1   = clip(v1 + s1 Psi^T xb, -1, 1)                      (prox of ||.||_1*)
    u    = v2 + s2 Phi xb ;  v2 = u - s2 P_eps(u / s2)        (prox of the ball's conjugate)
    x    = x+

with P_eps(z) = y + (z - y) min(1, eps / ||z - y||), tau = 0.49, s1 = 1,
s2 = 1 / ||Phi||^2 (so tau (s1 ||Psi||^2 + s2 ||Phi||^2) = 0.98 < 1), zero
start.  ||Phi||^2 comes from power iteration on Phi^H Phi from a given start
vector.

levels = 0 takes the Dirac basis Psi = I (Section 4.2), levels >= 1 the
Daubechies-8 wavelets with that many levels.

Residual image (Section 4.2): the difference of the dirty images of the
reconstruction and of the original, x_res = Phi^H Phi x_rec - Phi^H Phi x
(real part, the image domain is real).

Pins (tests/test_oracle_solver.py): noiseless full coverage converges (SNR
rises past 40 dB), the returned image satisfies the constraint, and the
Dirac basis with Phi = I against its closed form (soft thresholding of y at
the level where the residual norm equals eps).  Parity unpinned against the
paper's printed SNRs (they need its test images).
"""
from __future__ import annotations

import numpy as np

from .wavelet import dwt2, idwt2


def power_norm2(apply, apply_adj, x0: np.ndarray, iters: int = 50) -> float:
    """||Phi||^2 by power iteration on Phi^H Phi (real image domain)."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        z = np.real(apply_adj(apply(x)))
        lam = float(np.linalg.norm(z))
        x = z / lam
    return lam


def project_ball(z: np.ndarray, y: np.ndarray, eps: float) -> np.ndarray:
    r = z - y
    nr = np.linalg.norm(r)
    if nr <= eps:
        return z
    return y + r * (eps / nr)


def solve(y, apply, apply_adj, shape, eps: float, nu: float, iters: int,
          levels: int = 4, tau: float = 0.49, history: bool = False, x_true=None,
          dictionary=None, weights=None, x0=None, positive: bool = True):
    """Returns x (and the SNR history against x_true when asked).

    dictionary: optional (analysis, synthesis) pair replacing the wavelets of `levels`
    (it must satisfy ||Psi|| <= 1, as a tight frame normalised to 1 does); weights: optional
    non-negative array shaped like the coefficients, the weighted norm ||W Psi^T x||_1 (the
    prox of its conjugate clips coefficient i to [-w_i, w_i]); x0: start (zeros by default);
    positive=False drops the positivity constraint (Eq. 7 as printed).
    """
    if dictionary is None:
        analysis, synthesis = (lambda z: dwt2(z, levels)), (lambda c: idwt2(c, levels))
    else:
        analysis, synthesis = dictionary
    s1 = 1.0
    s2 = 1.0 / nu
    x = np.zeros(shape) if x0 is None else np.array(x0, dtype=np.float64)
    v1 = np.zeros_like(analysis(np.zeros(shape)))
    bound = 1.0 if weights is None else np.asarray(weights, dtype=np.float64)
    v2 = np.zeros(np.asarray(y).shape, dtype=np.complex128)
    hist = []
    for _ in range(iters):
        xn = x - tau * (synthesis(v1) + np.real(apply_adj(v2)))
        if positive:
            xn = np.maximum(0.0, xn)
        xb = 2.0 * xn - x
        v1 = np.clip(v1 + s1 * analysis(xb), -bound, bound)
        u = v2 + s2 * apply(xb)
        v2 = u - s2 * project_ball(u / s2, y, eps)
        x = xn
        if history and x_true is not None:
            from .metrics import snr_out
            hist.append(snr_out(x_true, x))
    return (x, hist) if history else x


def residual_image(apply, apply_adj, x_rec: np.ndarray, x_true: np.ndarray) -> np.ndarray:
    """x_res = Re Phi^H Phi x_rec - Re Phi^H Phi x_true (Section 4.2)."""
    return np.real(apply_adj(apply(x_rec))) - np.real(apply_adj(apply(x_true)))
