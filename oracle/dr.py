"""Douglas-Rachford splitting for Eq. 7, the solver Section 2.3 names.

Test infrastructure (see the package header).

Eq. 7 as printed: min_x ||Psi^T x||_1 subject to ||y - Phi x||_2 <= eps, x real.  With
f1 = ||Psi^T .||_1 and f2 the indicator of C = {x : ||y - Phi x|| <= eps}, Douglas-Rachford
(Combettes & Pesquet 2007, cited by the paper) iterates, from z = 0,

    x = P_C(z)                          (prox of f2: projection onto C)
    z = z + prox_{gamma f1}(2 x - z) - x

and x converges to a solution.  For an orthonormal Psi (Daubechies 8, or Dirac with levels = 0)
prox_{gamma f1}(r) = Psi soft_gamma(Psi^T r), soft_gamma(a) = sign(a) max(|a| - gamma, 0).

Reading (recorded with the design notes): Phi is not a tight frame here, so P_C has no closed
form; it is computed by forward-backward on its dual, from the previous outer iteration's dual
variable u (zero at the start):

    repeat `inner` times:  p = Phi (z - Re Phi^H u);  u = v - mu P_B(v / mu),  v = u + mu p

with mu = 1 / ||Phi||^2 and P_B the projection onto the ball of radius eps around y; then
P_C(z) = z - Re Phi^H u.  (The same update as the primal-dual solver's second dual variable.)

Pins (tests/test_oracle_dr.py): with Phi = I the projection is the closed-form ball projection;
the solution of Eq. 7 matches the primal-dual solver run without positivity; the returned x meets
the constraint.
"""
from __future__ import annotations

import numpy as np

from .wavelet import dwt2, idwt2


def soft(a: np.ndarray, g: float) -> np.ndarray:
    return np.sign(a) * np.maximum(np.abs(a) - g, 0.0)


def ball(v, y, eps: float):
    r = v - y
    nr = np.linalg.norm(r)
    return v if nr <= eps else y + r * (eps / nr)


def project_constraint(z, y, apply, apply_adj, eps: float, nu: float, inner: int, u=None):
    """(P_C(z), dual u) by dual forward-backward from u (zeros by default)."""
    mu = 1.0 / nu
    u = np.zeros(np.asarray(y).shape, dtype=np.complex128) if u is None else u
    for _ in range(inner):
        v = u + mu * apply(z - np.real(apply_adj(u)))
        u = v - mu * ball(v / mu, y, eps)
    return z - np.real(apply_adj(u)), u


def solve(y, apply, apply_adj, shape, eps: float, nu: float, iters: int, inner: int, gamma: float,
          levels: int = 4):
    z = np.zeros(shape)
    u = None
    x = z
    for _ in range(iters):
        x, u = project_constraint(z, y, apply, apply_adj, eps, nu, inner, u)
        r = 2.0 * x - z
        z = z + idwt2(soft(dwt2(r, levels), gamma), levels) - x
    return x
