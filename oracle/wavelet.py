"""Daubechies-8 wavelets (periodic, orthonormal) for the sparsity dictionary.

Test infrastructure (see the package header).

Section 4.2 uses Daubechies 8 wavelets as the sparsity basis Psi of Eq. 7.
"Daubechies 8" is read as the filter with 8 vanishing moments (16 taps).

Filter: Daubechies' spectral factorisation.  With p vanishing moments the
low-pass filter satisfies |m0|^2 = cos^(2p)(xi/2) Q(sin^2(xi/2)),
Q(y) = sum_{k<p} binom(p-1+k, k) y^k.  Each root y_i of Q gives the pair of
z-roots of (2 - z - 1/z)/4 = y_i; the minimum-phase filter keeps the root
inside the unit circle.  h has zeros at -1 (p-fold) and at those roots, read
as h_0 z^(L-1) + ... + h_(L-1), scaled so sum h = sqrt(2).  High-pass
g_n = (-1)^n h_(L-1-n).

Transform: one level along an axis of even length n maps x to
a_k = sum_n h_n x_((2k+n) mod n), d_k = sum_n g_n x_((2k+n) mod n), stored
[a | d].  2-D: rows (last axis) then columns, recursing on the top-left
approximation block.  The transform is orthonormal, so the synthesis is its
transpose.

Dirac basis: zero levels is the identity, Psi = I (the pixel basis that
Section 2.3 names as maximally incoherent with the Fourier basis and that
Section 4.2 uses beside Daubechies 8).

Pins (tests/test_oracle_wavelet.py): sum h = sqrt(2), sum h^2 = 1, even-shift
orthogonality, 8 vanishing moments of g, perfect reconstruction, db2 against
its closed form (1 + sqrt 3, 3 + sqrt 3, 3 - sqrt 3, 1 - sqrt 3) / (4 sqrt 2).
"""
from __future__ import annotations

from math import comb

import numpy as np


def daubechies_lowpass(p: int = 8) -> np.ndarray:
    q = [comb(p - 1 + k, k) for k in range(p)]          # Q(y) coefficients, ascending
    yroots = np.roots(q[::-1]) if p > 1 else np.array([])
    zroots = []
    for y in yroots:
        b = 1.0 - 2.0 * y                                # z^2 - 2 b z + 1 = 0
        d = np.sqrt(b * b - 1.0 + 0j)
        z1, z2 = b + d, b - d
        zroots.append(z1 if abs(z1) < 1.0 else z2)
    roots = np.concatenate([-np.ones(p), np.asarray(zroots, dtype=complex)])
    h = np.real(np.poly(roots))
    return h * (np.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    n = np.arange(h.size)
    return ((-1.0) ** n) * h[::-1]


def _analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    x = np.moveaxis(x, axis, -1)
    n = x.shape[-1]
    k = np.arange(n // 2)
    idx = (2 * k[:, None] + np.arange(h.size)[None, :]) % n      # [n/2, taps]
    seg = x[..., idx]
    a = seg @ h
    d = seg @ g
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def _synthesis_1d(c: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    c = np.moveaxis(c, axis, -1)
    n = c.shape[-1]
    a, d = c[..., : n // 2], c[..., n // 2:]
    out = np.zeros(c.shape, dtype=np.result_type(c, h))
    k = np.arange(n // 2)
    for t in range(h.size):
        pos = (2 * k + t) % n
        np.add.at(out, (..., pos), a * h[t] + d * g[t])
    return np.moveaxis(out, -1, axis)


def dwt2(x: np.ndarray, levels: int = 4, p: int = 8) -> np.ndarray:
    """Coefficients Psi^T x (same shape as x)."""
    h = daubechies_lowpass(p)
    g = highpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    n = c.shape[0]
    for _ in range(levels):
        blk = c[:n, :n]
        blk = _analysis_1d(blk, h, g, axis=1)
        blk = _analysis_1d(blk, h, g, axis=0)
        c[:n, :n] = blk
        n //= 2
    return c


def idwt2(c: np.ndarray, levels: int = 4, p: int = 8) -> np.ndarray:
    """Image Psi c."""
    h = daubechies_lowpass(p)
    g = highpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    if levels == 0:
        return x
    n = x.shape[0] >> (levels - 1)
    for _ in range(levels):
        blk = x[:n, :n]
        blk = _synthesis_1d(blk, h, g, axis=0)
        blk = _synthesis_1d(blk, h, g, axis=1)
        x[:n, :n] = blk
        n *= 2
    return x
