"""Sparse w-projection operator Phi = G F Z A and its adjoint, in FP64.

Test infrastructure (see the package header).

Method (Section 3 of the paper, generalised to continuous (u, v) with a
Kaiser-Bessel gridding window):

1. A, Z   multiply the image by the apodisation a = a_phys / (g(xi_l) g(xi_m))
          (g = FT of the KB window, xi = pixel offset / Ng) and zero-pad it to
          the Ng x Ng grid (Section 2.2's upsampling U, in the image domain).
2. F      centred, unnormalised 2-D DFT: X[q] = sum_j z_j exp(-2 pi i (j-c).(q-c)/Ng),
          c = Ng/2 (Eq. 6).
3. G      one row per measured visibility (the mask M of Eq. 6 folded into the
          rows, Eq. 8).  Row k is the visibility's KB taps convolved with the
          Fourier transform of its own chirp (Section 3.1: the w-modulation is
          computed in real space, Fourier transformed, and the result is one
          shifted row of C-hat):
              H_k(d) = Ng^-2 sum_t c_k(l_t) exp(-2 pi i t.d / Ng)
              g_k(q) = sum_q' KB(u~_k - q'_u) KB(v~_k - q'_v) H_k(q' - q)
          (indices modulo Ng).  This is exact: sum_q g_k(q) X[q] equals KB
          interpolation of F(z * c_k) at (u~_k, v~_k).
4. sparsify  keep, per row, the largest |g_k|^2 entries holding a fraction E
          of the row's energy sum |g_k|^2 (Section 3.2): take the energies in
          decreasing order, find the first position where the running sum
          reaches E times the total, take that entry's energy as the threshold
          tau and keep every entry >= tau (ties kept); E >= 1 keeps every
          non-zero entry.  No renormalisation.  The paper reaches tau by
          bisection; the ordered running sum gives the same threshold.
5. CSR    kept entries of each row in ascending flattened column q_v*Ng + q_u.

Adjoint: Phi^H = A Z^H F^H G^H with F^H the unnormalised inverse DFT.

For the linear chirp both the window and the chirp are separable, so
g_k = g_v (outer) g_u with 1-D factors built from the 1-D chirp spectrum
(h(d) = Ng^-1 sum_t exp(i pi w delta^2 t^2) exp(-2 pi i t d / Ng)).  The
2-D form is kept for the exact chirp and as a cross-check.

Pins (tests/test_oracle_wproj.py): direct DFT of the measurement equation
(error falls geometrically with W), adjoint identity to 1e-12, w = 0 gives
pure KB gridding, constant w equals image-domain modulation, quadratic Gauss
sum, separable == 2-D form, kept energy >= E, nnz monotone in E and w.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.sparse as sp

from . import geometry as geo
from .chirp import LINEAR, EXACT, chirp, chirp_1d
from .dde import gaussian_beam
from .kb import beatty_beta, kb, kb_ft, kb_taps


@dataclass(frozen=True)
class Setup:
    N: int
    L: float
    W: int = 4
    beta: float = None
    sigma: float = 2.0
    kind: str = LINEAR
    a_phys: str = "one"      # "one" (primary beam absorbed, Section 2.1) or "inv_n" (1/n of Eq. 1)

    def __post_init__(self):
        if self.beta is None:
            object.__setattr__(self, "beta", beatty_beta(self.W, self.sigma))

    @property
    def Ng(self) -> int:
        return geo.padded_size(self.N, self.sigma)

    @property
    def delta(self) -> float:
        return geo.pixel_size(self.N, self.L)


# ----------------------------------------------------------------------------- A, Z, F

def apodisation(s: Setup) -> np.ndarray:
    """a[i_m, i_l] = a_phys(l, m) / (g(xi_l) g(xi_m)), real N x N."""
    off = (np.arange(s.N) - s.N / 2) / s.Ng
    gh = kb_ft(off, s.W, s.beta)
    a = 1.0 / np.outer(gh, gh)
    if s.a_phys == "inv_n":
        l = geo.image_coords(s.N, s.L)
        r2 = l[None, :] ** 2 + l[:, None] ** 2
        a = a / np.sqrt(1.0 - r2)
    elif s.a_phys != "one":
        raise ValueError(s.a_phys)
    return a


def centred_fft2(z: np.ndarray) -> np.ndarray:
    """Centred unnormalised 2-D DFT (scipy.fft over every host thread; the same transform as numpy.fft)."""
    return np.fft.fftshift(scipy.fft.fft2(np.fft.ifftshift(z), workers=-1))


def centred_fft2_adjoint(X: np.ndarray) -> np.ndarray:
    """Exact adjoint of centred_fft2 (unnormalised inverse)."""
    n = X.shape[0] * X.shape[1]
    return n * np.fft.fftshift(scipy.fft.ifft2(np.fft.ifftshift(X), workers=-1))


def grid_forward(x: np.ndarray, s: Setup) -> np.ndarray:
    """X = F Z A x on the Ng x Ng grid."""
    z = np.zeros((s.Ng, s.Ng), dtype=np.complex128)
    o = geo.pad_offset(s.N, s.sigma)
    z[o:o + s.N, o:o + s.N] = np.asarray(x, dtype=np.complex128) * apodisation(s)
    return centred_fft2(z)


def grid_adjoint(X: np.ndarray, s: Setup) -> np.ndarray:
    """x = A Z^H F^H X (complex N x N)."""
    z = centred_fft2_adjoint(X)
    o = geo.pad_offset(s.N, s.sigma)
    return z[o:o + s.N, o:o + s.N] * apodisation(s)


# ----------------------------------------------------------------------------- kernel rows

def chirp_spectrum_1d(w: float, s: Setup) -> np.ndarray:
    """h[d mod Ng] = Ng^-1 sum_t exp(i pi w (t delta)^2) exp(-2 pi i t d / Ng)."""
    t = np.arange(s.Ng) - s.Ng // 2
    c = chirp_1d(t * s.delta, w)
    return np.fft.fft(np.fft.ifftshift(c)) / s.Ng


def chirp_spectrum_2d(w: float, s: Setup, beam=None) -> np.ndarray:
    """H[d_v mod Ng, d_u mod Ng] = Ng^-2 sum_t c(l_t, m_t) exp(-2 pi i t.d / Ng).

    beam: optional (l0, m0, sigma) of a Gaussian power pattern multiplied into c (oracle.dde).
    """
    l = geo.padded_coords(s.N, s.L, s.sigma)
    c = chirp(l[None, :], l[:, None], w, s.kind)
    if beam is not None:
        c = c * gaussian_beam(l[None, :], l[:, None], *beam)
    return np.fft.fft2(np.fft.ifftshift(c)) / (s.Ng * s.Ng)


def _taps(ut: float, s: Setup):
    qc, wt = kb_taps(ut, s.W, s.beta)
    return qc + s.Ng // 2, wt          # grid indices (may lie outside [0, Ng): taken mod Ng)


def row_factor_1d(ut: float, h: np.ndarray, s: Setup) -> np.ndarray:
    """g(q) = sum_i KB(u~ - q'_i) h((q'_i - q) mod Ng), q in [0, Ng)."""
    q = np.arange(s.Ng)
    g = np.zeros(s.Ng, dtype=np.complex128)
    for qp, wt in zip(*_taps(ut, s)):
        g += wt * h[(qp - q) % s.Ng]
    return g


def kernel_row_separable(ut: float, vt: float, w: float, s: Setup):
    """(g_v, g_u) with g_k[q_v, q_u] = g_v[q_v] g_u[q_u]  (linear chirp only)."""
    if s.kind != LINEAR:
        raise ValueError("the exact chirp is not separable")
    h = chirp_spectrum_1d(w, s)
    return row_factor_1d(vt, h, s), row_factor_1d(ut, h, s)


def kernel_row_2d(ut: float, vt: float, w: float, s: Setup, beam=None) -> np.ndarray:
    """Dense Ng x Ng row g_k[q_v, q_u] from the 2-D chirp spectrum (times the beam, if given)."""
    H = chirp_spectrum_2d(w, s, beam)
    q = np.arange(s.Ng)
    g = np.zeros((s.Ng, s.Ng), dtype=np.complex128)
    tv, wv = _taps(vt, s)
    tu, wu = _taps(ut, s)
    for qv, kv in zip(tv, wv):
        rows = (qv - q) % s.Ng
        for qu, ku in zip(tu, wu):
            cols = (qu - q) % s.Ng
            g += kv * ku * H[np.ix_(rows, cols)]
    return g


def kernel_row(ut: float, vt: float, w: float, s: Setup, beam=None) -> np.ndarray:
    if s.kind == LINEAR and beam is None:
        gv, gu = kernel_row_separable(ut, vt, w, s)
        return np.outer(gv, gu)
    return kernel_row_2d(ut, vt, w, s, beam)


# ----------------------------------------------------------------------------- sparsification

def energy_threshold(m: np.ndarray, E: float):
    """(tau, total) of Section 3.2's rule; entries m >= tau are kept.

    total is the row energy sum; the entries are taken in decreasing order and
    tau is the first one at which the running sum reaches E * total.  Only the
    largest entries are ever sorted: the K largest (K = 1024, 4096, ...) are
    selected, sorted and summed until their sum reaches E * total, so the
    crossing lies among them and the running sums are exactly those of a full
    sort.
    """
    m = np.asarray(m, dtype=np.float64).ravel()
    total = float(m.sum())
    if E >= 1.0:
        pos = m[m > 0]
        return (pos.min() if pos.size else np.inf), total
    n = m.size
    K = min(n, 1024)
    while True:
        top = m if K >= n else np.partition(m, n - K)[n - K:]
        srt = np.sort(top)[::-1]
        cs = np.cumsum(srt)
        if cs[-1] >= E * total or K >= n:
            k = min(int(np.searchsorted(cs, E * total, side="left")), srt.size - 1)
            return srt[k], total
        K = min(n, 4 * K)


def sparsify(m: np.ndarray, E: float) -> np.ndarray:
    tau, _ = energy_threshold(m, E)
    return np.asarray(m).ravel() >= tau


# ----------------------------------------------------------------------------- G

def build_rows(u, v, w, E: float, s: Setup, rows=None, with_info: bool = False, beam=None):
    """CSR of the sparsified rows (caller order) as scipy.sparse.csr_matrix.

    rows: optional subset of visibility indices; the matrix then has one row
    per selected visibility in that order.  beam: optional [M, 3] array of
    per-visibility Gaussian power patterns (l0, m0, sigma) (oracle.dde).
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    idx = np.arange(u.size) if rows is None else np.asarray(rows)
    ut = geo.grid_coord(u, s.N, s.L, s.sigma)
    vt = geo.grid_coord(v, s.N, s.L, s.sigma)
    indptr = [0]
    cols, vals, info = [], [], []
    for k in idx:
        g = kernel_row(ut[k], vt[k], w[k], s, None if beam is None else tuple(beam[k])).ravel()
        m = (g * g.conj()).real
        tau, total = energy_threshold(m, E)
        keep = np.nonzero(m >= tau)[0]
        cols.append(keep)
        vals.append(g[keep])
        indptr.append(indptr[-1] + keep.size)
        if with_info:
            info.append((tau, total, float(m[keep].sum())))
    G = sp.csr_matrix((np.concatenate(vals) if vals else np.zeros(0, complex),
                       np.concatenate(cols) if cols else np.zeros(0, int),
                       np.asarray(indptr)), shape=(idx.size, s.Ng * s.Ng))
    if with_info:
        return G, np.asarray(info)
    return G


def phi(G: sp.csr_matrix, x: np.ndarray, s: Setup) -> np.ndarray:
    """y = G F Z A x."""
    return G @ grid_forward(x, s).ravel()


def phi_adjoint(G: sp.csr_matrix, y: np.ndarray, s: Setup) -> np.ndarray:
    """x = A Z^H F^H G^H y."""
    X = (G.conj().T @ np.asarray(y, dtype=np.complex128)).reshape(s.Ng, s.Ng)
    return grid_adjoint(X, s)


def build_rows_csr_parts(args):
    """Worker form of build_rows for process pools: returns (indptr, indices, data, nrows)."""
    u, v, w, E, s, rows = args
    G = build_rows(u, v, w, E, s, rows=rows)
    return G.indptr, G.indices, G.data, G.shape[0]
