"""Pins of the oracle's sparse w-projection operator (CPU only).

Each test fixes the oracle against something other than itself: the direct
measurement sum, exact identities of the construction, closed forms and
special cases (see the oracle package header for the method).
"""
import numpy as np
import pytest

import synth
from oracle import dft, geometry, kb, wproj
from oracle.wproj import Setup

L = synth.fov_L()


def _vis(N, M, w_top, seed, dist="uniform"):
    rng = np.random.default_rng(seed)
    return synth.uvw(N, M, L, dist, 0.25, w_top, rng)


def _rc(shape, seed):
    return synth.random_complex(shape, np.random.default_rng(seed))


# --------------------------------------------------------------------------- P1: direct DFT

@pytest.mark.parametrize("kind", ["linear", "exact"])
@pytest.mark.parametrize("wmode", ["zero", "const", "random"])
def test_phi_converges_to_direct_measurement_sum(kind, wmode):
    """E = 1: Phi x approaches Eq. 1 / Eq. 3 geometrically as the KB support grows."""
    N = 16
    wtop = N / (2 * L * L)
    u, v, w = _vis(N, 24, wtop, 11)
    if wmode == "zero":
        w = np.zeros_like(w)
    elif wmode == "const":
        w = np.full_like(w, 0.7 * wtop)
    x = _rc((N, N), 12)
    yd = dft.measure(x, u, v, w, N, L, kind=kind)
    errs = []
    for W in (4, 6, 8):
        s = Setup(N=N, L=L, W=W, kind=kind)
        G = wproj.build_rows(u, v, w, 1.0, s)
        errs.append(np.linalg.norm(wproj.phi(G, x, s) - yd) / np.linalg.norm(yd))
    assert errs[0] < 3e-3
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20
    assert errs[2] < 1e-6


def test_phi_with_inverse_n_factor_matches_direct_sum():
    N = 16
    u, v, w = _vis(N, 16, N / (2 * L * L), 21)
    x = _rc((N, N), 22)
    s = Setup(N=N, L=L, W=8, kind="exact", a_phys="inv_n")
    G = wproj.build_rows(u, v, w, 1.0, s)
    yd = dft.measure(x, u, v, w, N, L, kind="exact", a_phys="inv_n")
    assert np.linalg.norm(wproj.phi(G, x, s) - yd) / np.linalg.norm(yd) < 1e-6


def test_adjoint_of_direct_sum_matches_phi_adjoint():
    N = 16
    u, v, w = _vis(N, 20, N / (2 * L * L), 31)
    y = _rc(20, 32)
    s = Setup(N=N, L=L, W=8)
    G = wproj.build_rows(u, v, w, 1.0, s)
    xd = dft.measure_adjoint(y, u, v, w, N, L)
    assert np.linalg.norm(wproj.phi_adjoint(G, y, s) - xd) / np.linalg.norm(xd) < 1e-6


# --------------------------------------------------------------------------- P2: adjoint identity

@pytest.mark.parametrize("E", [0.5, 0.99, 1.0])
def test_adjoint_identity(E):
    N, M = 32, 60
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, M, N / (2 * L * L), 41)
    G = wproj.build_rows(u, v, w, E, s)
    x = _rc((N, N), 42)
    y = _rc(M, 43)
    lhs = np.vdot(wproj.phi(G, x, s), y)
    rhs = np.vdot(x, wproj.phi_adjoint(G, y, s))
    scale = np.linalg.norm(wproj.phi(G, x, s)) * np.linalg.norm(y)
    assert abs(lhs - rhs) / scale < 1e-12


# --------------------------------------------------------------------------- P3: w = 0

def test_w_zero_rows_are_plain_kb_taps():
    """w = 0: the chirp spectrum is a delta, every row holds only the W x W KB taps."""
    N, W = 32, 4
    s = Setup(N=N, L=L, W=W)
    u, v, _ = _vis(N, 30, 0.0, 51)
    w = np.zeros_like(u)
    G = wproj.build_rows(u, v, w, 1.0, s)
    ut = geometry.grid_coord(u, N, L)
    vt = geometry.grid_coord(v, N, L)
    for k in range(u.size):
        row = G.getrow(k)
        assert row.nnz == W * W
        qu, ku = kb.kb_taps(ut[k], W, s.beta)
        qv, kv = kb.kb_taps(vt[k], W, s.beta)
        want = {((a + s.Ng // 2) % s.Ng) * s.Ng + (b + s.Ng // 2) % s.Ng: x * y
                for a, x in zip(qv, kv) for b, y in zip(qu, ku)}
        got = dict(zip(row.indices, row.data))
        assert set(got) == set(want)
        for c in want:
            assert abs(got[c] - want[c]) <= 1e-12 * abs(want[c])


# --------------------------------------------------------------------------- P4: constant w (Eq. 6)

@pytest.mark.parametrize("kind", ["linear", "exact"])
def test_constant_w_equals_image_domain_modulation(kind):
    """One w for every row: the uv convolution equals modulating the image before the FFT."""
    N = 32
    s = Setup(N=N, L=L, kind=kind)
    u, v, _ = _vis(N, 40, 0.0, 61)
    w0 = 0.6 * N / (2 * L * L)
    w = np.full_like(u, w0)
    x = _rc((N, N), 62)
    G = wproj.build_rows(u, v, w, 1.0, s)
    y = wproj.phi(G, x, s)
    # independent route: modulate the padded, apodised image, FFT, interpolate with KB
    Ng, o = s.Ng, geometry.pad_offset(N)
    z = np.zeros((Ng, Ng), complex)
    z[o:o + N, o:o + N] = x * wproj.apodisation(s)
    lj = geometry.padded_coords(N, L)
    from oracle.chirp import chirp
    z *= chirp(lj[None, :], lj[:, None], w0, kind)
    X = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(z)))
    ut, vt = geometry.grid_coord(u, N, L), geometry.grid_coord(v, N, L)
    yref = np.empty_like(y)
    for k in range(u.size):
        qu, ku = kb.kb_taps(ut[k], s.W, s.beta)
        qv, kv = kb.kb_taps(vt[k], s.W, s.beta)
        yref[k] = sum(a * b * X[(c + Ng // 2) % Ng, (d + Ng // 2) % Ng]
                      for c, a in zip(qv, kv) for d, b in zip(qu, ku))
    assert np.linalg.norm(y - yref) / np.linalg.norm(yref) < 1e-12


# --------------------------------------------------------------------------- P5: Gauss sum

@pytest.mark.parametrize("N", [64, 125, 128])
def test_chirp_spectrum_quadratic_gauss_sum(N):
    """w delta^2 Ng = 1: sum_t exp(i pi t^2/Ng) exp(-2 pi i t d/Ng) = sqrt(Ng) e^{i pi/4} e^{-i pi d^2/Ng}."""
    s = Setup(N=N, L=L)
    Ng = s.Ng
    w = 1.0 / (s.delta ** 2 * Ng)
    h = wproj.chirp_spectrum_1d(w, s)
    d = np.arange(Ng)
    closed = np.exp(1j * np.pi / 4) * np.exp(-1j * np.pi * d * d / Ng) / np.sqrt(Ng)
    assert np.abs(h - closed).max() < 1e-12


def test_chirp_spectrum_has_unit_energy():
    """The chirp has unit modulus, so its normalised spectrum has unit energy (Parseval)."""
    s = Setup(N=64, L=L)
    for w in (0.0, 3000.0, 20000.0):
        h = wproj.chirp_spectrum_1d(w, s)
        assert abs(np.sum(np.abs(h) ** 2) - 1.0) < 1e-12
        H = wproj.chirp_spectrum_2d(w, s)
        assert abs(np.sum(np.abs(H) ** 2) - 1.0) < 1e-12


# --------------------------------------------------------------------------- separable vs 2-D form

def test_separable_rows_equal_2d_rows():
    N = 32
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, 6, N / (2 * L * L), 71)
    ut, vt = geometry.grid_coord(u, N, L), geometry.grid_coord(v, N, L)
    for k in range(u.size):
        g2 = wproj.kernel_row_2d(ut[k], vt[k], w[k], s)
        gv, gu = wproj.kernel_row_separable(ut[k], vt[k], w[k], s)
        assert np.abs(g2 - np.outer(gv, gu)).max() < 1e-13 * np.abs(g2).max()


@pytest.mark.parametrize("E", [0.5, 0.99, 0.999])
def test_kept_set_is_a_staircase_of_the_one_dimensional_energies(E):
    """A tap's energy is the product A_a B_b of the 1-D factor energies, so the kept set is
    monotone in both: taking the u cells by descending A, each v cell keeps a prefix of them, and
    the prefix length does not increase with descending B.  The oracle's kept rows (threshold on
    the 2-D energies) agree with that staircase up to ties at the threshold."""
    N = 64
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, 12, N / (2 * L * L), 72)
    ut, vt = geometry.grid_coord(u, N, L), geometry.grid_coord(v, N, L)
    G = wproj.build_rows(u, v, w, E, s)
    for k in range(u.size):
        gv, gu = wproj.kernel_row_separable(ut[k], vt[k], w[k], s)
        A, B = np.abs(gu) ** 2, np.abs(gv) ** 2
        m = np.outer(B, A)
        tau, _ = wproj.energy_threshold(np.abs(np.outer(gv, gu)).ravel() ** 2, E)
        ua, vb = np.argsort(-A, kind="stable"), np.argsort(-B, kind="stable")
        nb = np.array([(A[ua] * B[b] >= tau).sum() for b in vb])
        assert np.all(np.diff(nb) <= 0)
        stair = np.zeros((s.Ng, s.Ng), dtype=bool)
        for b, n in zip(vb, nb):
            stair[b, ua[:n]] = True
        assert np.array_equal(stair, m >= tau)       # the staircase is the product-energy kept set
        kept = np.zeros(s.Ng * s.Ng, dtype=bool)
        kept[G.indices[G.indptr[k]:G.indptr[k + 1]]] = True
        diff = np.nonzero(kept != stair.ravel())[0]
        assert np.all(np.abs(m.ravel()[diff] - tau) <= 1e-12 * tau)


def test_linear_and_exact_chirp_agree_to_first_order():
    N = 32
    l = geometry.padded_coords(N, L)
    from oracle.chirp import chirp
    for w in (100.0, 1000.0, 10000.0):
        lin = chirp(l[None, :], l[:, None], w, "linear")
        ex = chirp(l[None, :], l[:, None], w, "exact")
        r2 = l[None, :] ** 2 + l[:, None] ** 2
        bound = np.pi * w * r2 ** 2 / 4 * 1.01 + 1e-15      # |phase difference| <= pi w r^4 / 4 (+ higher order)
        assert np.all(np.abs(np.angle(lin * ex.conj())) <= bound)


# --------------------------------------------------------------------------- sparsification

def test_threshold_keeps_minimal_set_reaching_E():
    rng = np.random.default_rng(81)
    for E in (0.1, 0.5, 0.9, 0.99, 0.999):
        m = rng.exponential(size=500) ** 3
        tau, T = wproj.energy_threshold(m, E)
        kept = m[m >= tau]
        assert kept.sum() >= E * T * (1 - 1e-15)
        assert kept.sum() - kept.min() < E * T   # dropping the weakest kept entry loses the target


def test_threshold_keeps_ties():
    m = np.array([4.0, 2.0, 2.0, 2.0, 1.0])
    tau, T = wproj.energy_threshold(m, 0.5)   # 4 + 2 reaches 5.5: tau = 2, all three 2s kept
    assert tau == 2.0 and np.count_nonzero(m >= tau) == 4


def test_rows_keep_energy_fraction_and_nnz_monotone_in_E():
    N = 32
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, 12, N / (2 * L * L), 91)
    prev = None
    for E in (0.5, 0.9, 0.99, 0.999, 1.0):
        G, info = wproj.build_rows(u, v, w, E, s, with_info=True)
        tau, T, kept = info.T
        assert np.all(kept >= np.minimum(E, 1.0) * T * (1 - 1e-12))
        nnz = np.diff(G.indptr)
        if prev is not None:
            assert np.all(nnz >= prev)
        prev = nnz


def test_nnz_grows_with_w():
    N = 64
    s = Setup(N=N, L=L)
    wtop = N / (2 * L * L)
    ut = np.full(1, 3.3)
    counts = []
    for frac in (0.0, 0.1, 0.3, 0.6, 1.0):
        G = wproj.build_rows(ut / (2 * L), ut / (2 * L), np.array([frac * wtop]), 0.99, s)
        counts.append(G.nnz)
    assert all(a < b for a, b in zip(counts, counts[1:]))


def test_operator_converges_as_E_goes_to_one():
    N = 32
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, 40, N / (2 * L * L), 101)
    x = _rc((N, N), 102)
    y1 = wproj.phi(wproj.build_rows(u, v, w, 1.0, s), x, s)
    errs = [np.linalg.norm(wproj.phi(wproj.build_rows(u, v, w, E, s), x, s) - y1) / np.linalg.norm(y1)
            for E in (0.9, 0.99, 0.999, 0.99999)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-2


def test_csr_columns_ascending_and_in_range():
    N = 32
    s = Setup(N=N, L=L)
    u, v, w = _vis(N, 25, N / (2 * L * L), 111)
    G = wproj.build_rows(u, v, w, 0.99, s)
    for k in range(G.shape[0]):
        c = G.indices[G.indptr[k]:G.indptr[k + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < s.Ng ** 2


def test_grid_transforms_are_adjoint_and_centred():
    N = 16
    s = Setup(N=N, L=L)
    x = _rc((N, N), 121)
    X = wproj.grid_forward(x, s)
    Y = _rc((s.Ng, s.Ng), 122)
    assert abs(np.vdot(X, Y) - np.vdot(x, wproj.grid_adjoint(Y, s))) < 1e-10 * np.linalg.norm(X) * np.linalg.norm(Y)
    # centred DFT written out
    j = np.arange(s.Ng) - s.Ng // 2
    Fm = np.exp(-2j * np.pi * np.outer(j, j) / s.Ng)
    z = np.zeros((s.Ng, s.Ng), complex)
    o = geometry.pad_offset(N)
    z[o:o + N, o:o + N] = x * wproj.apodisation(s)
    assert np.abs(Fm @ z @ Fm.T - X).max() < 1e-10 * np.abs(X).max()


@pytest.mark.parametrize("kind", ["linear", "exact"])
def test_taps_are_bounded_by_the_window_peak(kind):
    """|G_kc| <= (W I0(beta))^2 for every row (the scatter's fixed-point scale relies on it): each
    axis sums W window weights <= I0(beta) against chirp-spectrum values of modulus <= 1."""
    from scipy import special
    N = 32
    for W in (4, 6):
        s = Setup(N=N, L=0.3, W=W, kind=kind)
        bound = (W * special.i0(s.beta)) ** 2
        u, v, w = synth.uvw(N, 40, 0.3, "uniform", 0.25, N / (2 * 0.3 ** 2), np.random.default_rng(61 + W))
        w[:8] = 0.0                                    # w = 0 rows concentrate the most energy
        ut, vt = u * 2 * s.L, v * 2 * s.L
        peak = max(np.abs(wproj.kernel_row(ut[k], vt[k], w[k], s)).max() for k in range(40))
        assert peak <= bound
        assert peak > 1e-3 * bound                     # and the bound is not vacuous
