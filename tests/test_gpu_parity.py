"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: complex FP32 path, operator relative error <= 1e-5 against the
FP64 oracle built with the same (W, beta, E, chirp); index work (row
structure, kept sets) bit-exact except for taps tied with the row threshold
within FP64 rounding (1e-9 relative), where either decision is correct.
"""
import numpy as np
import pytest

import synth
from oracle import wproj
from oracle.wproj import Setup

from helpers import bf16_rms_bound, oracle_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402

L = synth.fov_L()
TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def c64(a):
    return dev(np.asarray(a, dtype=np.complex64).ravel())


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def say(msg):
    print(msg, flush=True)


def build(plan, u, v, w, E, taps=wp.WP_TAPS_C64):
    G = wp.build_G(plan, dev(u), dev(v), dev(w), E, taps=taps)
    torch.cuda.synchronize()
    return G


def gpu_rows(G):
    rp = G.rowptr.cpu().numpy()
    col = G.col.cpu().numpy()
    val = G.val.cpu().numpy() if G.taps == wp.WP_TAPS_C64 else None
    perm = G.perm.cpu().numpy()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    return rp, col, val, perm, inv


def check_rows(G, u, v, w, E, s, rows, beam=None):
    """Kept sets and values of the sampled rows against dense oracle rows."""
    rp, col, val, perm, inv = gpu_rows(G)
    ut = u * 2 * s.L          # u / du with du = 1 / (2L)
    vt = v * 2 * s.L
    for k in rows:
        g = wproj.kernel_row(ut[k], vt[k], w[k], s, None if beam is None else tuple(beam[k])).ravel()
        m = (g * g.conj()).real
        tau, _ = wproj.energy_threshold(m, E)
        want = np.nonzero(m >= tau)[0]
        r = inv[k]
        got = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(got) > 0), f"row {k}: columns not ascending"
        diff = np.setxor1d(got, want)
        if diff.size:
            assert np.all(np.abs(m[diff] - tau) <= 1e-9 * tau), f"row {k}: kept sets differ beyond ties"
        if val is not None:
            common, ig, iw = np.intersect1d(got, want, return_indices=True)
            gv = val[rp[r]:rp[r + 1]][ig]
            scale = np.abs(g).max()
            assert np.all(np.abs(gv - g[common]) <= 1e-6 * np.abs(g[common]) + 1e-7 * scale), f"row {k}: values"


# --------------------------------------------------------------------------- A, Z, F

@pytest.mark.parametrize("aphys", ["one", "inv_n"])
@pytest.mark.parametrize("N", [32, 64, 128, 256, 512, 1024, 2048])
def test_grid_forward_and_adjoint(N, aphys):
    """A, Z, F and their adjoint at every supported grid size (Ng = 64 .. 4096), with the plain
    apodisation and with the 1/n factor of Eq. 1 folded in."""
    say(f"grid transforms N={N} aphys={aphys}")
    s = Setup(N=N, L=L, a_phys=aphys)
    plan = wp.Plan(N, L, aphys=wp.WP_APHYS_INV_N if aphys == "inv_n" else wp.WP_APHYS_ONE)
    rng = np.random.default_rng(N)
    x = synth.random_complex((N, N), rng)
    X = wp.grid_forward(plan, c64(x)).cpu().numpy().reshape(s.Ng, s.Ng)
    assert relerr(X, wproj.grid_forward(x, s)) < TOL
    Y = synth.random_complex((s.Ng, s.Ng), rng)
    xa = wp.grid_adjoint(plan, c64(Y)).cpu().numpy().reshape(N, N)
    assert relerr(xa, wproj.grid_adjoint(Y, s)) < TOL


# --------------------------------------------------------------------------- builder

def test_build_tiny_form_all_rows():
    wl = synth.workload(0)
    say(f"build: {wl.name} N={wl.N} M={wl.M}")
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    Go = wproj.build_rows(u, v, w, wl.E, s)
    assert abs(G.nnz - Go.nnz) <= 1e-6 * Go.nnz
    check_rows(G, u, v, w, wl.E, s, range(wl.M))


def test_build_plain_form_sampled_rows():
    wl = synth.workload(1)
    say(f"build: {wl.name} N={wl.N} M={wl.M} (sampled rows)")
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    rows = synth.subset_rows(wl.M, 96, synth.rng_for(wl.seed, "subset"))
    rows = np.unique(np.concatenate([rows, [0, wl.M - 1]]))
    check_rows(G, u, v, w, wl.E, s, rows)
    # every row appears once in the tile order, row lengths add up
    rp, col, _, perm, _ = gpu_rows(G)
    assert np.array_equal(np.sort(perm), np.arange(wl.M))
    assert rp[0] == 0 and rp[-1] == G.nnz and np.all(np.diff(rp) > 0)
    assert col.min() >= 0 and col.max() < s.Ng ** 2


def test_work_items_cover_rows_once():
    wl = synth.workload(1)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    items = G.work.cpu().numpy()[:4 * G.n_work].reshape(-1, 4)
    seen = np.zeros(wl.M, dtype=int)
    for tv, tu, rb, re in items:
        assert rb < re
        seen[rb:re] += 1
    assert np.all(seen == 1)
    # rows of an item lie in its tile
    perm = G.perm.cpu().numpy()
    ut = u * 2 * wl.L + wl.Ng / 2
    vt = v * 2 * wl.L + wl.Ng / 2
    for tv, tu, rb, re in items[:: max(1, len(items) // 50)]:
        ks = perm[rb:re]
        assert np.all((vt[ks] // 32).astype(int) == tv) and np.all((ut[ks] // 32).astype(int) == tu)


# --------------------------------------------------------------------------- Phi and Phi^H

def test_phi_and_adjoint_tiny_form():
    wl = synth.workload(0)
    say(f"apply: {wl.name}")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    Go = wproj.build_rows(u, v, w, wl.E, s)
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y, wproj.phi(Go, x, s)) < TOL
    yv = synth.random_complex(wl.M, synth.rng_for(wl.seed, "y"))
    x_ref = wproj.phi_adjoint(Go, yv, s)
    for use_t in (True, False):            # gather over the transposed copy, tiled scatter
        G.use_transpose = use_t
        xa = wp.apply_PhiT(plan, G, c64(yv)).cpu().numpy().reshape(wl.N, wl.N)
        assert relerr(xa, x_ref) < TOL, use_t


@pytest.mark.parametrize("taps", ["c64", "bf16", "i16"])
def test_gather_and_scatter_grid_match_oracle(taps):
    wl = synth.workload(0)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    t = {"c64": wp.WP_TAPS_C64, "bf16": wp.WP_TAPS_BF16, "i16": wp.WP_TAPS_I16}[taps]
    G = build(plan, u, v, w, wl.E, taps=t)
    yv = synth.random_complex(wl.M, synth.rng_for(wl.seed, "y", 5))
    Xg = wp.grid_gather(plan, G, c64(yv)).cpu().numpy()
    Xs = wp.grid_scatter(plan, G, c64(yv)).cpu().numpy()
    G.use_blocks = False                   # one lane group per cell instead of the block table
    Xc = wp.grid_gather(plan, G, c64(yv)).cpu().numpy()
    G.use_blocks = True
    Go = wproj.build_rows(u, v, w, wl.E, s)
    X_ref = Go.conj().T @ yv
    x = synth.sky(wl.N, 4, 6, synth.rng_for(wl.seed, "sky", 5))
    y_ref = wproj.phi(Go, x, s)
    # bfloat16: 1.5 x the expected error of rounded taps under the rounding model (tests/helpers.py),
    # from the oracle's rows and vectors; int16 block floating point: 1e-4 (its rounding unit is
    # 2^-16 of the row's largest component, far inside the 1e-3 target)
    tol = {"c64": TOL, "bf16": 1.5 * bf16_rms_bound(Go, yv, True, X_ref) + TOL, "i16": 1e-4}[taps]
    tol_phi = {"c64": TOL, "bf16": 1.5 * bf16_rms_bound(Go, wproj.grid_forward(x, s).ravel(), False, y_ref) + TOL,
               "i16": 1e-4}[taps]
    say(f"gather/scatter {taps}: G^H err {relerr(Xg, X_ref):.3e} (tol {tol:.3e})")
    assert relerr(Xg, X_ref) < tol and relerr(Xs, X_ref) < tol and relerr(Xc, X_ref) < tol
    assert relerr(Xg, Xs) < 1e-5 and relerr(Xg, Xc) < 1e-5
    assert relerr(wp.apply_Phi(plan, G, c64(x)).cpu().numpy(), y_ref) < tol_phi


def gather_table_model(tcp, cells, B=512, CAP=64):
    """Block table of the transposed copy as the header defines it, from tcolptr."""
    nnz = int(tcp[-1])
    nslot = nnz // B + (cells - 1) // CAP + 1
    c = np.arange(cells)
    slot = tcp[:cells] // B + c // CAP
    first = np.ones(cells, dtype=bool)
    first[1:] = slot[1:] != slot[:-1]
    t = np.empty((nslot + 1, 2), dtype=np.int64)
    nb = int(first.sum())
    t[:nb, 0], t[:nb, 1] = c[first], tcp[:cells][first]
    t[nb:] = (cells, nnz)
    return t.ravel()


def test_gather_with_crowded_cells():
    """6000 visibilities within a 3 x 3 cell patch: cells hold up to ~5800 entries (many passes of
    each lane group) while most of the grid is empty."""
    N, M = 64, 6000
    say(f"gather: crowded cells N={N} M={M}")
    s = Setup(N=N, L=L)
    rng = np.random.default_rng(3)
    du = 1 / (2 * L)
    u = (rng.uniform(-1.5, 1.5, M) + 10.3) * du
    v = (rng.uniform(-1.5, 1.5, M) - 7.6) * du
    w = rng.uniform(0, 0.15 * N / (2 * L * L), M)
    plan = wp.Plan(N, L)
    G = build(plan, u, v, w, 0.99)
    tcp = G.tcolptr.cpu().numpy()
    assert np.diff(tcp).max() > 4096               # single cells span many chunks of a block
    assert np.array_equal(G.tblk.cpu().numpy(), gather_table_model(tcp, s.Ng ** 2))
    Go = wproj.build_rows(u, v, w, 0.99, s)
    assert abs(G.nnz - Go.nnz) <= 1e-6 * Go.nnz
    yv = synth.random_complex(M, synth.rng_for(1, "y", 9))
    X_ref = Go.conj().T @ yv
    Xg = wp.grid_gather(plan, G, c64(yv)).cpu().numpy()
    Xs = wp.grid_scatter(plan, G, c64(yv)).cpu().numpy()
    G.use_blocks = False
    Xc = wp.grid_gather(plan, G, c64(yv)).cpu().numpy()
    assert relerr(Xg, X_ref) < TOL and relerr(Xs, X_ref) < TOL and relerr(Xc, X_ref) < TOL
    assert np.all(Xg[X_ref == 0] == 0)             # empty cells are written as zeros


def _check_transposed_copy(G, M, Ng):
    rp, col, val, perm, inv = gpu_rows(G)
    tcp = G.tcolptr.cpu().numpy()
    trow = G.trow.cpu().numpy()[:G.nnz]
    tval = G.tval.cpu().numpy()[:G.nnz]
    assert tcp[0] == 0 and tcp[-1] == G.nnz and np.all(np.diff(tcp) >= 0)
    # same (row, cell, value) triples as the rows, each cell's entries ordered by sorted row
    rows_of = np.repeat(np.arange(M), np.diff(rp))
    a = np.lexsort((rows_of, col))
    cells_t = np.repeat(np.arange(tcp.size - 1), np.diff(tcp))
    assert np.array_equal(col[a], cells_t)
    assert np.array_equal(rows_of[a], trow)
    assert np.array_equal(val[a], tval)
    assert np.array_equal(G.tblk.cpu().numpy(), gather_table_model(tcp, Ng ** 2))
    return np.diff(tcp)


def test_transposed_copy_structure():
    wl = synth.workload(1)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    _check_transposed_copy(G, wl.M, wl.Ng)


def test_transposed_copy_crowded_cells():
    """Cells of up to 2500 entries (the builder sorts cells of more than 1024 entries by another
    path than the rest) keep the same structure."""
    wl = synth.workload(0)
    N, M = wl.N, 2500
    rng = np.random.default_rng(41)
    cell = 1.0 / (2 * wl.L)
    u = 3.2 * cell + rng.uniform(-0.3, 0.3, M) * cell
    v = -5.7 * cell + rng.uniform(-0.3, 0.3, M) * cell
    w = rng.uniform(0, synth.configs.w_for_support(8, 4, wl.L), M)
    plan = wp.Plan(N, wl.L)
    G = build(plan, u, v, w, 0.99)
    lengths = _check_transposed_copy(G, M, 2 * N)
    assert lengths.max() > 1024 and np.any((lengths > 1) & (lengths <= 1024))


def test_phi_plain_form_sampled_rows():
    wl = synth.workload(1)
    say(f"apply: {wl.name} full size, sampled outputs")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=True)
    rows = synth.subset_rows(wl.M, 4096, synth.rng_for(wl.seed, "subset", 1))
    Go = oracle_rows(u, v, w, wl.E, s, rows)
    y_ref = Go @ wproj.grid_forward(x, s).ravel()
    for fac in (False, True):              # stored taps, factor records
        G.use_factors = fac
        y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
        assert relerr(y[rows], y_ref) < TOL, fac


def test_phi_adjoint_plain_form_on_sampled_support():
    """Phi^H of a y that is non-zero on 4096 of the 32768 rows: the oracle needs only those rows.
    Through the blocked gather (the benchmark's form), the per-cell gather and the tiled scatter."""
    wl = synth.workload(1)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    rows = synth.subset_rows(wl.M, 4096, synth.rng_for(wl.seed, "subset", 2))
    yv = np.zeros(wl.M, dtype=np.complex128)
    yv[rows] = synth.random_complex(rows.size, synth.rng_for(wl.seed, "y", 2))
    Go = oracle_rows(u, v, w, wl.E, s, rows)
    x_ref = wproj.phi_adjoint(Go, yv[rows], s)
    for use_t, blocks in ((True, True), (True, False), (False, True)):
        G.use_transpose, G.use_blocks = use_t, blocks
        xa = wp.apply_PhiT(plan, G, c64(yv)).cpu().numpy().reshape(wl.N, wl.N)
        assert relerr(xa, x_ref) < TOL, (use_t, blocks)


def test_adjoint_identity_full_size():
    wl = synth.workload(1)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    rng = synth.rng_for(wl.seed, "x", 3)
    x = c64(synth.random_complex(wl.N * wl.N, rng))
    yv = c64(synth.random_complex(wl.M, rng))
    Px = wp.apply_Phi(plan, G, x)
    Py = wp.apply_PhiT(plan, G, yv)
    lhs = torch.vdot(Px.to(torch.complex128), yv.to(torch.complex128)).item()
    rhs = torch.vdot(x.to(torch.complex128), Py.to(torch.complex128)).item()
    scale = (torch.linalg.norm(Px.to(torch.complex128)) * torch.linalg.norm(yv.to(torch.complex128))).item()
    assert abs(lhs - rhs) / scale < 1e-5


def test_phi_deterministic_and_adjoint_repeatable():
    wl = synth.workload(1)
    x, u, v, w = synth.workload_inputs(wl)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    xd = c64(x)
    y1 = wp.apply_Phi(plan, G, xd)
    y2 = wp.apply_Phi(plan, G, xd)
    assert torch.equal(y1, y2)
    a1 = wp.apply_PhiT(plan, G, y1)
    a2 = wp.apply_PhiT(plan, G, y1)
    assert torch.equal(a1, a2)                 # gather form: no atomics, bitwise repeatable
    G.use_transpose = False
    s1 = wp.apply_PhiT(plan, G, y1)
    s2 = wp.apply_PhiT(plan, G, y1)
    assert (torch.linalg.norm(s1 - s2) / torch.linalg.norm(s1)).item() < 1e-6
    assert (torch.linalg.norm(s1 - a1) / torch.linalg.norm(a1)).item() < 1e-5


def test_sorted_order_matches_caller_order():
    wl = synth.workload(1)
    x, u, v, w = synth.workload_inputs(wl)
    plan = wp.Plan(wl.N, wl.L)
    G = build(plan, u, v, w, wl.E)
    xd = c64(x)
    yc = wp.apply_Phi(plan, G, xd)
    G.order = wp.WP_ORDER_SORTED
    ys = wp.apply_Phi(plan, G, xd)
    assert torch.equal(wp.to_sorted(G, yc), ys)
    assert torch.equal(wp.to_caller(G, ys), yc)
    for use_t in (True, False):
        G.use_transpose = use_t
        G.order = wp.WP_ORDER_SORTED
        a_s = wp.apply_PhiT(plan, G, ys)
        G.order = wp.WP_ORDER_CALLER
        a_c = wp.apply_PhiT(plan, G, yc)
        assert (torch.linalg.norm(a_s - a_c) / torch.linalg.norm(a_c)).item() < 1e-6


# --------------------------------------------------------------------------- edge cases

def test_single_visibility_and_band_edges():
    N = 64
    s = Setup(N=N, L=L)
    plan = wp.Plan(N, L)
    B = N / (2 * L)
    u = np.array([-B * (1 - 1e-9), B * (1 - 1e-6), 0.0, -B * 0.999, 0.3])
    v = np.array([B * (1 - 1e-6), -B * (1 - 1e-9), 0.0, B * 0.5, -B * 0.999])
    w = np.array([0.0, 900.0, 0.0, 26000.0, 13000.0])
    x = synth.random_complex((N, N), np.random.default_rng(5))
    for sel in ([0], [1], [2], [0, 1, 2, 3, 4]):
        sel = np.array(sel)
        G = build(plan, u[sel], v[sel], w[sel], 0.99)
        Go = wproj.build_rows(u[sel], v[sel], w[sel], 0.99, s)
        assert relerr(wp.apply_Phi(plan, G, c64(x)).cpu().numpy(), wproj.phi(Go, x, s)) < TOL
        yv = synth.random_complex(sel.size, np.random.default_rng(6))
        xa = wp.apply_PhiT(plan, G, c64(yv)).cpu().numpy().reshape(N, N)
        assert relerr(xa, wproj.phi_adjoint(Go, yv, s)) < TOL


def test_w_zero_and_full_energy_small_grid():
    N = 32
    s = Setup(N=N, L=L)
    plan = wp.Plan(N, L)
    u, v, _ = synth.uvw(N, 37, L, "uniform", 0.0, 0.0, np.random.default_rng(8))
    x = synth.random_complex((N, N), np.random.default_rng(9))
    for w, E in ((np.zeros(37), 0.99), (np.random.default_rng(10).uniform(0, N / (2 * L * L), 37), 1.0)):
        G = build(plan, u, v, w, E)
        Go = wproj.build_rows(u, v, w, E, s)
        assert G.nnz == Go.nnz
        assert relerr(wp.apply_Phi(plan, G, c64(x)).cpu().numpy(), wproj.phi(Go, x, s)) < TOL


def decode_records(G):
    """Per sorted row: (ua, vb, nb, gu, gv) of its factor record, as the header defines it."""
    frec = G.frec.cpu().numpy()
    fd = G.fdat.cpu().numpy()
    out = []
    for r in range(G.M):
        o = int(frec[r])
        nu, nv = (int(x) for x in fd[o:o + 4].view(np.uint16))
        ua = fd[o + 4:o + 4 + 2 * nu].view(np.uint16).astype(np.int64)
        vb = fd[o + 4 + 2 * nu:o + 4 + 2 * nu + 2 * nv].view(np.uint16).astype(np.int64)
        nb = fd[o + 4 + 2 * nu + 2 * nv:o + 4 + 2 * nu + 4 * nv].view(np.uint16).astype(np.int64)
        vo = o + ((4 + 2 * nu + 4 * nv + 7) & ~7)
        gu = fd[vo:vo + 8 * nu].view(np.complex64)
        gv = fd[vo + 8 * nu:vo + 8 * (nu + nv)].view(np.complex64)
        assert int(frec[r + 1]) - o == (((4 + 2 * nu + 4 * nv + 7) & ~7) + 8 * (nu + nv))
        out.append((ua, vb, nb, gu, gv))
    return out


def check_records(G, Ng):
    """Every record expands to its stored row: the same cells, taps equal to the stored values up
    to complex-float rounding of the two factors."""
    rp = G.rowptr.cpu().numpy()
    col = G.col.cpu().numpy()
    val = G.val.cpu().numpy()
    for r, (ua, vb, nb, gu, gv) in enumerate(decode_records(G)):
        assert np.all(np.diff(nb) <= 0) and nb.size and nb[0] == ua.size and np.all(nb >= 1)
        assert np.all(np.diff(np.abs(gu.astype(np.complex128)) ** 2) <= 1e-6 * np.abs(gu[0]) ** 2)
        b_idx = np.repeat(np.arange(vb.size), nb)
        a_idx = np.concatenate([np.arange(n) for n in nb])
        cells = vb[b_idx] * Ng + ua[a_idx]
        taps = gv[b_idx].astype(np.complex128) * gu[a_idx].astype(np.complex128)
        o = np.argsort(cells)
        c_row = col[rp[r]:rp[r + 1]]
        assert np.array_equal(cells[o], c_row), f"row {r}: kept cells differ"
        v_row = val[rp[r]:rp[r + 1]].astype(np.complex128)
        assert np.all(np.abs(taps[o] - v_row) <= 3e-7 * np.abs(v_row).max() + 3e-7 * np.abs(v_row)), f"row {r}"


def test_factor_records_tiny_form():
    """Every row of the tiny form: records expand to the stored rows; their factors are the
    oracle's 1-D factors; the degrid from records matches the oracle."""
    wl = synth.workload(0)
    say(f"factor records: {wl.name}")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=True)
    torch.cuda.synchronize()
    check_records(G, wl.Ng)
    perm = G.perm.cpu().numpy()
    recs = decode_records(G)
    for r in range(0, wl.M, 37):
        k = perm[r]
        gv_o, gu_o = wproj.kernel_row_separable(u[k] * 2 * s.L, v[k] * 2 * s.L, w[k], s)
        ua, vb, nb, gu, gv = recs[r]
        assert np.all(np.abs(gu - gu_o[ua]) <= 1e-6 * np.abs(gu_o).max())
        assert np.all(np.abs(gv - gv_o[vb]) <= 1e-6 * np.abs(gv_o).max())
    Go = wproj.build_rows(u, v, w, wl.E, s)
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y, wproj.phi(Go, x, s)) < TOL
    G.use_factors = False
    assert relerr(wp.apply_Phi(plan, G, c64(x)).cpu().numpy(), y) < 1e-6


def test_factor_records_plain_form():
    wl = synth.workload(1)
    say(f"factor records: {wl.name}")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=True)
    torch.cuda.synchronize()
    check_records(G, wl.Ng)
    rows = synth.subset_rows(wl.M, 64, synth.rng_for(wl.seed, "subset", 1))
    Go = wproj.build_rows(u, v, w, wl.E, s, rows=rows)
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y[rows], Go @ wproj.grid_forward(x, s).ravel()) < TOL
    X = c64(synth.random_complex(wl.Ng ** 2, np.random.default_rng(15)))
    y1 = wp.degrid(plan, G, X).cpu().numpy()
    G.use_factors = False
    assert relerr(y1, wp.degrid(plan, G, X).cpu().numpy()) < 1e-6


@pytest.mark.parametrize("workload", [0, 1])
def test_factor_record_form_without_stored_taps(workload):
    """G kept as factor records only (no taps, no columns, no transposed copy): Phi from the records
    and Phi^H scattered from them, against the oracle (every row of the tiny form; 4096 sampled rows of
    the plain form), and adjoint to each other; a fraction of the stored form's bytes."""
    wl = synth.workload(workload)
    say(f"factor-record form: {wl.name}")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=True, transpose=False, stored=False)
    torch.cuda.synchronize()
    assert G.col is None and G.val is None and G.tcolptr is None
    rows = np.arange(wl.M) if workload == 0 else synth.subset_rows(wl.M, 4096, synth.rng_for(wl.seed, "subset", 3))
    Go = oracle_rows(u, v, w, wl.E, s, rows)
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y[rows], Go @ wproj.grid_forward(x, s).ravel()) < TOL
    yv = np.zeros(wl.M, dtype=np.complex128)
    yv[rows] = synth.random_complex(rows.size, synth.rng_for(wl.seed, "y", 3))
    xa = wp.apply_PhiT(plan, G, c64(yv)).cpu().numpy().reshape(wl.N, wl.N)
    assert relerr(xa, wproj.phi_adjoint(Go, yv[rows], s)) < TOL
    # the two products of the record form are adjoint (random x and y over every row)
    rng = np.random.default_rng(17)
    xr = c64(synth.random_complex(wl.N * wl.N, rng))
    yr = c64(synth.random_complex(wl.M, rng))
    Px = wp.apply_Phi(plan, G, xr).to(torch.complex128)
    Py = wp.apply_PhiT(plan, G, yr).to(torch.complex128)
    lhs = torch.vdot(Px, yr.to(torch.complex128)).item()
    rhs = torch.vdot(xr.to(torch.complex128), Py).item()
    assert abs(lhs - rhs) <= 1e-5 * (torch.linalg.norm(Px) * torch.linalg.norm(yr.to(torch.complex128))).item()
    Gs = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=True)
    assert G.nbytes() < 0.25 * Gs.nbytes()
    with pytest.raises(ValueError):
        wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, factors=False, transpose=False, stored=False)


def test_factor_records_wide_rows_and_edges():
    """E = 1: rows with w > 0 keep the whole 512 x 512 grid (nu = nv = 512, eight u candidates
    per lane), rows with w = 0 a 4 x 4 box; plus visibilities at the band edges."""
    N, M = 256, 24
    s = Setup(N=N, L=L)
    plan = wp.Plan(N, L)
    u, v, w = synth.uvw(N, M, L, "uniform", 0.0, N / (2 * L * L), np.random.default_rng(13))
    w[::2] = 0.0
    B = N / (2 * L)
    u[:4] = [-B * 0.9999, B * 0.9999, 0.0, -B * 0.9999]
    v[:4] = [B * 0.9999, -B * 0.9999, -B * 0.9999, 0.0]
    G = wp.build_G(plan, dev(u), dev(v), dev(w), 1.0, factors=True)
    torch.cuda.synchronize()
    check_records(G, s.Ng)
    x = synth.random_complex((N, N), np.random.default_rng(14))
    Go = wproj.build_rows(u, v, w, 1.0, s)
    assert relerr(wp.apply_Phi(plan, G, c64(x)).cpu().numpy(), wproj.phi(Go, x, s)) < TOL


@pytest.mark.parametrize("E", [0.1, 0.5, 0.9, 0.999])
def test_energy_levels(E):
    N, M = 64, 53
    s = Setup(N=N, L=L)
    plan = wp.Plan(N, L)
    u, v, w = synth.uvw(N, M, L, "gaussian", 0.25, N / (2 * L * L), np.random.default_rng(11))
    G = build(plan, u, v, w, E)
    check_rows(G, u, v, w, E, s, range(M))


def test_invalid_visibilities_raise():
    N = 64
    plan = wp.Plan(N, L)
    B = N / (2 * L)
    good = np.array([0.0, 1.0, 2.0])
    with pytest.raises(wp.WprojError, match="WP_EINVAL"):
        wp.build_G(plan, dev(np.array([0.0, 1.1 * B, 0.0])), dev(good), dev(good), 0.9)
    with pytest.raises(wp.WprojError, match="WP_EINVAL"):
        wp.build_G(plan, dev(good), dev(good), dev(np.array([0.0, np.nan, 1.0])), 0.9)
    with pytest.raises(wp.WprojError, match="WP_EINVAL"):
        wp.build_G(plan, dev(good), dev(good), dev(good), 1.5)


# --------------------------------------------------------------------------- exact chirp (Eq. 4)

def test_exact_chirp_tiny_form_all_rows_and_operator():
    wl = synth.workload(0)
    say(f"build exact chirp: {wl.name} N={wl.N} M={wl.M}")
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L, kind="exact")
    plan = wp.Plan(wl.N, wl.L, chirp=wp.WP_CHIRP_EXACT)
    G = build(plan, u, v, w, wl.E)
    Go = wproj.build_rows(u, v, w, wl.E, s)
    assert abs(G.nnz - Go.nnz) <= 1e-6 * Go.nnz
    check_rows(G, u, v, w, wl.E, s, range(wl.M))
    G.order = wp.WP_ORDER_CALLER
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y, wproj.phi(Go, x, s)) < TOL
    r = synth.random_complex(wl.M, np.random.default_rng(5))
    xa = wp.apply_PhiT(plan, G, c64(r)).cpu().numpy().reshape(wl.N, wl.N)
    assert relerr(xa, wproj.phi_adjoint(Go, r, s)) < TOL


@pytest.mark.parametrize("E", [0.5, 1.0])
def test_exact_chirp_wide_field(E):
    """L = 0.5: the exact and linear chirps differ (O(w r^4)); E = 1 keeps every non-zero entry."""
    N, M, Lw = 64, 96, 0.5
    say(f"build exact chirp: wide field N={N} M={M} L={Lw} E={E}")
    s = Setup(N=N, L=Lw, kind="exact")
    u, v, w = synth.uvw(N, M, Lw, "uniform", 0.0, N / (2 * Lw * Lw), np.random.default_rng(21))
    plan = wp.Plan(N, Lw, chirp=wp.WP_CHIRP_EXACT)
    G = build(plan, u, v, w, E)
    check_rows(G, u, v, w, E, s, range(M))
    # the linear chirp's operator differs at this field size
    plan_lin = wp.Plan(N, Lw)
    G_lin = build(plan_lin, u, v, w, E)
    G.order = G_lin.order = wp.WP_ORDER_CALLER
    x = c64(np.random.default_rng(22).normal(size=(N, N)))
    y = wp.apply_Phi(plan, G, x).cpu().numpy()
    assert relerr(wp.apply_Phi(plan_lin, G_lin, x).cpu().numpy(), y) > 1e-3


def test_exact_chirp_plain_form_sampled_rows():
    wl = synth.workload(1)
    M = 4096
    say(f"build exact chirp: {wl.name} N={wl.N} first {M} visibilities (sampled rows)")
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    u, v, w = u[:M], v[:M], w[:M]
    s = Setup(N=wl.N, L=wl.L, kind="exact")
    plan = wp.Plan(wl.N, wl.L, chirp=wp.WP_CHIRP_EXACT)
    G = build(plan, u, v, w, wl.E)
    rows = np.unique(np.concatenate([synth.subset_rows(M, 20, synth.rng_for(wl.seed, "subset")), [0, M - 1]]))
    check_rows(G, u, v, w, wl.E, s, rows)
    rp, col, _, perm, _ = gpu_rows(G)
    assert np.array_equal(np.sort(perm), np.arange(M))
    assert rp[-1] == G.nnz and np.all(np.diff(rp) > 0) and col.max() < s.Ng ** 2


@pytest.mark.parametrize("taps", ["bf16", "i16"])
def test_exact_chirp_precision_forms(taps):
    wl = synth.workload(0)
    x, u, v, w = synth.workload_inputs(wl)
    plan = wp.Plan(wl.N, wl.L, chirp=wp.WP_CHIRP_EXACT)
    t = {"bf16": wp.WP_TAPS_BF16, "i16": wp.WP_TAPS_I16}[taps]
    G = build(plan, u, v, w, wl.E, taps=t)
    G.order = wp.WP_ORDER_CALLER
    s = Setup(N=wl.N, L=wl.L, kind="exact")
    Go = wproj.build_rows(u, v, w, wl.E, s)
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    y_ref = wproj.phi(Go, x, s)
    tol = {"bf16": 1.5 * bf16_rms_bound(Go, wproj.grid_forward(x, s).ravel(), False, y_ref) + TOL,
           "i16": 1e-4}[taps]
    assert relerr(y, y_ref) < tol


def test_exact_chirp_limits():
    z = np.zeros(3)
    with pytest.raises(wp.WprojError, match="WP_EUNSUPPORTED"):      # Ng = 1024 > 512: a window of each row, E < 1
        wp.build_G(wp.Plan(512, L, chirp=wp.WP_CHIRP_EXACT), dev(z), dev(z), dev(z), 1.0)
    big = wp.Plan(512, L, chirp=wp.WP_CHIRP_EXACT)
    big.set_tuning("exact_rows", 2)                                  # whole 2-D rows asked for at Ng = 1024
    with pytest.raises(wp.WprojError, match="WP_EUNSUPPORTED"):
        wp.build_G(big, dev(z), dev(z), dev(z), 0.9)
    with pytest.raises(wp.WprojError, match="WP_EINVAL"):            # 2 L^2 >= 1
        wp.build_G(wp.Plan(64, 0.75, chirp=wp.WP_CHIRP_EXACT), dev(z), dev(z), dev(z), 0.9)
    with pytest.raises(wp.WprojError, match="WP_EUNSUPPORTED"):      # rows are not separable
        wp.build_G(wp.Plan(64, L, chirp=wp.WP_CHIRP_EXACT), dev(z), dev(z), dev(z), 0.9, factors=True)


# --------------------------------------------------------------------------- direction-dependent effect

def _beams(M, Lf, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-0.2, 0.2, M) * Lf, rng.uniform(-0.2, 0.2, M) * Lf,
                     rng.uniform(0.3, 0.8, M) * Lf], axis=1)


@pytest.mark.parametrize("chirp", ["linear", "exact"])
def test_dde_rows_and_operator_match_oracle(chirp):
    wl = synth.workload(0)
    say(f"build with beams: {wl.name} N={wl.N} M={wl.M} chirp={chirp}")
    x, u, v, w = synth.workload_inputs(wl)
    beam = _beams(wl.M, wl.L, 51)
    s = Setup(N=wl.N, L=wl.L, kind=chirp)
    plan = wp.Plan(wl.N, wl.L, chirp=wp.WP_CHIRP_EXACT if chirp == "exact" else wp.WP_CHIRP_LINEAR)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E, beam=dev(beam))
    torch.cuda.synchronize()
    Go = wproj.build_rows(u, v, w, wl.E, s, beam=beam)
    assert abs(G.nnz - Go.nnz) <= 1e-6 * Go.nnz
    check_rows(G, u, v, w, wl.E, s, range(0, wl.M, 3), beam=beam)
    G.order = wp.WP_ORDER_CALLER
    y = wp.apply_Phi(plan, G, c64(x)).cpu().numpy()
    assert relerr(y, wproj.phi(Go, x, s)) < TOL
    r = synth.random_complex(wl.M, np.random.default_rng(52))
    xa = wp.apply_PhiT(plan, G, c64(r)).cpu().numpy().reshape(wl.N, wl.N)
    assert relerr(xa, wproj.phi_adjoint(Go, r, s)) < TOL


def test_dde_invalid_beams_and_limits():
    N = 64
    plan = wp.Plan(N, L)
    z = np.zeros(3)
    for bad in ([0.0, 0.0, 0.0], [0.0, np.nan, 0.01], [np.inf, 0.0, 0.01]):
        beam = np.tile([0.0, 0.0, 0.01], (3, 1))
        beam[1] = bad
        with pytest.raises(wp.WprojError, match="WP_EINVAL"):
            wp.build_G(plan, dev(z), dev(z), dev(z), 0.9, beam=dev(beam))
    with pytest.raises(wp.WprojError, match="WP_EUNSUPPORTED"):       # Ng = 1024 > 512
        wp.build_G(wp.Plan(512, L), dev(z), dev(z), dev(z), 0.9, beam=dev(np.tile([0.0, 0.0, 0.01], (3, 1))))
