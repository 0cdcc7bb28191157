"""The exact operator of the 2048-pixel form (N = 2048, Ng = 4096, M = 16 777 216, supports to 32
cells) at full size, in the launch forms the benchmark times, against the FP64 oracle on a seeded
4096-visibility subset: Phi from the factor records and from the stored taps, Phi^H through the
blocked gather over the transposed copy (cells average about 210 entries) and through the
per-cell gather; then the factor-record form (no stored taps, no transposed copy: Phi from the
records, Phi^H scattered from them).  G holds about 3.5e9 taps, so row and cell offsets run past 2^31.

Tolerance: 1e-5 (the FP32 target), against the oracle's rows with the same (W, beta, E, chirp).
"""
import numpy as np
import pytest

import synth
from oracle import wproj
from oracle.wproj import Setup

from helpers import oracle_rows, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402

ROWS = 4096


def test_surrogate_form_exact_operator_full_size():
    wl = synth.workload(4)
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    rows = synth.subset_rows(wl.M, ROWS, synth.rng_for(wl.seed, "subset"))
    print(f"full size {wl.name}: oracle rows {ROWS}", flush=True)
    Go = oracle_rows(u, v, w, wl.E, s, rows)
    y_ref = Go @ wproj.grid_forward(x, s).ravel()
    ys = synth.random_complex(ROWS, synth.rng_for(wl.seed, "y", 4))
    x_ref = wproj.phi_adjoint(Go, ys, s)
    print(f"full size {wl.name}: building G on the GPU", flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, t(u), t(v), t(w), wl.E, transpose=True, factors=True)
    torch.cuda.synchronize()
    assert G.nnz > 2 ** 31 and G.tblk is not None
    assert abs(G.nnz / wl.M - Go.nnz / ROWS) < 0.05 * Go.nnz / ROWS     # the subset is representative
    # the subset's rows sit across the whole sorted order, so their offsets span the int32 range
    perm = G.perm.cpu().numpy()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    rp = G.rowptr.cpu().numpy()
    assert rp[inv[rows]].max() > 2 ** 31
    xd = t(x.astype(np.complex64).ravel())
    for fac in (True, False):
        G.use_factors = fac
        y = wp.apply_Phi(plan, G, xd).cpu().numpy()[rows]
        e = relerr(y, y_ref)
        print(f"full size: Phi ({'factor records' if fac else 'stored taps'}) rel err {e:.3e}", flush=True)
        assert e < 1e-5, fac
    yfull = np.zeros(wl.M, dtype=np.complex64)
    yfull[rows] = ys
    yfd = t(yfull)
    for blocks in (True, False):
        G.use_blocks = blocks
        xa = wp.apply_PhiT(plan, G, yfd).cpu().numpy().reshape(wl.N, wl.N)
        e = relerr(xa, x_ref)
        print(f"full size: Phi^H ({'blocked' if blocks else 'per-cell'} gather) rel err {e:.3e}", flush=True)
        assert e < 1e-5, blocks
    stored_bytes = G.nbytes()
    del G
    torch.cuda.empty_cache()
    # the factor-record form: no stored taps, no transposed copy; Phi^H scattered from the records
    print(f"full size {wl.name}: factor-record form", flush=True)
    G = wp.build_G(plan, t(u), t(v), t(w), wl.E, transpose=False, factors=True, stored=False)
    torch.cuda.synchronize()
    assert G.nbytes() < 0.1 * stored_bytes
    e = relerr(wp.apply_Phi(plan, G, xd).cpu().numpy()[rows], y_ref)
    xa = wp.apply_PhiT(plan, G, yfd).cpu().numpy().reshape(wl.N, wl.N)
    e2 = relerr(xa, x_ref)
    print(f"full size: record form Phi rel err {e:.3e}, Phi^H (scatter from records) rel err {e2:.3e}, "
          f"{G.nbytes() / 1e9:.1f} GB against {stored_bytes / 1e9:.1f} GB", flush=True)
    assert e < 1e-5 and e2 < 1e-5
    del G
    torch.cuda.empty_cache()
    plan.close()
