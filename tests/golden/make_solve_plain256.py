"""Write solve_plain256.json: the FP64 oracle's reconstruction of the plain 256-pixel form.

Test infrastructure: calls only `oracle/` (and the seeded input generators of `synth/`).  The
plain form's operator (N = 256, M = 32768 Gaussian (u, v), E = 0.99) applied to the seeded sky,
30 dB of visibility-domain noise, ||Phi||^2 by 50 power-iteration steps from the seeded start,
then 500 primal-dual iterations of the l1-analysis problem of Eq. 7 (Daubechies 8, 4 levels,
positivity), as `wp_solve` runs them.  The GPU test compares its own solve of the same problem
with the SNR recorded here (within 0.1 dB).

    python tests/golden/make_solve_plain256.py [--workers 8]

The oracle's rows take about 100 s of one core; the 500 iterations about 75 s.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import metrics, solver, wproj  # noqa: E402
from oracle.wproj import Setup  # noqa: E402

OUT = os.path.join(HERE, "solve_plain256.json")


def oracle_G(u, v, w, E, s, workers):
    chunks = np.array_split(np.arange(u.size), workers * 4)
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(wproj.build_rows_csr_parts, [(u[c], v[c], w[c], E, s, None) for c in chunks])
    return sp.vstack([sp.csr_matrix((d, i, p), shape=(n, s.Ng * s.Ng)) for p, i, d, n in parts]).tocsr()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    wl = synth.workload(1)
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L, W=wl.W)
    t0 = time.time()
    Go = oracle_G(u, v, w, wl.E, s, args.workers)
    print(f"oracle rows: nnz {Go.nnz} in {time.time() - t0:.1f} s", flush=True)
    A = lambda z: wproj.phi(Go, z, s)
    AH = lambda r: wproj.phi_adjoint(Go, r, s)
    y0 = A(x)
    sig = metrics.noise_sigma(y0, wl.snr_in_db)
    y = y0 + synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise"))
    eps = metrics.l2_ball_radius(sig, wl.M)
    x0 = synth.rng_for(wl.seed, "x").normal(size=(wl.N, wl.N))
    nu = solver.power_norm2(A, AH, x0, 50)
    t0 = time.time()
    xr, hist = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, wl.iters, levels=4, history=True, x_true=x)
    print(f"oracle solve: {wl.iters} iterations in {time.time() - t0:.1f} s, SNR {hist[-1]:.4f} dB", flush=True)
    res = float(np.linalg.norm(y - A(xr)))
    rec = {
        "what": "FP64 oracle solve of the plain 256-pixel form (Eq. 7, primal-dual, Daubechies 8, 4 levels, "
                "positivity), written by tests/golden/make_solve_plain256.py from oracle/ only",
        "workload": wl.name, "N": wl.N, "M": wl.M, "E": wl.E, "iterations": wl.iters, "snr_in_db": wl.snr_in_db,
        "noise": "sigma_n = 10^(-snr_in/20) rms(Phi x), eps^2 = sigma_n^2 (M + 2 sqrt M)",
        "power_iterations": 50, "nu": nu, "sigma_n": sig, "eps": eps, "nnz": int(Go.nnz),
        "snr_out_db": hist[-1], "snr_out_db_at": {str(k): hist[k - 1] for k in (50, 100, 200, 300, 400, 500)},
        "residual_norm": res, "x_rec_sum": float(xr.sum()), "x_rec_max": float(xr.max()),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
