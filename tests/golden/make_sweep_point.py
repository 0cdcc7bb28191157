"""Write sweep_point.json: one point of Section 4's experiments computed by the FP64 oracle alone.

Test infrastructure: calls only `oracle/` and the seeded input generators of `synth/`.  The point is the
coverage experiment of Section 4.2 at the tiny form's geometry (N = 64, Ng = 128, the seeded 10-blob /
20-point sky): 10 % coverage (M = 0.1 Ng^2 visibilities uniform in the band), w = w_d w_max with
w_d ~ U(0, 1) and w_max = N / (2 L^2), data from the E = 1 operator plus 30 dB visibility-domain noise,
reconstruction with the operator sparsified at E = 0.99 (200 primal-dual iterations, Daubechies 8,
4 levels, positivity), the same protocol as `bench.py --sweep coverage` runs on the GPU.

    python tests/golden/make_sweep_point.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import metrics, solver, wproj  # noqa: E402
from oracle.wproj import Setup  # noqa: E402

OUT = os.path.join(HERE, "sweep_point.json")
COVERAGE, E, ITERS = 0.1, 0.99, 200


def main():
    wl = synth.workload(0)
    N, L = wl.N, wl.L
    Ng = 2 * N
    s = Setup(N=N, L=L)
    x = synth.sky(N, wl.n_blobs, wl.n_points, synth.rng_for(wl.seed, "sky"))
    M = int(round(COVERAGE * Ng * Ng))
    rng = synth.rng_for(wl.seed, "sweep", int(1000 * COVERAGE))
    u, v, _ = synth.uvw(N, M, L, "uniform", 0.0, 0.0, rng)
    w = rng.uniform(0.0, N / (2 * L * L), M)
    t0 = time.time()
    G1 = wproj.build_rows(u, v, w, 1.0, s)
    y0 = wproj.phi(G1, x, s)
    sig = metrics.noise_sigma(y0, 30.0)
    y = y0 + synth.noise(M, sig, synth.rng_for(wl.seed, "noise", int(1000 * COVERAGE)))
    G = wproj.build_rows(u, v, w, E, s)
    print(f"oracle rows: E = 1 nnz {G1.nnz}, E = {E} nnz {G.nnz} in {time.time() - t0:.1f} s", flush=True)
    A = lambda z: wproj.phi(G, z, s)
    AH = lambda r: wproj.phi_adjoint(G, r, s)
    eps = metrics.l2_ball_radius(sig, M)
    x0 = synth.rng_for(wl.seed, "x").normal(size=(N, N))
    nu = solver.power_norm2(A, AH, x0, 50)
    xr = solver.solve(y, A, AH, (N, N), eps, nu, ITERS, levels=4)
    snr = metrics.snr_out(x, xr)
    print(f"oracle solve: SNR {snr:.4f} dB", flush=True)
    rec = {"what": "Section 4.2 coverage experiment, one point, FP64 oracle only (tests/golden/make_sweep_point.py)",
           "N": N, "coverage": COVERAGE, "M": M, "w_d": "U(0,1)", "E": E, "iterations": ITERS, "basis": "db8",
           "nnz_E1": int(G1.nnz), "nnz": int(G.nnz), "nnz_fraction": G.nnz / (M * Ng * Ng), "sigma_n": sig,
           "nu": nu, "snr_out_db": snr}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
