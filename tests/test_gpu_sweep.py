"""One point of Section 4's experiments on the GPU against the FP64 oracle's run of the same point
(tests/golden/sweep_point.json, written by make_sweep_point.py from oracle/ only): the coverage experiment
at 10 % coverage, w_d ~ U(0, 1), E = 0.99, Daubechies 8, 200 iterations, in the protocol of
`bench.py --sweep coverage`.  The non-zero counts of the sparsified operators are integers and must match
exactly; the reconstruction SNR within 0.1 dB.  (The paper's printed SNRs need its test images and stay
unpinned.)"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402


def test_coverage_sweep_point_matches_oracle():
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sweep_point.json")))
    wl = synth.workload(0)
    N, L = wl.N, wl.L
    cov, E = ref["coverage"], ref["E"]
    x = synth.sky(N, wl.n_blobs, wl.n_points, synth.rng_for(wl.seed, "sky"))
    M = ref["M"]
    rng = synth.rng_for(wl.seed, "sweep", int(1000 * cov))
    u, v, _ = synth.uvw(N, M, L, "uniform", 0.0, 0.0, rng)
    w = rng.uniform(0.0, N / (2 * L * L), M)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = wp.Plan(N, L)
    G1 = wp.build_G(plan, t(u), t(v), t(w), 1.0, transpose=False)
    assert G1.nnz == ref["nnz_E1"]
    y0 = wp.apply_Phi(plan, G1, t(x.astype(np.complex64).ravel())).cpu().numpy().astype(np.complex128)
    sig = metrics.noise_sigma(y0, 30.0)
    assert abs(sig - ref["sigma_n"]) < 1e-5 * ref["sigma_n"]
    y = y0 + synth.noise(M, sig, synth.rng_for(wl.seed, "noise", int(1000 * cov)))
    G = wp.build_G(plan, t(u), t(v), t(w), E)
    assert G.nnz == ref["nnz"]
    G.order = wp.WP_ORDER_SORTED
    ys = wp.to_sorted(G, t(y.astype(np.complex64)))
    eps = metrics.l2_ball_radius(sig, M)
    x0 = t(synth.rng_for(wl.seed, "x").normal(size=(N, N)).astype(np.float32).ravel())
    nu = wp.power_norm2(plan, G, x0, 50)
    assert abs(nu - ref["nu"]) < 1e-4 * ref["nu"]
    xr = wp.solve(plan, G, ys, eps, nu, ref["iterations"]).cpu().numpy().reshape(N, N)
    snr = metrics.snr_out(x, xr)
    print(f"sweep point: nnz {G.nnz} (oracle {ref['nnz']}), SNR gpu {snr:.3f} dB, oracle {ref['snr_out_db']:.3f} dB",
          flush=True)
    assert abs(snr - ref["snr_out_db"]) < 0.1
