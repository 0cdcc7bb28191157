"""GPU parity of SARA (Section 4.2's third dictionary): the nine-basis transforms and the
reweighted solve against the oracle."""
import numpy as np
import pytest

import synth
from oracle import metrics, sara, solver, wproj
from oracle.wproj import Setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("N,levels", [(64, 4), (32, 2), (256, 4), (128, 5)])
def test_sara_transforms_match_oracle(N, levels):
    print(f"sara transforms N={N} levels={levels}", flush=True)
    plan = wp.Plan(N, synth.fov_L())
    rng = np.random.default_rng(N + levels)
    x = rng.normal(size=(N, N))
    c = wp.sara_analysis(plan, f32(x), levels).cpu().numpy().reshape(9, N, N)
    assert relerr(c, sara.analysis(x, levels)) < 1e-5
    assert relerr(wp.sara_synthesis(plan, f32(c), levels).cpu().numpy().reshape(N, N), x) < 1e-5
    d = rng.normal(size=(9, N, N))
    assert relerr(wp.sara_synthesis(plan, f32(d), levels).cpu().numpy().reshape(N, N), sara.synthesis(d, levels)) < 1e-5


def test_sara_levels_rejected():
    plan = wp.Plan(64, synth.fov_L())
    x = f32(np.zeros((64, 64)))
    for bad in (0, 5):
        with pytest.raises(wp.WprojError, match="WP_EINVAL"):
            wp.sara_analysis(plan, x, bad)


def _problem():
    wl = synth.workload(0)
    x, u, v, w = synth.workload_inputs(wl)
    s = Setup(N=wl.N, L=wl.L)
    Go = wproj.build_rows(u, v, w, wl.E, s)
    A = lambda z: wproj.phi(Go, z, s)
    AH = lambda r: wproj.phi_adjoint(Go, r, s)
    y0 = A(x)
    sig = metrics.noise_sigma(y0, wl.snr_in_db)
    y = y0 + synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise"))
    eps = metrics.l2_ball_radius(sig, wl.M)
    x0 = synth.rng_for(wl.seed, "x").normal(size=(wl.N, wl.N))
    nu = solver.power_norm2(A, AH, x0, 50)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(w).cuda(), wl.E)
    G.order = wp.WP_ORDER_CALLER
    yd = torch.from_numpy(y.astype(np.complex64)).cuda()
    return wl, x, A, AH, y, eps, nu, plan, G, yd


def test_sara_solve_matches_oracle():
    wl, x, A, AH, y, eps, nu, plan, G, yd = _problem()
    print(f"sara solve: {wl.name}", flush=True)
    # early iterates of two rounds (the second with weights) agree closely
    xg = wp.sara_solve(plan, G, yd, eps, nu, 6, 2).cpu().numpy().reshape(wl.N, wl.N)
    xr, _ = sara.solve(y, A, AH, (wl.N, wl.N), eps, nu, 6, rounds=2)
    assert relerr(xg, xr) < 1e-3
    # a full reweighted solve reaches the oracle's quality
    xg = wp.sara_solve(plan, G, yd, eps, nu, 80, 3).cpu().numpy().reshape(wl.N, wl.N)
    xr, _ = sara.solve(y, A, AH, (wl.N, wl.N), eps, nu, 80, rounds=3)
    snr_g, snr_r = metrics.snr_out(x, xg), metrics.snr_out(x, xr)
    print(f"SARA SNR_out gpu {snr_g:.3f} dB, oracle {snr_r:.3f} dB", flush=True)
    assert abs(snr_g - snr_r) < 0.1
    assert np.all(xg >= 0)
