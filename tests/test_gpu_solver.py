"""GPU parity of the reconstruction path: Daubechies-8 transforms, power iteration, full solve."""
import numpy as np
import pytest

import synth
from oracle import metrics, solver, wavelet, wproj
from oracle.wproj import Setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()


def c64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64).ravel()).cuda()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("N,levels", [(64, 4), (256, 4), (128, 2), (32, 3), (64, 0), (1024, 4), (512, 5), (256, 1)])
def test_dwt_matches_oracle(N, levels):
    print(f"dwt N={N} levels={levels}", flush=True)
    plan = wp.Plan(N, synth.fov_L())
    x = np.random.default_rng(N + levels).normal(size=(N, N))
    c = wp.dwt2(plan, f32(x), levels).cpu().numpy().reshape(N, N)
    assert relerr(c, wavelet.dwt2(x, levels)) < 1e-5
    xr = wp.idwt2(plan, f32(c), levels).cpu().numpy().reshape(N, N)
    assert relerr(xr, x) < 1e-5
    cc = np.random.default_rng(N).normal(size=(N, N))
    assert relerr(wp.idwt2(plan, f32(cc), levels).cpu().numpy().reshape(N, N), wavelet.idwt2(cc, levels)) < 1e-5


@pytest.mark.parametrize("N,levels", [(64, 4), (256, 3)])
def test_dwt_in_place_matches_oracle(N, levels):
    """x and c may alias: the in-place form runs one pass per axis and level through the scratch."""
    plan = wp.Plan(N, synth.fov_L())
    x = np.random.default_rng(N + 7).normal(size=(N, N))
    xd = f32(x)
    wp.dwt2(plan, xd, levels, out=xd)
    assert relerr(xd.cpu().numpy().reshape(N, N), wavelet.dwt2(x, levels)) < 1e-5
    c = xd.cpu().numpy().reshape(N, N).astype(np.float64)
    wp.idwt2(plan, xd, levels, out=xd)
    assert relerr(xd.cpu().numpy().reshape(N, N), wavelet.idwt2(c, levels)) < 1e-5
    assert relerr(xd.cpu().numpy().reshape(N, N), x) < 1e-5


def _tiny_problem():
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
    return wl, x, u, v, w, s, A, AH, y, eps, x0


def test_power_norm_matches_oracle():
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    nu_gpu = wp.power_norm2(plan, G, f32(x0), 50)
    nu_ref = solver.power_norm2(A, AH, x0, 50)
    assert abs(nu_gpu - nu_ref) / nu_ref < 1e-5


@pytest.mark.parametrize("order", ["caller", "sorted"])
def test_solve_tiny_form_matches_oracle(order):
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    print(f"solve: {wl.name} {wl.iters} iterations, order={order}", flush=True)
    nu = solver.power_norm2(A, AH, x0, 50)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    yd = c64(y)
    if order == "sorted":
        yd = wp.to_sorted(G, yd)
        G.order = wp.WP_ORDER_SORTED
    # early iterates agree closely
    x5 = wp.solve(plan, G, yd, eps, nu, 5).cpu().numpy().reshape(wl.N, wl.N)
    x5_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, 5)
    assert relerr(x5, x5_ref) < 1e-4
    xg = wp.solve(plan, G, yd, eps, nu, wl.iters).cpu().numpy().reshape(wl.N, wl.N)
    x_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, wl.iters)
    snr_g, snr_r = metrics.snr_out(x, xg), metrics.snr_out(x, x_ref)
    print(f"SNR_out gpu {snr_g:.3f} dB, oracle {snr_r:.3f} dB", flush=True)
    assert abs(snr_g - snr_r) < 0.1
    assert np.all(xg >= 0)


def test_solve_dirac_basis_matches_oracle():
    """levels = 0: the Dirac (pixel) basis of Section 4.2."""
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    print(f"solve dirac: {wl.name} {wl.iters} iterations", flush=True)
    nu = solver.power_norm2(A, AH, x0, 50)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    yd = c64(y)
    x5 = wp.solve(plan, G, yd, eps, nu, 5, levels=0).cpu().numpy().reshape(wl.N, wl.N)
    x5_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, 5, levels=0)
    assert relerr(x5, x5_ref) < 1e-4
    xg = wp.solve(plan, G, yd, eps, nu, wl.iters, levels=0).cpu().numpy().reshape(wl.N, wl.N)
    x_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, wl.iters, levels=0)
    snr_g, snr_r = metrics.snr_out(x, xg), metrics.snr_out(x, x_ref)
    print(f"SNR_out dirac gpu {snr_g:.3f} dB, oracle {snr_r:.3f} dB", flush=True)
    assert abs(snr_g - snr_r) < 0.1
    assert np.all(xg >= 0)
    # the two dictionaries give different estimates
    xw = wp.solve(plan, G, yd, eps, nu, 5).cpu().numpy().reshape(wl.N, wl.N)
    assert relerr(xw, x5) > 1e-3


def test_levels_rejected():
    plan = wp.Plan(64, synth.fov_L())
    x = f32(np.zeros((64, 64)))
    for bad in (-1, 5):          # 64 >> 4 = 4 < 8 samples per line at the coarsest level
        with pytest.raises(wp.WprojError):
            wp.dwt2(plan, x, bad)


@pytest.mark.parametrize("levels", [4, 0])
def test_douglas_rachford_matches_oracle(levels):
    """Douglas-Rachford for Eq. 7 without positivity (Section 2.3)."""
    from oracle import dr
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    print(f"douglas-rachford: {wl.name} levels={levels}", flush=True)
    nu = solver.power_norm2(A, AH, x0, 50)
    gamma = 0.01 * np.abs(wavelet.dwt2(np.real(AH(y)) / nu, levels)).max()
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    G.order = wp.WP_ORDER_CALLER
    yd = c64(y)
    xg = wp.dr_solve(plan, G, yd, eps, nu, 4, 3, gamma, levels).cpu().numpy().reshape(wl.N, wl.N)
    xr = dr.solve(y, A, AH, (wl.N, wl.N), eps, nu, 4, 3, gamma, levels)
    assert relerr(xg, xr) < 1e-4
    xg = wp.dr_solve(plan, G, yd, eps, nu, 60, 3, gamma, levels).cpu().numpy().reshape(wl.N, wl.N)
    xr = dr.solve(y, A, AH, (wl.N, wl.N), eps, nu, 60, 3, gamma, levels)
    print(f"DR SNR_out gpu {metrics.snr_out(x, xg):.3f} dB, oracle {metrics.snr_out(x, xr):.3f} dB", flush=True)
    assert relerr(xg, xr) < 1e-3
    assert abs(metrics.snr_out(x, xg) - metrics.snr_out(x, xr)) < 0.05


def test_solve_plain_form_matches_oracle_snr():
    """The plain 256-pixel form's 500-iteration solve against the FP64 oracle's solve of the same
    problem (tests/golden/solve_plain256.json, written by make_solve_plain256.py from oracle/ only):
    the same sky, noise draw, ball radius and power-iteration start; SNR_out within 0.1 dB."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "solve_plain256.json")))
    wl = synth.workload(1)
    x, u, v, w = synth.workload_inputs(wl)
    print(f"solve: {wl.name} {wl.iters} iterations against the oracle's SNR {ref['snr_out_db']:.3f} dB", flush=True)
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    y0 = wp.apply_Phi(plan, G, c64(x)).cpu().numpy().astype(np.complex128)
    sig = metrics.noise_sigma(y0, wl.snr_in_db)
    assert abs(sig - ref["sigma_n"]) < 1e-5 * ref["sigma_n"]          # same data as the oracle's
    y = y0 + synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise"))
    eps = metrics.l2_ball_radius(sig, wl.M)
    x0 = synth.rng_for(wl.seed, "x").normal(size=(wl.N, wl.N))
    nu = wp.power_norm2(plan, G, f32(x0), 50)
    assert abs(nu - ref["nu"]) < 1e-4 * ref["nu"]
    G.order = wp.WP_ORDER_SORTED
    yd = wp.to_sorted(G, c64(y))
    xg = wp.solve(plan, G, yd, eps, nu, wl.iters).cpu().numpy().reshape(wl.N, wl.N)
    snr_g = metrics.snr_out(x, xg)
    print(f"SNR_out gpu {snr_g:.3f} dB, oracle {ref['snr_out_db']:.3f} dB", flush=True)
    assert abs(snr_g - ref["snr_out_db"]) < 0.1
    assert np.all(xg >= 0)


def test_solve_two_streams_match_one():
    """With wavelets the loop can run on two streams (the analysis of xb and the next synthesis up to
    its last level beside Phi xb, the ball step and Phi^H v2): the same kernels on the same buffers in
    an order the events fix, so the iterates equal the one-stream loop's; twice in a row, with eager
    work on the caller's stream in between."""
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    yd = c64(y)
    nu = solver.power_norm2(A, AH, x0, 50)
    plan.set_tuning("solve_streams", 1)
    ref = wp.solve(plan, G, yd, eps, nu, 40, levels=4).cpu().numpy()
    plan.set_tuning("solve_streams", 2)
    for rep in range(2):
        got = wp.solve(plan, G, yd, eps, nu, 40, levels=4).cpu().numpy()
        assert relerr(got, ref) < 1e-6, rep
        wp.apply_Phi(plan, G, c64(x))
        torch.cuda.synchronize()
    x_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, 40, levels=4)
    assert relerr(ref.reshape(wl.N, wl.N), x_ref) < 1e-4


@pytest.mark.parametrize("levels", [4, 0])
def test_solve_graph_replays_match_direct_launches(levels):
    """The solver loop replayed from a captured HIP graph (chunks of 10 iterations) against the same
    iterations launched one by one: identical iterates, for 35 iterations (three replays and five
    direct ones) and again after eager work on the same stream in between."""
    wl, x, u, v, w, s, A, AH, y, eps, x0 = _tiny_problem()
    plan = wp.Plan(wl.N, wl.L)
    G = wp.build_G(plan, dev(u), dev(v), dev(w), wl.E)
    yd = c64(y)
    nu = solver.power_norm2(A, AH, x0, 50)
    plan.set_tuning("solve_graph", 2)
    plan.set_tuning("solve_streams", 1)              # the graph captures the one-stream loop
    ref = wp.solve(plan, G, yd, eps, nu, 35, levels=levels).cpu().numpy()
    plan.set_tuning("solve_graph", 1)
    for rep in range(3):
        got = wp.solve(plan, G, yd, eps, nu, 35, levels=levels).cpu().numpy()
        assert np.array_equal(got, ref), rep
        wp.apply_Phi(plan, G, c64(x))                 # eager work between the replays
        torch.cuda.synchronize()
    x_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu, 35, levels=levels)
    assert relerr(ref.reshape(wl.N, wl.N), x_ref) < 1e-4
