"""Benchmark: visibilities/s of Phi + Phi^H on one MI355X, with roofline and a CPU-oracle baseline.

A step is one Phi (apodise, pad, FFT, degrid SpMV) followed by one Phi^H
(tiled gridding scatter, inverse FFT, crop, apodise) over all M visibilities of
the plain FP32 workload (N = 256, M = 32768, E = 0.99, supports 4..32 cells).
G is built once on the GPU before timing (its build time is reported apart).
Inputs are resident in HBM when the timed region starts.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=1)
    ap.add_argument("--taps", choices=["c64", "bf16"], default="c64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=384)
    return ap.parse_args()


def degrid_bytes(G, M, Ng, tap_bytes):
    """Algorithmic HBM bytes of one degrid launch: taps + indices once, rowptr, perm, y, one grid read."""
    return G.nnz * (tap_bytes + 4) + (M + 1) * 8 + M * 4 + M * 8 + Ng * Ng * 8


def scatter_bytes(G, M, Ng, tap_bytes):
    """Same stream as degrid plus the work list; the grid is written once (read y instead of writing it)."""
    return G.nnz * (tap_bytes + 4) + (M + 1) * 8 + M * 4 + M * 8 + Ng * Ng * 8 + G.n_work * 16


def gather_bytes(G, M, Ng, tap_bytes):
    """Transposed copy streamed once (value + visibility index), cell offsets, y read once, grid written once."""
    return G.nnz * (tap_bytes + 4) + (Ng * Ng + 1) * 8 + M * 8 + Ng * Ng * 8


def time_region(fn, steps, stream, torch):
    s_ev = torch.cuda.Event(enable_timing=True)
    e_ev = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s_ev.record(stream)
    for _ in range(steps):
        fn()
    e_ev.record(stream)
    torch.cuda.synchronize()
    return s_ev.elapsed_time(e_ev) / steps      # ms per call


def cpu_baseline(wl, x, u, v, w, rows_n):
    """The FP64 oracle's Phi + Phi^H on a bounded sample of rows, scaled to all M rows."""
    from oracle import wproj
    from oracle.wproj import Setup
    import synth
    s = Setup(N=wl.N, L=wl.L, W=wl.W)
    rows = synth.subset_rows(wl.M, rows_n, synth.rng_for(wl.seed, "subset", 9))
    Gs = wproj.build_rows(u, v, w, wl.E, s, rows=rows)          # setup, not timed
    yv = synth.random_complex(rows.size, synth.rng_for(wl.seed, "y", 9))
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        X = wproj.grid_forward(x, s)
    t_fft_fwd = (time.perf_counter() - t0) / reps
    Xf = X.ravel()
    t0 = time.perf_counter()
    for _ in range(reps):
        Gs @ Xf
    t_deg = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        Xa = (Gs.conj().T @ yv)
    t_grid = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        wproj.grid_adjoint(Xa.reshape(s.Ng, s.Ng), s)
    t_fft_adj = (time.perf_counter() - t0) / reps
    scale = wl.M / rows.size
    t_step = t_fft_fwd + t_fft_adj + scale * (t_deg + t_grid)
    return {"value": wl.M / t_step, "unit": "visibilities/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows.size} of {wl.M} rows (seeded subset), sparse products scaled x{scale:.1f}, "
                      f"full FP64 FFTs; NumPy FFT and SciPy CSR products are single-threaded",
            "cpu": platform.processor() or platform.machine(), "host_threads": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1307_3424_amd as wp
    import synth

    wl = synth.workload(args.workload)
    if wl.channels is not None:
        raise SystemExit("the batched form is benchmarked by its own script")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: workload {wl.name} N={wl.N} M={wl.M} E={wl.E} taps={args.taps}")
    x, u, v, w = synth.workload_inputs(wl)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    plan = wp.Plan(wl.N, wl.L, kb_W=wl.W)
    taps = wp.WP_TAPS_C64 if args.taps == "c64" else wp.WP_TAPS_BF16
    tap_bytes = 8 if taps == wp.WP_TAPS_C64 else 4
    ud, vd, wd = t(u), t(v), t(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = wp.build_G(plan, ud, vd, wd, wl.E, taps=taps)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"bench: G built in {build_s:.3f} s, nnz={G.nnz} ({G.nnz / wl.M:.1f}/vis), work items {G.n_work}")
    xd = t(x.astype(np.complex64).ravel())
    yd = torch.empty(wl.M, dtype=torch.complex64, device=dev)
    xa = torch.empty(wl.N * wl.N, dtype=torch.complex64, device=dev)
    grid = plan.new_grid()
    stream = torch.cuda.current_stream()
    # visibility vectors stay in G's sorted row order inside the timed loop (an iterative
    # solver permutes its data vector once); the caller-order cost is reported beside it
    G.order = wp.WP_ORDER_SORTED

    def step():
        wp.apply_Phi(plan, G, xd, yd, grid)
        wp.apply_PhiT(plan, G, yd, xa, grid)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = time_region(step, args.steps, stream, torch)
    log(f"bench: {ms * 1e3:.1f} us per Phi+Phi^H")
    # per-stage timings (same stream, HIP events around repeated launches of one stage)
    ks = max(20, args.steps)
    ms_phi = time_region(lambda: wp.apply_Phi(plan, G, xd, yd, grid), ks, stream, torch)
    ms_phit = time_region(lambda: wp.apply_PhiT(plan, G, yd, xa, grid), ks, stream, torch)
    ms_fwd = time_region(lambda: wp.grid_forward(plan, xd, grid), ks, stream, torch)
    wp.grid_forward(plan, xd, grid)
    ms_deg = time_region(lambda: wp.degrid(plan, G, grid, yd), ks, stream, torch)
    ms_sc = time_region(lambda: wp.grid_scatter(plan, G, yd, grid), ks, stream, torch)
    ms_ga = time_region(lambda: wp.grid_gather(plan, G, yd, grid), ks, stream, torch)
    G.use_transpose = False
    ms_phit_sc = time_region(lambda: wp.apply_PhiT(plan, G, yd, xa, grid), ks, stream, torch)
    G.use_transpose = True
    ms_adj = time_region(lambda: wp.grid_adjoint(plan, grid, xa), ks, stream, torch)
    G.order = wp.WP_ORDER_CALLER
    ms_caller = time_region(step, ks, stream, torch)
    G.order = wp.WP_ORDER_SORTED
    db = degrid_bytes(G, wl.M, plan.Ng, tap_bytes)
    sb = scatter_bytes(G, wl.M, plan.Ng, tap_bytes)
    deg_gbs = db / (ms_deg * 1e-3) / 1e9
    sc_gbs = sb / (ms_sc * 1e-3) / 1e9
    gb = gather_bytes(G, wl.M, plan.Ng, tap_bytes)
    ga_gbs = gb / (ms_ga * 1e-3) / 1e9
    log(f"bench: Phi {ms_phi * 1e3:.1f} us, Phi^H {ms_phit * 1e3:.1f} us | fwd FFT {ms_fwd * 1e3:.1f} us, "
        f"degrid {ms_deg * 1e3:.1f} us ({deg_gbs:.0f} GB/s), scatter+zero {ms_sc * 1e3:.1f} us ({sc_gbs:.0f} GB/s), "
        f"gather {ms_ga * 1e3:.1f} us ({ga_gbs:.0f} GB/s), Phi^H via scatter {ms_phit_sc * 1e3:.1f} us, "
        f"adj FFT {ms_adj * 1e3:.1f} us")
    out = {
        "metric": "visibilities/s for Phi+Phi† (exact vs surrogate kernels) and % HBM roofline",
        "value": wl.M / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64" if taps == wp.WP_TAPS_C64 else "bf16x2-taps/f32-accumulate",
        "data": "synthetic (seeded sky and baselines; the paper's M31 / 30Dor images are not used)",
        "config": {"workload": wl.name, "N": wl.N, "Ng": plan.Ng, "M": wl.M, "E": wl.E, "kb_W": wl.W,
                   "uv": f"{wl.uv} sigma={wl.uv_sigma}B", "w_top": wl.w_top, "kernel": "exact (stored G)",
                   "nnz": G.nnz, "nnz_per_vis": G.nnz / wl.M, "G_bytes": G.nbytes()},
        "roofline": {"bound": "hbm", "kernel": "degrid (Phi sparse product)", "achieved": deg_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": deg_gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": db, "launch_us": ms_deg * 1e3},
        "stages_us": {"phi": ms_phi * 1e3, "phiT": ms_phit * 1e3, "grid_forward": ms_fwd * 1e3,
                      "degrid": ms_deg * 1e3, "gather": ms_ga * 1e3, "scatter_incl_zero": ms_sc * 1e3,
                      "grid_adjoint": ms_adj * 1e3, "phiT_via_scatter": ms_phit_sc * 1e3,
                      "step_caller_order": ms_caller * 1e3},
        "gather_roofline": {"achieved": ga_gbs, "frac": ga_gbs / HBM_PEAK_GBS, "bytes_per_launch": gb},
        "scatter_roofline": {"achieved": sc_gbs, "frac": sc_gbs / HBM_PEAK_GBS, "bytes_per_launch": sb},
        "phi_vis_per_s": wl.M / (ms_phi * 1e-3), "phiT_vis_per_s": wl.M / (ms_phit * 1e-3),
        "build_G_s": build_s,
    }
    if not args.no_cpu:
        log("bench: timing the FP64 oracle on a bounded sample (CPU)")
        out["cpu_baseline"] = cpu_baseline(wl, x, u, v, w, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
