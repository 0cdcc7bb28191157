"""Benchmark: visibilities/s of Phi + Phi^H on one MI355X, exact and surrogate kernels, with the roofline
of the dominant kernel and the FP64 CPU oracle timed beside it.

Default workload: the learned-surrogate form (N = 2048, Ng = 4096, M = 16 777 216 Gaussian (u, v), w up to
supports of 32 cells, E = 0.99).  A step is one Phi followed by one Phi^H over all M visibilities, with the
visibility vectors resident in HBM in the operator's own order:

* exact form: apodisation, zero-padding and FFT, then the degrid (from the factor records, taps formed in
  registers, or from the stored taps: whichever times faster before the timed loop); Phi^H: the gather over
  the transposed copy (one wavefront per block of cells), inverse FFT, crop, apodisation;
* surrogate form: the same transforms; rows that pass the run-time check (from the check lattice, no exact
  row) through the network's per-cell output-layer products (bfloat16 MFMA, FP32 accumulation), the other
  rows through an exact G of their own.

`value` is the surrogate form's rate (the workload's form); the exact form's rate, their ratio, both
reconstructions' SNR (200 iterations from the same data), per-stage times, the MFMA roofline of the
surrogate's dominant product and the HBM rooflines of the exact products are in the same line.  The plain
256-pixel form's figures ride along under "plain_256" (--no-plain drops them).

Other forms: --workload 1 (plain 256, with its 500-iteration solve), 2 (precision, --taps c64|bf16|i16),
3 (batched, 48 x 512: one persistent launch per product against 48 sequential launches); --sweep runs the
paper's experiments on synthetic skies.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 4] [--no-cpu] [--no-solve]
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
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bfloat16 MFMA, TFLOP/s
METRIC = "visibilities/s for Phi+Phi† (exact vs surrogate kernels) and % HBM roofline"
DATA = "synthetic (seeded sky and baselines; the paper's M31 / 30Dor images are not used)"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--taps", choices=["c64", "bf16", "i16"], default="c64")
    ap.add_argument("--phi", choices=["auto", "factors", "stored"], default="auto",
                    help="exact forms: Phi from the factor records (taps formed in registers), from the stored "
                         "taps, or whichever degrid times faster before the timed loop")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample rows (0: the workload's default)")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="surrogate form: skip the plain 256 figures")
    ap.add_argument("--channels", type=int, default=0, help="batched form: first K channels only (0: all)")
    ap.add_argument("--train-epochs", type=int, default=300, help="surrogate form: training passes")
    ap.add_argument("--tol", type=float, default=1e-3, help="surrogate form: per-row energy error tolerance")
    ap.add_argument("--pixels", type=int, default=0,
                    help="surrogate form: image side N instead of the workload's (the same M visibilities on a "
                         "smaller image: more of them per grid cell)")
    ap.add_argument("--check-nw", type=int, default=257, help="surrogate form: check lattice nodes along w")
    ap.add_argument("--check-nd", type=int, default=33, help="surrogate form: check lattice nodes per offset axis")
    ap.add_argument("--save-params", default=None,
                    help="surrogate form: write the trained network's parameters to this .npy file")
    ap.add_argument("--load-params", default=None,
                    help="surrogate form: take the network's parameters from this .npy file (written by "
                         "--save-params) instead of training; for counter runs, whose profiler slows the training's "
                         "many small launches")
    ap.add_argument("--sweep", choices=["energy", "coverage", "images"], default=None,
                    help="the paper's experiments on synthetic skies (tiny-form geometry): reconstruction SNR "
                         "and non-zero fraction against the preserved energy E, SNR against uv coverage "
                         "(Dirac, Daubechies-8 and SARA), or the reconstructed, error and residual images at "
                         "10 %% coverage and E = 0.75; for w_d = 0, U(0, 1) and 1; one JSON line per point")
    ap.add_argument("--images-out", default=None,
                    help="--sweep images: also write the sky and every scenario's reconstructed, error and "
                         "residual images to this .npz file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (reference for hardware byte counters)")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="wp_plan_set_tuning on the benchmark's plans (repeatable), e.g. sur_degrid=1")
    args = ap.parse_args()
    tune = []
    for kv in args.tune:
        k, _, v = kv.partition("=")
        if not k or not v.lstrip("-").isdigit():
            ap.error(f"--tune {kv!r}: expected KEY=INTEGER")
        tune.append((k, int(v)))
    args.tune = tune
    return args


def tuned(plan, args):
    """Apply the --tune settings to a plan."""
    for k, v in args.tune:
        plan.set_tuning(k, v)
    return plan


def degrid_bytes(G, M, Ng, tap_bytes):
    """Algorithmic HBM bytes of one degrid launch: taps + indices once, rowptr, perm, y, one grid read."""
    return G.nnz * (tap_bytes + 4) + (M + 1) * 8 + M * 4 + M * 8 + Ng * Ng * 8


def factor_degrid_bytes(G, M, Ng):
    """Algorithmic HBM bytes of one degrid from factor records: the records once, their offsets,
    y, one grid read."""
    return G.fdat.numel() + (M + 1) * 8 + M * 8 + Ng * Ng * 8


def scatter_bytes(G, M, Ng, tap_bytes):
    """Same stream as degrid plus the work list; the grid is written once (read y instead of writing it)."""
    return G.nnz * (tap_bytes + 4) + (M + 1) * 8 + M * 4 + M * 8 + Ng * Ng * 8 + G.n_work * 16


def gather_bytes(G, M, Ng, tap_bytes):
    """Transposed copy streamed once (value + visibility index), cell offsets and block table, y read once,
    grid written once."""
    table = 16 * (G.n_tblk + 1) if G.tblk is not None else 0
    return G.nnz * (tap_bytes + 4) + (Ng * Ng + 1) * 8 + table + M * 8 + Ng * Ng * 8


SOURCES = {"spmv": ("spmv.hip", "gather_block.h"), "surrogate": ("surrogate.hip",)}


def source_hash(kind="spmv"):
    """First 16 hex digits of the SHA-256 of the kernels' code (comments removed, whitespace runs
    collapsed): traffic counters stay valid while the code of these files is unchanged."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1307_3424_amd", "csrc")
    for f in SOURCES[kind]:
        path = os.path.join(csrc, f)
        if os.path.exists(path):
            code = open(path, encoding="utf-8").read()
            code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
            code = re.sub(r"//[^\n]*", " ", code)
            h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(tag, kernel, kind="spmv"):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary
    profiles/traffic_<tag>.md, or None if the summary is missing or the kernel's source changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith(("#", "|", "`")):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    if kv.get(f"{kind}_source_sha256_16") != source_hash(kind):
        return None
    v = kv.get(f"traffic_bytes.{kernel}")
    return float(v) if v is not None else None


def time_region(fn, steps, stream, torch):
    """Mean time of one call of fn (ms): HIP events recorded on the stream every launch goes to."""
    s_ev = torch.cuda.Event(enable_timing=True)
    e_ev = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s_ev.record(stream)
    for _ in range(steps):
        fn()
    e_ev.record(stream)
    torch.cuda.synchronize()
    return s_ev.elapsed_time(e_ev) / steps      # ms per call


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(wl, x, u, v, w, rows_n):
    """The FP64 oracle's Phi + Phi^H on a bounded sample: its rows for a seeded subset of the visibilities
    (built in a process pool, not timed), its sparse products on them scaled to all M rows, and its full
    FP64 grid transforms (scipy.fft over every host thread)."""
    import multiprocessing as mp
    import scipy.sparse as sp
    from oracle import wproj
    from oracle.wproj import Setup
    import synth
    s = Setup(N=wl.N, L=wl.L, W=wl.W)
    rows = synth.subset_rows(wl.M, rows_n, synth.rng_for(wl.seed, "subset", 9))
    workers = cpu_threads()
    chunks = [c for c in np.array_split(rows, workers * 4) if c.size]
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(wproj.build_rows_csr_parts, [(u[c], v[c], w[c], wl.E, s, None) for c in chunks])
    Gs = sp.vstack([sp.csr_matrix((d, i, p), shape=(n, s.Ng * s.Ng)) for p, i, d, n in parts]).tocsr()
    yv = synth.random_complex(rows.size, synth.rng_for(wl.seed, "y", 9))
    reps = 2 if s.Ng >= 2048 else 3
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
    return {"value": wl.M / t_step, "unit": "visibilities/s", "cores": workers, "kind": "oracle",
            "sample": f"{rows.size} of {wl.M} rows (seeded subset), sparse products (SciPy CSR, one thread) "
                      f"scaled x{scale:.1f} (subset-extrapolated), full FP64 grid transforms (scipy.fft, "
                      f"{workers} threads)",
            "cpu": cpu_model(), "step_s": t_step,
            "parts_s": {"fft_forward": t_fft_fwd, "fft_adjoint": t_fft_adj, "degrid_subset": t_deg,
                        "grid_subset": t_grid}}


def full_solve(wp, torch, plan, G, wl, x, xd, dev):
    """Reconstruction of the workload's sky from y = Phi x + n (30 dB) with its iteration count."""
    import synth
    G.order = wp.WP_ORDER_SORTED
    y0 = wp.apply_Phi(plan, G, xd)
    rms = float(torch.sqrt(torch.mean(torch.abs(y0.to(torch.complex128)) ** 2)))
    sig = 10 ** (-wl.snr_in_db / 20) * rms
    n = synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise"))
    nd = wp.to_sorted(G, torch.from_numpy(n.astype(np.complex64)).to(dev))
    y = y0 + nd
    eps = float(np.sqrt(sig ** 2 * (wl.M + 2 * np.sqrt(wl.M))))
    x0 = torch.from_numpy(synth.rng_for(wl.seed, "x").normal(size=wl.N * wl.N).astype(np.float32)).to(dev)
    t0 = time.perf_counter()
    nu = wp.power_norm2(plan, G, x0, 50)
    t_pow = time.perf_counter() - t0
    xr = torch.zeros(wl.N * wl.N, dtype=torch.float32, device=dev)
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s_ev.record()
    wp.solve(plan, G, y, eps, nu, wl.iters, 4, x=xr)
    e_ev.record()
    torch.cuda.synchronize()
    t_solve = s_ev.elapsed_time(e_ev) * 1e-3
    snr = _solve_snr(x, xr, wl.N)
    log(f"bench: solve {wl.iters} iterations in {t_solve * 1e3:.1f} ms (+ power iteration {t_pow * 1e3:.1f} ms), "
        f"SNR_out {snr:.2f} dB")
    # the other dictionaries of Section 4.2 on the same data: Dirac, and SARA (3 reweighting rounds
    # sharing the iteration count)
    others = {}
    for name in ("dirac", "sara"):
        xo = torch.zeros(wl.N * wl.N, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        s_ev.record()
        if name == "dirac":
            wp.solve(plan, G, y, eps, nu, wl.iters, 0, x=xo)
        else:
            wp.sara_solve(plan, G, y, eps, nu, wl.iters // 3, 3, 4, x=xo)
        e_ev.record()
        torch.cuda.synchronize()
        t = s_ev.elapsed_time(e_ev) * 1e-3
        it = wl.iters if name == "dirac" else 3 * (wl.iters // 3)
        so = _solve_snr(x, xo, wl.N)
        others[name] = {"iterations": it, "solve_s": t, "per_iteration_us": t / it * 1e6, "snr_out_db": so}
        log(f"bench: {name} solve {it} iterations in {t * 1e3:.1f} ms, SNR_out {so:.2f} dB")
    return {"iterations": wl.iters, "solve_s": t_solve, "power_iteration_s": t_pow, "per_iteration_us":
            t_solve / wl.iters * 1e6, "snr_out_db": snr, "snr_in_db": wl.snr_in_db, "dictionary": "Db8, 4 levels",
            "other_dictionaries": others}


def _solve_snr(x, xr, N):
    xr_h = xr.cpu().numpy().reshape(N, N).astype(np.float64)
    return float(20 * np.log10(np.std(x) / np.std(x - xr_h)))


def choose_degrid_form(wp, torch, plan, G, xd, yd, grid, stream, mode, M):
    """Degrid from the factor records or from the stored taps: `mode`, or for "auto" whichever of the two
    times faster on this workload (timed before the timed loop)."""
    if mode != "auto" or G.frec is None:
        G.use_factors = mode == "factors" and G.frec is not None
        return
    wp.grid_forward(plan, xd, grid)
    reps = 20 if M < 1 << 20 else 3
    tf = {}
    for fac in (True, False, True, False):
        G.use_factors = fac
        tf[fac] = min(tf.get(fac, 1e30), time_region(lambda: wp.degrid(plan, G, grid, yd), reps, stream, torch))
    G.use_factors = tf[True] < tf[False]


def bench_plain(args, wl, with_cpu=True, with_solve=True):
    """Exact operator of one single-problem form (plain 256 or precision 1024): the step, its stages, the
    HBM roofline of the slower sparse product, the solve (plain form) and the oracle's rate."""
    import torch
    import paper_1307_3424_amd as wp
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    import synth
    log(f"bench: workload {wl.name} N={wl.N} M={wl.M} E={wl.E} taps={args.taps}")
    x, u, v, w = synth.workload_inputs(wl)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    plan = tuned(wp.Plan(wl.N, wl.L, kb_W=wl.W), args)
    taps = {"c64": wp.WP_TAPS_C64, "bf16": wp.WP_TAPS_BF16, "i16": wp.WP_TAPS_I16}[args.taps]
    tap_bytes = 8 if taps == wp.WP_TAPS_C64 else 4
    ud, vd, wd = t(u), t(v), t(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = wp.build_G(plan, ud, vd, wd, wl.E, taps=taps, factors=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"bench: G built in {build_s:.3f} s, nnz={G.nnz} ({G.nnz / wl.M:.1f}/vis), work items {G.n_work}, "
        f"factor records {G.fdat.numel() / wl.M:.0f} B/vis")
    xd = t(x.astype(np.complex64).ravel())
    yd = torch.empty(wl.M, dtype=torch.complex64, device=dev)
    xa = torch.empty(wl.N * wl.N, dtype=torch.complex64, device=dev)
    grid = plan.new_grid()
    stream = torch.cuda.current_stream()
    # visibility vectors stay in G's sorted row order inside the timed loop (an iterative
    # solver permutes its data vector once); the caller-order cost is reported beside it
    G.order = wp.WP_ORDER_SORTED
    choose_degrid_form(wp, torch, plan, G, xd, yd, grid, stream, args.phi, wl.M)
    log(f"bench: Phi from {'factor records' if G.use_factors else 'stored taps'}")

    def step():
        wp.apply_Phi(plan, G, xd, yd, grid)
        wp.apply_PhiT(plan, G, yd, xa, grid)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = time_region(step, args.steps, stream, torch)
    log(f"bench: {ms * 1e3:.1f} us per Phi+Phi^H")
    # per-stage timings (same stream, HIP events around repeated launches of one stage)
    ks = max(20, args.steps) if wl.M < 1 << 20 else max(5, args.steps // 2)
    ms_phi = time_region(lambda: wp.apply_Phi(plan, G, xd, yd, grid), ks, stream, torch)
    ms_phit = time_region(lambda: wp.apply_PhiT(plan, G, yd, xa, grid), ks, stream, torch)
    ms_fwd = time_region(lambda: wp.grid_forward(plan, xd, grid), ks, stream, torch)
    wp.grid_forward(plan, xd, grid)
    ms_deg = time_region(lambda: wp.degrid(plan, G, grid, yd), ks, stream, torch)
    G.use_factors = not G.use_factors          # the other form of the degrid, for comparison
    ms_deg_alt = time_region(lambda: wp.degrid(plan, G, grid, yd), ks, stream, torch)
    G.use_factors = not G.use_factors
    ms_deg_f, ms_deg_s = (ms_deg, ms_deg_alt) if G.use_factors else (ms_deg_alt, ms_deg)
    ms_sc = time_region(lambda: wp.grid_scatter(plan, G, yd, grid), ks, stream, torch)
    ms_ga = time_region(lambda: wp.grid_gather(plan, G, yd, grid), ks, stream, torch)
    G.use_transpose = False
    ms_phit_sc = time_region(lambda: wp.apply_PhiT(plan, G, yd, xa, grid), ks, stream, torch)
    G.use_transpose = True
    ms_adj = time_region(lambda: wp.grid_adjoint(plan, grid, xa), ks, stream, torch)
    G.order = wp.WP_ORDER_CALLER
    ms_caller = time_region(step, ks, stream, torch)
    G.order = wp.WP_ORDER_SORTED
    db_s = degrid_bytes(G, wl.M, plan.Ng, tap_bytes)
    db_f = factor_degrid_bytes(G, wl.M, plan.Ng)
    db = db_f if G.use_factors else db_s
    sb = scatter_bytes(G, wl.M, plan.Ng, tap_bytes)
    deg_gbs = db / (ms_deg * 1e-3) / 1e9
    sc_gbs = sb / (ms_sc * 1e-3) / 1e9
    gb = gather_bytes(G, wl.M, plan.Ng, tap_bytes)
    ga_gbs = gb / (ms_ga * 1e-3) / 1e9
    # the library takes the blocked gather while cells average fewer than 512 entries
    blocked = G.tblk is not None and G.nnz < 512 * plan.Ng * plan.Ng
    ga_kernel = "k_gather_wave" if blocked else "k_gather"
    ga_label = "gather (Phi^H sparse product, transposed copy, " + ("one wave per block of cells)" if blocked
                                                                 else "one lane group per cell)")
    log(f"bench: Phi {ms_phi * 1e3:.1f} us, Phi^H {ms_phit * 1e3:.1f} us | fwd FFT {ms_fwd * 1e3:.1f} us, "
        f"degrid {ms_deg * 1e3:.1f} us ({deg_gbs:.0f} GB/s), scatter+zero {ms_sc * 1e3:.1f} us ({sc_gbs:.0f} GB/s), "
        f"gather {ms_ga * 1e3:.1f} us ({ga_gbs:.0f} GB/s), Phi^H via scatter {ms_phit_sc * 1e3:.1f} us, "
        f"adj FFT {ms_adj * 1e3:.1f} us")
    deg_kernel = "k_degrid_sep" if G.use_factors else "k_degrid"
    deg_label = ("degrid (Phi sparse product, taps formed from factor records)" if G.use_factors
                 else "degrid (Phi sparse product, stored taps)")
    tag = wl.name if args.taps == "c64" else f"{wl.name}-{args.taps}"
    # the roofline object describes the sparse product that takes longest in a step
    if ms_ga >= ms_deg:
        dominant = {"bound": "hbm", "kernel": ga_label, "achieved": ga_gbs,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ga_gbs / HBM_PEAK_GBS,
                    "traffic": profiled_traffic(tag, ga_kernel), "bytes_per_launch": gb, "launch_us": ms_ga * 1e3}
    else:
        dominant = {"bound": "hbm", "kernel": deg_label, "achieved": deg_gbs,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": deg_gbs / HBM_PEAK_GBS,
                    "traffic": profiled_traffic(tag, deg_kernel), "bytes_per_launch": db, "launch_us": ms_deg * 1e3}
    out = {
        "metric": METRIC,
        "value": wl.M / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "c64", "bf16": "bf16x2-taps/f32-accumulate",
                  "i16": "int16x2-block-float-taps/f32-accumulate"}[args.taps],
        "data": DATA,
        "config": {"workload": wl.name, "N": wl.N, "Ng": plan.Ng, "M": wl.M, "E": wl.E, "kb_W": wl.W,
                   "uv": f"{wl.uv} sigma={wl.uv_sigma}B", "w_top": wl.w_top,
                   "kernel": ("exact: Phi from factor records, Phi^H from the transposed copy" if G.use_factors
                              else "exact: stored G, Phi^H from the transposed copy"),
                   "nnz": G.nnz, "nnz_per_vis": G.nnz / wl.M, "G_bytes": G.nbytes(),
                   "factor_record_bytes": G.fdat.numel()},
        "roofline": dominant,
        "degrid_roofline": {"kernel": deg_label, "achieved": deg_gbs, "frac": deg_gbs / HBM_PEAK_GBS,
                            "bytes_per_launch": db, "launch_us": ms_deg * 1e3,
                            "traffic": profiled_traffic(tag, deg_kernel)},
        "degrid_forms_us": {"factor_records": ms_deg_f * 1e3, "stored_taps": ms_deg_s * 1e3,
                            "factor_records_bytes": db_f, "stored_taps_bytes": db_s},
        "stages_us": {"phi": ms_phi * 1e3, "phiT": ms_phit * 1e3, "grid_forward": ms_fwd * 1e3,
                      "degrid": ms_deg * 1e3, "gather": ms_ga * 1e3, "scatter_incl_zero": ms_sc * 1e3,
                      "grid_adjoint": ms_adj * 1e3, "phiT_via_scatter": ms_phit_sc * 1e3,
                      "step_caller_order": ms_caller * 1e3},
        "gather_roofline": {"kernel": ga_label, "achieved": ga_gbs, "frac": ga_gbs / HBM_PEAK_GBS,
                            "bytes_per_launch": gb, "launch_us": ms_ga * 1e3,
                            "traffic": profiled_traffic(tag, ga_kernel)},
        "scatter_roofline": {"achieved": sc_gbs, "frac": sc_gbs / HBM_PEAK_GBS, "bytes_per_launch": sb},
        "phi_vis_per_s": wl.M / (ms_phi * 1e-3), "phiT_vis_per_s": wl.M / (ms_phit * 1e-3),
        "build_G_s": build_s,
    }
    if with_solve and wl.iters and not args.no_solve:
        out["solve"] = full_solve(wp, torch, plan, G, wl, x, xd, dev)
    if with_cpu and not args.no_cpu:
        log("bench: timing the FP64 oracle on a bounded sample (CPU)")
        out["cpu_baseline"] = cpu_baseline(wl, x, u, v, w, args.cpu_rows or (4096 if wl.M > 1 << 20 else 384))
    del G
    torch.cuda.empty_cache()
    return out


def bench_batched(args, wl):
    """Batched form: all channels' Phi / Phi^H in one persistent launch each vs one launch per channel."""
    import torch
    import paper_1307_3424_amd as wp
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = len(wl.channels) if args.channels <= 0 else min(args.channels, len(wl.channels))
    log(f"bench: workload {wl.name} N={wl.N} channels={P} M_total={sum(wl.channels[:P])}")
    plan = tuned(wp.Plan(wl.N, wl.L, kb_W=wl.W), args)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Gs, skies = [], []
    t0 = time.perf_counter()
    for c in range(P):
        wtop = wl.w_top * wl.w_scale[c]
        u, v, w = synth.uvw(wl.N, wl.channels[c], wl.L, wl.uv, wl.uv_sigma, wtop, synth.rng_for(wl.seed, "uvw", c))
        G = wp.build_G(plan, t(u), t(v), t(w), wl.E)
        G.order = wp.WP_ORDER_SORTED
        del G._ws
        Gs.append(G)
        skies.append(synth.sky(wl.N, wl.n_blobs, wl.n_points, synth.rng_for(wl.seed, "sky", c)))
        if c % 8 == 7:
            torch.cuda.synchronize()
            log(f"bench: built {c + 1}/{P} channels ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    nnz = sum(G.nnz for G in Gs)
    log(f"bench: {P} G built in {build_s:.1f} s, nnz={nnz} ({nnz / sum(G.M for G in Gs):.1f}/vis), "
        f"{sum(G.nbytes() for G in Gs) / 1e9:.1f} GB")
    B = wp.Batch(plan, Gs)
    x, y, grids = B.new_buffers()
    x.copy_(t(np.concatenate([s_.ravel() for s_ in skies]).astype(np.complex64)))
    xa = torch.empty_like(x)
    best = B.autotune(x, y, grids)
    shapes = B.shapes()
    log(f"bench: autotuned shapes {shapes}, best degrid {best[0]:.0f} us, gather {best[1]:.0f} us")
    stream = torch.cuda.current_stream()
    N2, Ng2 = wl.N * wl.N, plan.Ng * plan.Ng
    offs = np.concatenate([[0], np.cumsum([G.M for G in Gs])])

    def batched():
        B.apply_Phi(x, y, grids)
        B.apply_PhiT(y, xa, grids)

    def sequential():
        for p_, G in enumerate(Gs):
            wp.apply_Phi(plan, G, x[p_ * N2:(p_ + 1) * N2], y[offs[p_]:offs[p_ + 1]], grids[:Ng2])
            wp.apply_PhiT(plan, G, y[offs[p_]:offs[p_ + 1]], xa[p_ * N2:(p_ + 1) * N2], grids[:Ng2])

    for _ in range(args.warmup):
        batched()
    ms_b = time_region(batched, args.steps, stream, torch)
    for _ in range(max(1, args.warmup // 4)):
        sequential()
    ms_s = time_region(sequential, max(3, args.steps // 4), stream, torch)
    ms_phi = time_region(lambda: B.apply_Phi(x, y, grids), args.steps, stream, torch)
    M_tot = int(offs[-1])
    tap_b = 8
    deg_bytes = nnz * (tap_b + 4) + sum((G.M + 1) * 8 + G.M * 4 + G.M * 8 for G in Gs) + P * Ng2 * 8
    ga_bytes = sum(gather_bytes(G, G.M, plan.Ng, tap_b) for G in Gs)
    log(f"bench: batched {ms_b:.3f} ms per Phi+Phi^H, sequential {ms_s:.3f} ms ({ms_s / ms_b:.2f}x)")
    rl = {"degrid": ("k_degrid_persist", deg_bytes, best[0]), "gather": ("k_gather_persist", ga_bytes, best[1])}
    dk = "gather" if best[1] >= best[0] else "degrid"
    dom = rl[dk]
    out = {
        "metric": METRIC,
        "value": M_tot / (ms_b * 1e-3), "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic (seeded skies and baselines per channel)",
        "config": {"workload": wl.name, "N": wl.N, "channels": P, "M_total": M_tot, "E": wl.E,
                   "w_scale": [wl.w_scale[0], wl.w_scale[P - 1]], "nnz": nnz, "kernel": "exact (stored G)"},
        "sequential_ms_per_step": ms_s, "speedup_vs_sequential": ms_s / ms_b,
        "sequential_vis_per_s": M_tot / (ms_s * 1e-3),
        "autotuned_shapes": {"degrid": shapes[:3], "gather": shapes[3:]},
        "autotune_best_us": best, "phi_ms": ms_phi,
        "roofline": {"bound": "hbm", "kernel": f"persistent {dk} over all channels ({dom[0]})",
                     "achieved": dom[1] / (dom[2] * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom[1] / (dom[2] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(wl.name, dom[0]), "bytes_per_launch": dom[1],
                     "launch_us": dom[2]},
        "degrid_roofline": {"achieved": deg_bytes / (best[0] * 1e-6) / 1e9,
                            "frac": deg_bytes / (best[0] * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": deg_bytes},
        "gather_roofline": {"achieved": ga_bytes / (best[1] * 1e-6) / 1e9,
                            "frac": ga_bytes / (best[1] * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": ga_bytes},
        "build_G_s": build_s,
    }
    del B, Gs
    torch.cuda.empty_cache()
    if not args.no_cpu:
        # the oracle on two channels (a 1024-row sample of each plus full FP64 transforms), extrapolated per
        # visibility and per channel to all channels
        log("bench: timing the FP64 oracle on two channels (CPU)")
        parts = []
        for c in range(min(2, P)):
            wtop = wl.w_top * wl.w_scale[c]
            u, v, w = synth.uvw(wl.N, wl.channels[c], wl.L, wl.uv, wl.uv_sigma, wtop, synth.rng_for(wl.seed, "uvw", c))
            wl_c = wl.scaled(M=wl.channels[c], w_top=wtop, channels=None, w_scale=None)
            parts.append(cpu_baseline(wl_c, skies[c], u, v, w, min(1024, wl.channels[c])))
        fft_s = np.mean([p_["parts_s"]["fft_forward"] + p_["parts_s"]["fft_adjoint"] for p_ in parts])
        per_vis = np.mean([(p_["step_s"] - p_["parts_s"]["fft_forward"] - p_["parts_s"]["fft_adjoint"]) /
                           wl.channels[c] for c, p_ in enumerate(parts)])
        t_all = P * fft_s + M_tot * per_vis
        out["cpu_baseline"] = {"value": M_tot / t_all, "unit": "visibilities/s", "cores": parts[0]["cores"],
                               "kind": "oracle", "cpu": parts[0]["cpu"],
                               "sample": f"channels 0 and 1: 1024-row samples of each (sparse products, SciPy CSR, "
                                         f"one thread) and full FP64 grid transforms (scipy.fft, {parts[0]['cores']} "
                                         f"threads), extrapolated per visibility to {M_tot} visibilities and per "
                                         f"channel to {P} channels"}
    return out



def bench_surrogate(args, wl):
    """Learned-surrogate form: the exact operator and the surrogate operator (network rows where the run-time
    check from the lattice passes, exact fallback rows elsewhere) on the same visibilities, timed the same
    way, with the surrogate's error against the exact operator, a reconstruction by each from the same data
    (Eq. 7, 200 iterations), and the rooflines (MFMA for the network's products, HBM for the exact ones)."""
    import torch
    import paper_1307_3424_amd as wp
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    log(f"bench: workload {wl.name} N={wl.N} M={wl.M} E={wl.E}: exact and surrogate forms")
    x, u, v, w = synth.workload_inputs(wl)
    plan = tuned(wp.Plan(wl.N, wl.L, kb_W=wl.W), args)
    ud, vd, wd = t(u), t(v), t(w)
    xd = t(x.astype(np.complex64).ravel())
    stream = torch.cuda.current_stream()
    sync = torch.cuda.synchronize
    ks = max(5, args.steps // 2)
    # ---- exact form
    sync()
    t0 = time.perf_counter()
    G = wp.build_G(plan, ud, vd, wd, wl.E, factors=True)
    sync()
    build_s = time.perf_counter() - t0
    G.order = wp.WP_ORDER_SORTED
    log(f"bench: exact G built in {build_s:.1f} s, nnz={G.nnz} ({G.nnz / wl.M:.1f}/vis), {G.nbytes() / 1e9:.1f} GB")
    yd = torch.empty(wl.M, dtype=torch.complex64, device=dev)
    xa = torch.empty(wl.N * wl.N, dtype=torch.complex64, device=dev)
    grid = plan.new_grid()
    choose_degrid_form(wp, torch, plan, G, xd, yd, grid, stream, args.phi, wl.M)
    step_e = lambda: (wp.apply_Phi(plan, G, xd, yd, grid), wp.apply_PhiT(plan, G, yd, xa, grid))
    for _ in range(args.warmup):
        step_e()
    ms_e = time_region(step_e, args.steps, stream, torch)
    ms_phi_e = time_region(lambda: wp.apply_Phi(plan, G, xd, yd, grid), ks, stream, torch)
    ms_phit_e = time_region(lambda: wp.apply_PhiT(plan, G, yd, xa, grid), ks, stream, torch)
    ms_fwd = time_region(lambda: wp.grid_forward(plan, xd, grid), ks, stream, torch)
    ms_adj = time_region(lambda: wp.grid_adjoint(plan, grid, xa), ks, stream, torch)
    wp.grid_forward(plan, xd, grid)
    ms_deg_e = time_region(lambda: wp.degrid(plan, G, grid, yd), ks, stream, torch)
    ms_ga_e = time_region(lambda: wp.grid_gather(plan, G, yd, grid), ks, stream, torch)
    log(f"bench: exact Phi+Phi^H {ms_e:.2f} ms (Phi {ms_phi_e:.2f}, Phi^H {ms_phit_e:.2f}; degrid {ms_deg_e:.2f}, "
        f"gather {ms_ga_e:.2f}, FFTs {ms_fwd:.2f} + {ms_adj:.2f})")
    # ---- the factor-record form of the exact operator: no stored taps, no transposed copy
    sync()
    t0 = time.perf_counter()
    Gr = wp.build_G(plan, ud, vd, wd, wl.E, factors=True, transpose=False, stored=False)
    sync()
    build_r_s = time.perf_counter() - t0
    Gr.order = wp.WP_ORDER_SORTED
    step_r = lambda: (wp.apply_Phi(plan, Gr, xd, yd, grid), wp.apply_PhiT(plan, Gr, yd, xa, grid))
    step_r()
    ms_r = time_region(step_r, ks, stream, torch)
    ms_sc_r = time_region(lambda: wp.grid_scatter(plan, Gr, yd, grid), ks, stream, torch)
    record_form = {"value": wl.M / (ms_r * 1e-3), "ms_per_step": ms_r, "scatter_ms": ms_sc_r,
                   "bytes": Gr.nbytes(), "bytes_per_vis": Gr.nbytes() / wl.M, "build_s": build_r_s}
    log(f"bench: factor-record form Phi+Phi^H {ms_r:.2f} ms (scatter from records {ms_sc_r:.2f} ms), "
        f"{Gr.nbytes() / 1e9:.2f} GB against {G.nbytes() / 1e9:.1f} GB stored")
    del Gr
    torch.cuda.empty_cache()
    # ---- network trained on rows the builder makes
    rng = synth.rng_for(wl.seed, "train")
    tu, tv, tw = (t(a) for a in synth.training_positions(wl, wl.train_samples, rng))
    sync()
    t0 = time.perf_counter()
    Gt = wp.build_G(plan, tu, tv, tw, wl.E, transpose=False)
    mlp = wp.Mlp(max_batch=8192)
    s_out = wp.Mlp.output_scale(plan)
    mlp.set_params(synth.mlp_init(wl.seed), wl.w_top, s_out)
    T, lost = mlp.box_targets(plan, Gt, tu, tv, s_out)
    ft = mlp.features(plan, tu, tv, tw)
    lost_max = float(lost.max())
    del Gt, lost
    sync()
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    if args.load_params:
        mlp.set_params(np.load(args.load_params), wl.w_top, s_out)
        hist = [float("nan"), float("nan")]
        log(f"bench: network parameters from {args.load_params} (no training)")
    else:
        log(f"bench: {wl.train_samples} exact training rows in {data_s:.1f} s (largest energy outside the box "
            f"{lost_max:.2e}); training {args.train_epochs} passes")
        hist = mlp.train(ft, T, 8192, args.train_epochs, 2e-3)
    sync()
    train_s = time.perf_counter() - t0
    del T, ft
    torch.cuda.empty_cache()
    log(f"bench: trained in {train_s:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    if args.save_params:
        np.save(args.save_params, mlp.get_params()[0])
    # ---- run-time check from the lattice (no exact row), surrogate set-up, fallback G
    t0 = time.perf_counter()
    table = mlp.check_table(plan, wl.E, args.check_nw, args.check_nd)
    feat = mlp.features(plan, ud, vd, wd)
    est = mlp.row_check(plan, table, args.check_nw, args.check_nd, feat)
    sync()
    check_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    sur = wp.Surrogate(plan, mlp, ud, vd, wd, eps=est, tol=args.tol)
    Gf = None
    if sur.Mf:
        fu, fv, fw = sur.fallback_coords()
        Gf = wp.build_G(plan, fu, fv, fw, wl.E, factors=True)
        Gf.order = wp.WP_ORDER_SORTED
        Gf.use_factors = G.use_factors
        del fu, fv, fw
    sync()
    setup_s = time.perf_counter() - t0
    # measurement only (not part of the check): the served rows' true errors against the exact rows
    eps_true = mlp.row_errors(plan, G, ud, vd, feat)
    served = est <= args.tol
    et = eps_true[served].cpu().numpy()
    del feat, eps_true
    over = float(np.mean(et > args.tol)) if et.size else 0.0
    log(f"bench: check {check_s:.2f} s: {sur.Ms} network rows ({sur.Ms / wl.M:.1%}), {sur.Mf} exact fallback rows, "
        f"{sur.ncell} occupied cells; served rows over tol {over:.2%}; surrogate set-up {setup_s:.1f} s")
    ys = torch.zeros(wl.M, dtype=torch.complex64, device=dev)
    step_s = lambda: (sur.apply_Phi(xd, ys, grid, Gf=Gf), sur.apply_PhiT(ys, xa, grid, Gf=Gf))
    for _ in range(args.warmup):
        step_s()
    ms_s = time_region(step_s, args.steps, stream, torch)
    ms_phi_s = time_region(lambda: sur.apply_Phi(xd, ys, grid, Gf=Gf), ks, stream, torch)
    ms_phit_s = time_region(lambda: sur.apply_PhiT(ys, xa, grid, Gf=Gf), ks, stream, torch)
    wp.grid_forward(plan, xd, grid)
    ms_sdeg = time_region(lambda: sur.degrid(grid, ys), ks, stream, torch)
    grid2 = plan.new_grid()
    ms_sgrid = time_region(lambda: sur.grid_add(ys, grid2), ks, stream, torch)
    ms_fdeg = ms_fga = 0.0
    if Gf is not None:
        yf = torch.empty(sur.Mf, dtype=torch.complex64, device=dev)
        ms_fdeg = time_region(lambda: wp.degrid(plan, Gf, grid, yf), ks, stream, torch)
        ms_fga = time_region(lambda: wp.grid_gather(plan, Gf, yf, grid2), ks, stream, torch)
        del yf
    del grid2
    log(f"bench: surrogate Phi+Phi^H {ms_s:.2f} ms (Phi {ms_phi_s:.2f}, Phi^H {ms_phit_s:.2f}; network degrid "
        f"{ms_sdeg:.2f}, network grid {ms_sgrid:.2f}, fallback degrid {ms_fdeg:.2f}, fallback gather {ms_fga:.2f})")
    # ---- accuracy of the surrogate operator against the exact one
    y_e = wp.to_caller(G, wp.apply_Phi(plan, G, xd))
    y_s = sur.apply_Phi(xd, Gf=Gf)
    y_e_slots = sur.to_slots(y_e, Gf=Gf)
    phi_err = float(torch.linalg.norm(y_s - y_e_slots) / torch.linalg.norm(y_e_slots))
    del y_s, y_e_slots
    yc = t(synth.random_complex(wl.M, synth.rng_for(wl.seed, "y", 4)).astype(np.complex64))
    xa_e = wp.apply_PhiT(plan, G, wp.to_sorted(G, yc))
    xa_s = sur.apply_PhiT(sur.to_slots(yc, Gf=Gf), Gf=Gf)
    phit_err = float(torch.linalg.norm(xa_s - xa_e) / torch.linalg.norm(xa_e))
    del yc
    log(f"bench: surrogate vs exact operator: Phi rel. error {phi_err:.3e}, Phi^H rel. error {phit_err:.3e}")
    # ---- reconstruction with each operator from the same data (30 dB, exact operator)
    solves = {}
    if not args.no_solve:
        rms = float(torch.sqrt(torch.mean(torch.abs(y_e.to(torch.complex128)) ** 2)))
        sig = 10 ** (-wl.snr_in_db / 20) * rms
        y_meas = y_e + t(synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise")).astype(np.complex64))
        ball = float(np.sqrt(sig ** 2 * (wl.M + 2 * np.sqrt(wl.M))))
        x0 = t(synth.rng_for(wl.seed, "x").normal(size=wl.N * wl.N).astype(np.float32))
        for form in ("exact", "surrogate"):
            sync()
            t0 = time.perf_counter()
            if form == "exact":
                nu = wp.power_norm2(plan, G, x0, 50)
                yv = wp.to_sorted(G, y_meas)
            else:
                nu = sur.power_norm2(x0, 50, Gf=Gf)
                yv = sur.to_slots(y_meas, Gf=Gf)
            sync()
            t_pow = time.perf_counter() - t0
            xr = torch.zeros(wl.N * wl.N, dtype=torch.float32, device=dev)
            s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            sync()
            s_ev.record()
            if form == "exact":
                wp.solve(plan, G, yv, ball, nu, wl.iters, 4, x=xr)
            else:
                sur.solve(yv, ball, nu, wl.iters, 4, x=xr, Gf=Gf)
            e_ev.record()
            sync()
            t_solve = s_ev.elapsed_time(e_ev) * 1e-3
            snr = _solve_snr(x, xr, wl.N)
            solves[form] = {"iterations": wl.iters, "solve_s": t_solve, "power_iteration_s": t_pow, "nu": nu,
                            "snr_out_db": snr}
            log(f"bench: {form} solve {wl.iters} iterations in {t_solve:.2f} s, SNR_out {snr:.2f} dB")
            del yv, xr
    # ---- rooflines: the network's products are MFMA work (2 x 2048 x 512 per occupied cell per product);
    # the exact products stream bytes
    flop = 2.0 * 2048 * 512 * sur.ncell
    deg_tf = flop / (ms_sdeg * 1e-3) / 1e12
    grd_tf = flop / (ms_sgrid * 1e-3) / 1e12
    # the timed calls: wp_surrogate_grid_add = k_sur_cell_s + k_sur_grid_ring, wp_surrogate_degrid =
    # k_grid_bf16_pad + k_sur_degrid_ring (the default forms); the small first kernel of each is counted in
    # the launch time, so the figure is a lower bound for the product kernel alone
    dom = (("k_sur_cell_s", "k_sur_grid_ring"), "gridding, k_sur_cell_s + k_sur_grid_ring", grd_tf, ms_sgrid) \
        if ms_sgrid >= ms_sdeg else (("k_grid_bf16_pad", "k_sur_degrid_ring"),
                                     "degridding, k_grid_bf16_pad + k_sur_degrid_ring", deg_tf, ms_sdeg)
    tag = wl.name
    # HBM bytes of the timed pair of kernels (both counted, as the launch time counts both)
    dom_tr = [profiled_traffic(tag, k, "surrogate") for k in dom[0]]
    dom_traffic = sum(dom_tr) if all(v is not None for v in dom_tr) else None
    db = factor_degrid_bytes(G, wl.M, plan.Ng) if G.use_factors else degrid_bytes(G, wl.M, plan.Ng, 8)
    gb = gather_bytes(G, wl.M, plan.Ng, 8)
    deg_kernel = "k_degrid_sep" if G.use_factors else "k_degrid"
    # hidden layers, per-cell s and sums, the bfloat16 grid copy, the fallback rows' G, the check table
    sur_bytes = (sur.Ms * 512 + (sur.ncell + 1) * 1024 + sur.ncell * 16 + plan.Ng * (plan.Ng + 32) * 4 +
                 (Gf.nbytes() if Gf is not None else 0) + table.numel() * 4)
    out = {
        "metric": METRIC,
        "value": wl.M / (ms_s * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_s,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mfma/f32-accumulate (network rows), c64 (fallback rows)",
        "data": DATA,
        "config": {"workload": wl.name, "N": wl.N, "Ng": plan.Ng, "M": wl.M, "E": wl.E, "kb_W": wl.W,
                   "uv": f"{wl.uv} sigma={wl.uv_sigma}B", "w_top": wl.w_top,
                   "kernel": "surrogate network + exact fallback (run-time check from the lattice)",
                   "network": "MLP 3-256-256-256-2048 GELU, bf16 products", "train_samples": wl.train_samples,
                   "train_epochs": args.train_epochs, "tol": args.tol,
                   "check_lattice": [args.check_nw, args.check_nd, args.check_nd]},
        "roofline": {"bound": "mfma", "kernel": f"surrogate {dom[1]} (per-cell output-layer product)",
                     "achieved": dom[2], "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": dom[2] / MFMA_BF16_PEAK_TFLOPS, "traffic": dom_traffic,
                     "flop_per_launch": flop, "launch_us": dom[3] * 1e3},
        "exact_rooflines": {
            "degrid": {"kernel": deg_kernel, "bound": "hbm", "achieved": db / (ms_deg_e * 1e-3) / 1e9,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": db / (ms_deg_e * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "bytes_per_launch": db, "launch_us": ms_deg_e * 1e3,
                       "traffic": profiled_traffic(tag, deg_kernel)},
            "gather": {"kernel": "k_gather_wave", "bound": "hbm", "achieved": gb / (ms_ga_e * 1e-3) / 1e9,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gb / (ms_ga_e * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "bytes_per_launch": gb, "launch_us": ms_ga_e * 1e3,
                       "traffic": profiled_traffic(tag, "k_gather_wave")}},
        "surrogate": {"rows_network": sur.Ms, "rows_fallback": sur.Mf, "occupied_cells": sur.ncell,
                      "frac_rows_network": sur.Ms / wl.M, "served_rows_over_tol": over,
                      "served_true_error_median": float(np.median(et)) if et.size else None,
                      "served_true_error_p99": float(np.quantile(et, 0.99)) if et.size else None,
                      "phi_rel_error_vs_exact": phi_err, "phiT_rel_error_vs_exact": phit_err,
                      "train_s": train_s, "train_data_s": data_s, "train_loss_first_last": [hist[0], hist[-1]],
                      "check_s": check_s, "setup_s": setup_s, "bytes": sur_bytes, "bytes_per_vis": sur_bytes / wl.M,
                      "stages_ms": {"phi": ms_phi_s, "phiT": ms_phit_s, "network_degrid": ms_sdeg,
                                    "network_grid": ms_sgrid, "fallback_degrid": ms_fdeg, "fallback_gather": ms_fga},
                      "degrid_tflops": deg_tf, "grid_tflops": grd_tf},
        "exact": {"value": wl.M / (ms_e * 1e-3), "ms_per_step": ms_e, "build_G_s": build_s, "nnz": G.nnz,
                  "bytes": G.nbytes(), "bytes_per_vis": G.nbytes() / wl.M,
                  "degrid_form": "factor records" if G.use_factors else "stored taps",
                  "stages_ms": {"phi": ms_phi_e, "phiT": ms_phit_e, "grid_forward": ms_fwd, "grid_adjoint": ms_adj,
                                "degrid": ms_deg_e, "gather": ms_ga_e}},
        "exact_factor_record_form": record_form,
        "surrogate_over_exact": ms_e / ms_s,
        # against the exact operator that keeps no stored taps either (the factor-record form)
        "surrogate_over_exact_record_form": record_form["ms_per_step"] / ms_s,
        "solve": solves,
        "solve_snr_gap_db": (solves["surrogate"]["snr_out_db"] - solves["exact"]["snr_out_db"]) if solves else None,
    }
    sur.close()
    mlp.close()
    del G, Gf, sur, table, est, grid, ys, xa, yd, y_e
    torch.cuda.empty_cache()
    if not args.no_cpu:
        log("bench: timing the FP64 oracle on a bounded sample (CPU)")
        out["cpu_baseline"] = cpu_baseline(wl, x, u, v, w, args.cpu_rows or 4096)
    return out


def bench_sweep(args):
    """Section 4's experiments on synthetic skies with the GPU path (tiny-form geometry, N = 64):
    visibilities uniform in the band with w = w_d w_max (w_max = N / (2 L^2): the chirp spans the
    field's band), data from the E = 1 operator plus 30 dB noise, reconstruction with the operator
    sparsified at E (200 primal-dual iterations, positivity) in the Daubechies-8 basis, and for the
    coverage sweep also in the Dirac basis and with SARA (three reweighting rounds of 66 iterations;
    Section 4.2).  The images sweep (10 % coverage,
    E = 0.75, Daubechies 8) also reports the error image x - x_rec and the residual image
    Re Phi^H Phi x_rec - Re Phi^H Phi x, with Phi the operator at E (Section 4.2)."""
    import torch
    import paper_1307_3424_amd as wp
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.workload(0)
    N, L, iters = wl.N, wl.L, 200
    Ng = 2 * N
    plan = wp.Plan(N, L)
    x = synth.sky(N, wl.n_blobs, wl.n_points, synth.rng_for(wl.seed, "sky"))
    xd = torch.from_numpy(x.astype(np.complex64).ravel()).to(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    w_max = N / (2 * L * L)
    bases = [("db8", 4)]
    if args.sweep == "energy":
        points = [(0.5, E) for E in (0.1, 0.25, 0.5, 0.75, 0.9, 0.99, 0.999, 1.0)]
    elif args.sweep == "coverage":
        points = [(c, 0.99) for c in (0.1, 0.3, 0.5, 0.7, 0.9)]
        bases = [("dirac", 0), ("db8", 4), ("sara", 4)]
    else:
        points = [(0.1, 0.75)]
    images = {"sky": x}
    for wd in ("0", "U(0,1)", "1"):
        for cov, E in points:
            M = int(round(cov * Ng * Ng))
            rng = synth.rng_for(wl.seed, "sweep", int(1000 * cov))
            u, v, _ = synth.uvw(N, M, L, "uniform", 0.0, 0.0, rng)
            w = {"0": np.zeros(M), "U(0,1)": rng.uniform(0.0, w_max, M), "1": np.full(M, w_max)}[wd]
            ud, vd, wdv = t(u), t(v), t(w)
            G1 = wp.build_G(plan, ud, vd, wdv, 1.0, transpose=False)
            G1.order = wp.WP_ORDER_CALLER
            y0 = wp.apply_Phi(plan, G1, xd)
            nnz1 = G1.nnz
            del G1
            rms = float(torch.sqrt(torch.mean(torch.abs(y0.to(torch.complex128)) ** 2)))
            sig = 10 ** (-30.0 / 20) * rms
            n = synth.noise(M, sig, synth.rng_for(wl.seed, "noise", int(1000 * cov)))
            y = y0 + t(n.astype(np.complex64))
            G = wp.build_G(plan, ud, vd, wdv, E)
            G.order = wp.WP_ORDER_SORTED
            ys = wp.to_sorted(G, y)
            eps = float(np.sqrt(sig ** 2 * (M + 2 * np.sqrt(M))))
            x0 = torch.from_numpy(synth.rng_for(wl.seed, "x").normal(size=N * N).astype(np.float32)).to(dev)
            nu = wp.power_norm2(plan, G, x0, 50)
            for basis, levels in bases:
                xr = torch.zeros(N * N, dtype=torch.float32, device=dev)
                s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                s_ev.record()
                if basis == "sara":       # three reweighting rounds sharing the iteration budget
                    wp.sara_solve(plan, G, ys, eps, nu, iters // 3, 3, levels, x=xr)
                else:
                    wp.solve(plan, G, ys, eps, nu, iters, levels, x=xr)
                e_ev.record()
                torch.cuda.synchronize()
                xr_h = xr.cpu().numpy().reshape(N, N).astype(np.float64)
                snr = float(20 * np.log10(np.std(x) / np.std(x - xr_h)))
                rec = {"sweep": args.sweep, "w_d": wd, "coverage": cov, "M": M, "E": E, "basis": basis,
                       "nnz_fraction": G.nnz / (M * Ng * Ng), "nnz_fraction_E1": nnz1 / (M * Ng * Ng),
                       "snr_out_db": snr, "iterations": 3 * (iters // 3) if basis == "sara" else iters,
                       "solve_ms": s_ev.elapsed_time(e_ev)}
                if args.sweep == "images":
                    # dirty images of the reconstruction and of the sky through the operator at E
                    dirty = lambda img: wp.apply_PhiT(plan, G, wp.apply_Phi(plan, G, img)).real
                    res = (dirty(xr.to(torch.complex64)) - dirty(xd)).cpu().numpy().reshape(N, N)
                    err = x - xr_h
                    rec.update({"error_rms": float(np.sqrt(np.mean(err ** 2))),
                                "error_max": float(np.abs(err).max()),
                                "residual_rms": float(np.sqrt(np.mean(res.astype(np.float64) ** 2))),
                                "dirty_sky_rms": float(np.sqrt(np.mean(
                                    dirty(xd).cpu().numpy().astype(np.float64) ** 2)))})
                    images[f"wd={wd}"] = np.stack([xr_h, err, res.astype(np.float64)])
                print(json.dumps(rec), flush=True)
            del G
    if args.sweep == "images" and args.images_out:
        np.savez_compressed(args.images_out, **images)



def main():
    args = parse()
    if args.sweep:
        return bench_sweep(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (every form fits one MI355X); "
                                   "--gpus must be 1"}))
        sys.exit(2)
    import synth
    wl = synth.workload(args.workload)
    if args.pixels:
        if not wl.train_samples or args.pixels < 64 or args.pixels & (args.pixels - 1):
            print(json.dumps({"error": "--pixels takes a power of two >= 64 and only the surrogate form"}))
            sys.exit(2)
        wl = wl.scaled(N=args.pixels, name=f"{wl.name}-at-{args.pixels}px")
    if wl.channels is not None:
        out = bench_batched(args, wl)
    elif wl.train_samples:
        out = bench_surrogate(args, wl)
        if not args.no_plain:
            # the plain 256-pixel form rides along: its step, stages, rooflines and 500-iteration solve
            p = bench_plain(args, synth.workload(1), with_cpu=not args.no_cpu, with_solve=True)
            out["plain_256"] = {k: p.get(k) for k in ("value", "ms_per_step", "config", "roofline", "degrid_roofline",
                                                     "gather_roofline", "degrid_forms_us", "stages_us", "solve",
                                                     "cpu_baseline", "phi_vis_per_s", "phiT_vis_per_s")}
    else:
        out = bench_plain(args, wl)
    if args.copy_probe:
        # one 256 MiB device copy: the reference dispatch for the hardware byte counters
        import torch
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 4
        del a, b
    if args.tune:
        out["config"]["tuning"] = dict(args.tune)
    out["extra_keys"] = sorted(k for k in out if k not in (
        "metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
