"""Sparse w-projection measurement operator on MI355X (gfx950).

Python face of libwproj.so (include/wproj.h): the same entry points, taking
torch tensors for device memory and the current torch stream.  No arithmetic
happens here.

    plan = Plan(N, L)                      # geometry + device tables
    G = build_G(plan, u, v, w, E)          # sparse w-projection matrix (two-phase build)
    y = apply_Phi(plan, G, x)              # y = G F Z A x
    x = apply_PhiT(plan, G, y)             # x = A Z^H F^H G^H y
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import _lib
from ._lib import (WP_APHYS_INV_N, WP_APHYS_ONE, WP_CHIRP_EXACT, WP_CHIRP_LINEAR, WP_ORDER_CALLER,
                   WP_ORDER_SORTED, WP_TAPS_BF16, WP_TAPS_C64, WP_TAPS_I16, WprojError, check, load)

__all__ = ["Plan", "GMatrix", "build_G", "build_G_batch", "apply_Phi", "apply_Phi_noalloc", "apply_PhiT", "grid_forward", "grid_adjoint",
           "degrid", "grid_scatter", "grid_gather", "load", "WprojError", "WP_TAPS_C64", "WP_TAPS_BF16", "WP_TAPS_I16",
           "WP_CHIRP_LINEAR", "WP_CHIRP_EXACT", "WP_APHYS_ONE", "WP_APHYS_INV_N", "WP_ORDER_CALLER",
           "WP_ORDER_SORTED", "to_sorted", "to_caller", "db8_filter", "dwt2", "idwt2", "power_norm2", "solve", "dr_solve", "sara_analysis", "sara_synthesis",
           "sara_solve", "Batch", "Mlp", "Surrogate"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev_c64(t, n, name):
    torch = _torch()
    if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous complex64 CUDA tensor with {n} elements")
    return t


def _dev_f64(t, n, name):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor with {n} elements")
    return t


class Plan:
    """wp_plan_create / wp_plan_destroy."""

    def __init__(self, N: int, fov_L: float, kb_W: int = 4, kb_beta: float = 0.0,
                 chirp: int = WP_CHIRP_LINEAR, aphys: int = WP_APHYS_ONE):
        lib = load()
        h = C.c_void_p()
        check(lib.wp_plan_create(C.byref(h), int(N), float(fov_L), int(kb_W), float(kb_beta),
                                 int(chirp), int(aphys)), "wp_plan_create")
        self._h = h
        self.N = int(N)
        ng, gb = C.c_int64(), C.c_int64()
        check(lib.wp_plan_info(h, C.byref(ng), C.byref(gb)), "wp_plan_info")
        self.Ng = ng.value
        self.grid_bytes = gb.value

    @property
    def handle(self):
        return self._h

    def set_tuning(self, key: str, value: int):
        """wp_plan_set_tuning (autotuner hook; 0 restores the automatic choice)."""
        check(load().wp_plan_set_tuning(self._h, key.encode(), int(value)), "wp_plan_set_tuning")

    def new_grid(self):
        torch = _torch()
        return torch.empty(self.Ng * self.Ng, dtype=torch.complex64, device="cuda")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().wp_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GMatrix:
    """CSR buffers of G (torch device tensors) and the wp_G descriptor pointing at them."""
    M: int
    nnz: int
    taps: int
    rowptr: object
    col: object
    val: object
    perm: object
    work: object
    n_work: int
    tcolptr: object = None
    trow: object = None
    tval: object = None
    rscale: object = None
    tblk: object = None              # block table of the transposed copy
    n_tblk: int = 0
    use_transpose: bool = True
    use_blocks: bool = True          # blocked gather when the table exists
    frec: object = None              # factor records (separable rows) read by the degrid
    fdat: object = None
    use_factors: bool = True         # degrid from the factor records when they exist
    order: int = WP_ORDER_CALLER     # order of the visibility vectors passed with this G

    def desc(self, transpose=None) -> _lib.WpG:
        d = _lib.WpG()
        d.M, d.nnz, d.taps, d.n_work, d.order = self.M, self.nnz, self.taps, self.n_work, self.order
        d.rowptr = self.rowptr.data_ptr()
        d.col = self.col.data_ptr() if self.col is not None else None
        d.val = self.val.data_ptr() if self.val is not None else None
        d.perm, d.work = self.perm.data_ptr(), self.work.data_ptr()
        if self.rscale is not None:
            d.rscale = self.rscale.data_ptr()
        if self.use_factors and self.frec is not None:
            d.frec, d.fdat, d.fbytes = self.frec.data_ptr(), self.fdat.data_ptr(), self.fdat.numel()
        use = self.use_transpose if transpose is None else transpose
        if use and self.tcolptr is not None:
            d.tcolptr, d.trow, d.tval = self.tcolptr.data_ptr(), self.trow.data_ptr(), self.tval.data_ptr()
            if self.use_blocks and self.tblk is not None:
                d.tblk, d.n_tblk = self.tblk.data_ptr(), self.n_tblk
        return d

    def nbytes(self) -> int:
        ts = [self.rowptr, self.col, self.val, self.perm, self.work, self.tcolptr, self.trow, self.tval,
              self.rscale, self.tblk, self.frec, self.fdat]
        return sum(t.numel() * t.element_size() for t in ts if t is not None)


def _new_G(plan: Plan, M: int, nnz: int, nwork: int, taps: int, transpose: bool, dev, stored: bool = True) -> GMatrix:
    """G's arrays for pass 2 of the build, sized from pass 1 (factor records aside); stored=False leaves
    out the taps and their columns (the factor-record form)."""
    torch = _torch()
    lib = load()
    G = GMatrix(M=M, nnz=nnz, taps=int(taps),
                rowptr=torch.empty(M + 1, dtype=torch.int64, device=dev),
                col=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev) if stored else None,
                val=(torch.empty(max(nnz, 1), dtype=(torch.complex64 if taps == WP_TAPS_C64 else torch.int32),
                                 device=dev) if stored else None),
                perm=torch.empty(M, dtype=torch.int32, device=dev),
                work=torch.empty(4 * max(nwork, 1), dtype=torch.int32, device=dev),
                n_work=nwork)
    if taps == WP_TAPS_I16:
        G.rscale = torch.empty(M, dtype=torch.float32, device=dev)
    if transpose:
        G.tcolptr = torch.empty(plan.Ng * plan.Ng + 1, dtype=torch.int64, device=dev)
        G.trow = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        G.tval = torch.empty_like(G.val)
        nt = C.c_int64()
        check(lib.wp_gather_table_size(plan.handle, nnz, C.byref(nt)), "wp_gather_table_size")
        G.n_tblk = nt.value
        G.tblk = torch.empty(2 * (nt.value + 1), dtype=torch.int64, device=dev)
    return G


def build_G(plan: Plan, u, v, w, E: float, taps: int = WP_TAPS_C64, transpose: bool = True,
            factors: bool = False, stream=None, beam=None, stored: bool = True) -> GMatrix:
    """wp_build_workspace_bytes + wp_build_G_count (+ wp_build_factor_bytes) + wp_build_G_fill
    (u, v, w: float64 CUDA tensors).

    transpose: also build the transposed copy used by the gather form of G^H (and its block table).
    factors: also build the factor records the degrid forms its taps from.
    stored: False keeps only the factor records (needs factors=True, transpose=False): no taps, no
    columns, no transposed copy; Phi forms its taps from the records and Phi^H scatters from them.
    beam: optional [M, 3] float64 CUDA tensor of per-visibility Gaussian power patterns
    (l0, m0, sigma): the rows carry that direction-dependent effect (wp_build_G_dde_*).
    """
    torch = _torch()
    lib = load()
    M = int(u.numel())
    for t, nm in ((u, "u"), (v, "v"), (w, "w")):
        _dev_f64(t, M, nm)
    if beam is not None:
        _dev_f64(beam, 3 * M, "beam")
    s = _stream(stream)
    wsb = C.c_int64()
    if beam is None:
        check(lib.wp_build_workspace_bytes(plan.handle, M, C.byref(wsb)), "wp_build_workspace_bytes")
    else:
        check(lib.wp_build_dde_workspace_bytes(plan.handle, M, C.byref(wsb)), "wp_build_dde_workspace_bytes")
    ws = torch.empty(wsb.value, dtype=torch.uint8, device="cuda")
    nnz, nwork = C.c_int64(), C.c_int64()
    if beam is None:
        check(lib.wp_build_G_count(plan.handle, M, _ptr(u), _ptr(v), _ptr(w), float(E), _ptr(ws),
                                   C.byref(nnz), C.byref(nwork), s), "wp_build_G_count")
    else:
        check(lib.wp_build_G_dde_count(plan.handle, M, _ptr(u), _ptr(v), _ptr(w), _ptr(beam), float(E), _ptr(ws),
                                       C.byref(nnz), C.byref(nwork), s), "wp_build_G_dde_count")
    dev = u.device
    if not stored and (not factors or transpose or beam is not None):
        raise ValueError("stored=False needs factors=True, transpose=False and no beam")
    G = _new_G(plan, M, nnz.value, nwork.value, taps, transpose, dev, stored)
    if factors:
        fb = C.c_int64()
        check(lib.wp_build_factor_bytes(plan.handle, M, _ptr(ws), C.byref(fb), s), "wp_build_factor_bytes")
        G.frec = torch.empty(M + 1, dtype=torch.int64, device=dev)
        G.fdat = torch.empty(fb.value, dtype=torch.uint8, device=dev)
    d = G.desc()
    if beam is None:
        check(lib.wp_build_G_fill(plan.handle, M, _ptr(u), _ptr(v), _ptr(w), float(E), _ptr(ws), C.byref(d), s),
              "wp_build_G_fill")
    else:
        check(lib.wp_build_G_dde_fill(plan.handle, M, _ptr(u), _ptr(v), _ptr(w), _ptr(beam), float(E), _ptr(ws),
                                      C.byref(d), s), "wp_build_G_dde_fill")
    G._ws = ws          # keep the workspace alive until the stream has consumed it
    return G


def build_G_batch(plans, us, vs, ws_, Es, taps: int = WP_TAPS_C64, transpose: bool = True, stream=None):
    """wp_build_G_count_batch + wp_build_G_fill_batch: one G per problem (lists of plans and float64
    CUDA tensors u, v, w, and energies)."""
    torch = _torch()
    lib = load()
    P = len(plans)
    M = [int(u.numel()) for u in us]
    for p in range(P):
        for t, nm in ((us[p], "u"), (vs[p], "v"), (ws_[p], "w")):
            _dev_f64(t, M[p], f"{nm}[{p}]")
    s = _stream(stream)
    work = []
    for p in range(P):
        b = C.c_int64()
        check(lib.wp_build_workspace_bytes(plans[p].handle, M[p], C.byref(b)), "wp_build_workspace_bytes")
        work.append(torch.empty(b.value, dtype=torch.uint8, device="cuda"))
    VP = C.c_void_p * P
    pl = VP(*[q.handle for q in plans])
    Ma = (C.c_int64 * P)(*M)
    ua, va, wa = VP(*[_ptr(t) for t in us]), VP(*[_ptr(t) for t in vs]), VP(*[_ptr(t) for t in ws_])
    Ea = (C.c_double * P)(*[float(e) for e in Es])
    wsa = VP(*[_ptr(t) for t in work])
    nnz, nwork = (C.c_int64 * P)(), (C.c_int64 * P)()
    check(lib.wp_build_G_count_batch(P, pl, Ma, ua, va, wa, Ea, wsa, nnz, nwork, s), "wp_build_G_count_batch")
    Gs = [_new_G(plans[p], M[p], nnz[p], nwork[p], taps, transpose, us[p].device) for p in range(P)]
    descs = [G.desc() for G in Gs]
    Ga = VP(*[C.addressof(d) for d in descs])
    check(lib.wp_build_G_fill_batch(P, pl, Ma, ua, va, wa, Ea, wsa, Ga, s), "wp_build_G_fill_batch")
    for G, wk in zip(Gs, work):
        G._ws = wk
    return Gs


def apply_Phi(plan: Plan, G: GMatrix, x, y=None, grid=None, stream=None):
    torch = _torch()
    _dev_c64(x, plan.N * plan.N, "x")
    y = torch.empty(G.M, dtype=torch.complex64, device=x.device) if y is None else _dev_c64(y, G.M, "y")
    grid = plan.new_grid() if grid is None else grid
    d = G.desc()
    check(load().wp_apply_Phi(plan.handle, C.byref(d), _ptr(x), _ptr(y), _ptr(grid), _stream(stream)),
          "wp_apply_Phi")
    return y


def apply_Phi_noalloc(plan: Plan, G: GMatrix, x, y, stream=None):
    """wp_apply_Phi_noalloc: y = Phi x with the library's static grid (no device allocation; y given)."""
    _dev_c64(x, plan.N * plan.N, "x")
    _dev_c64(y, G.M, "y")
    d = G.desc()
    check(load().wp_apply_Phi_noalloc(plan.handle, C.byref(d), _ptr(x), _ptr(y), _stream(stream)),
          "wp_apply_Phi_noalloc")
    return y


def apply_PhiT(plan: Plan, G: GMatrix, y, x=None, grid=None, stream=None):
    torch = _torch()
    _dev_c64(y, G.M, "y")
    x = torch.empty(plan.N * plan.N, dtype=torch.complex64, device=y.device) if x is None else \
        _dev_c64(x, plan.N * plan.N, "x")
    grid = plan.new_grid() if grid is None else grid
    d = G.desc()
    check(load().wp_apply_PhiT(plan.handle, C.byref(d), _ptr(y), _ptr(x), _ptr(grid), _stream(stream)),
          "wp_apply_PhiT")
    return x


def grid_forward(plan: Plan, x, grid=None, stream=None):
    _dev_c64(x, plan.N * plan.N, "x")
    grid = plan.new_grid() if grid is None else grid
    check(load().wp_grid_forward(plan.handle, _ptr(x), _ptr(grid), _stream(stream)), "wp_grid_forward")
    return grid


def grid_adjoint(plan: Plan, grid, x=None, stream=None):
    torch = _torch()
    _dev_c64(grid, plan.Ng * plan.Ng, "grid")
    x = torch.empty(plan.N * plan.N, dtype=torch.complex64, device=grid.device) if x is None else x
    check(load().wp_grid_adjoint(plan.handle, _ptr(grid), _ptr(x), _stream(stream)), "wp_grid_adjoint")
    return x


def degrid(plan: Plan, G: GMatrix, grid, y=None, stream=None):
    torch = _torch()
    _dev_c64(grid, plan.Ng * plan.Ng, "grid")
    y = torch.empty(G.M, dtype=torch.complex64, device=grid.device) if y is None else y
    d = G.desc()
    check(load().wp_degrid(plan.handle, C.byref(d), _ptr(grid), _ptr(y), _stream(stream)), "wp_degrid")
    return y


def grid_scatter(plan: Plan, G: GMatrix, y, grid=None, stream=None):
    _dev_c64(y, G.M, "y")
    grid = plan.new_grid() if grid is None else grid
    d = G.desc()
    check(load().wp_grid_scatter(plan.handle, C.byref(d), _ptr(y), _ptr(grid), _stream(stream)),
          "wp_grid_scatter")
    return grid


def grid_gather(plan: Plan, G: GMatrix, y, grid=None, stream=None):
    _dev_c64(y, G.M, "y")
    grid = plan.new_grid() if grid is None else grid
    d = G.desc(transpose=True)
    check(load().wp_grid_gather(plan.handle, C.byref(d), _ptr(y), _ptr(grid), _stream(stream)),
          "wp_grid_gather")
    return grid


def to_sorted(G: GMatrix, y, out=None, stream=None):
    """wp_to_sorted: out[r] = y[perm[r]] (caller order -> G's sorted row order)."""
    torch = _torch()
    _dev_c64(y, G.M, "y")
    out = torch.empty_like(y) if out is None else out
    d = G.desc()
    check(load().wp_to_sorted(C.byref(d), _ptr(y), _ptr(out), _stream(stream)), "wp_to_sorted")
    return out


def to_caller(G: GMatrix, y, out=None, stream=None):
    """wp_to_caller: out[perm[r]] = y[r] (sorted row order -> caller order)."""
    torch = _torch()
    _dev_c64(y, G.M, "y")
    out = torch.empty_like(y) if out is None else out
    d = G.desc()
    check(load().wp_to_caller(C.byref(d), _ptr(y), _ptr(out), _stream(stream)), "wp_to_caller")
    return out


def db8_filter():
    """wp_db8_filter: the 16 Daubechies-8 low-pass taps (host list)."""
    h = (C.c_double * 16)()
    check(load().wp_db8_filter(h), "wp_db8_filter")
    return list(h)


def _dev_f32(t, n, name):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous float32 CUDA tensor with {n} elements")
    return t


def dwt2(plan: Plan, x, levels: int = 4, out=None, stream=None):
    torch = _torch()
    _dev_f32(x, plan.N * plan.N, "x")
    out = torch.empty_like(x) if out is None else out
    scratch = torch.empty_like(x)
    check(load().wp_dwt2(plan.handle, int(levels), _ptr(x), _ptr(out), _ptr(scratch), _stream(stream)), "wp_dwt2")
    return out


def idwt2(plan: Plan, c, levels: int = 4, out=None, stream=None):
    torch = _torch()
    _dev_f32(c, plan.N * plan.N, "c")
    out = torch.empty_like(c) if out is None else out
    scratch = torch.empty_like(c)
    check(load().wp_idwt2(plan.handle, int(levels), _ptr(c), _ptr(out), _ptr(scratch), _stream(stream)),
          "wp_idwt2")
    return out


def _solver_ws(plan: Plan, G: GMatrix, d):
    torch = _torch()
    b = C.c_int64()
    check(load().wp_solver_workspace_bytes(plan.handle, C.byref(d), C.byref(b)), "wp_solver_workspace_bytes")
    return torch.empty(b.value, dtype=torch.uint8, device="cuda")


def power_norm2(plan: Plan, G: GMatrix, x0, iters: int = 50, stream=None) -> float:
    """wp_power_norm2 (synchronises)."""
    _dev_f32(x0, plan.N * plan.N, "x0")
    d = G.desc()
    ws = _solver_ws(plan, G, d)
    nu = C.c_double()
    check(load().wp_power_norm2(plan.handle, C.byref(d), _ptr(x0), int(iters), _ptr(ws), C.byref(nu),
                                _stream(stream)), "wp_power_norm2")
    return nu.value


def solve(plan: Plan, G: GMatrix, y, eps: float, nu: float, iters: int, levels: int = 4, x=None, ws=None,
          stream=None):
    """wp_solve: x (float32 N*N, zeros by default) is updated in place and returned."""
    torch = _torch()
    _dev_c64(y, G.M, "y")
    x = torch.zeros(plan.N * plan.N, dtype=torch.float32, device=y.device) if x is None else \
        _dev_f32(x, plan.N * plan.N, "x")
    d = G.desc()
    ws = _solver_ws(plan, G, d) if ws is None else ws
    check(load().wp_solve(plan.handle, C.byref(d), _ptr(y), float(eps), float(nu), int(iters), int(levels),
                          _ptr(x), _ptr(ws), _stream(stream)), "wp_solve")
    x._wp_ws = ws
    return x


def dr_solve(plan: Plan, G: GMatrix, y, eps: float, nu: float, iters: int, inner: int, gamma: float,
             levels: int = 4, x=None, stream=None):
    """wp_dr_solve: Douglas-Rachford for Eq. 7 without positivity; returns x (float32 N*N)."""
    torch = _torch()
    _dev_c64(y, G.M, "y")
    x = torch.empty(plan.N * plan.N, dtype=torch.float32, device=y.device) if x is None else \
        _dev_f32(x, plan.N * plan.N, "x")
    d = G.desc()
    b = C.c_int64()
    check(load().wp_dr_workspace_bytes(plan.handle, C.byref(d), C.byref(b)), "wp_dr_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
    check(load().wp_dr_solve(plan.handle, C.byref(d), _ptr(y), float(eps), float(nu), int(iters), int(inner),
                             float(gamma), int(levels), _ptr(x), _ptr(ws), _stream(stream)), "wp_dr_solve")
    x._wp_ws = ws
    return x


def sara_analysis(plan: Plan, x, levels: int = 4, out=None, stream=None):
    """wp_sara_analysis: [9, N, N] coefficients (Dirac, then Daubechies 1..8), flattened."""
    torch = _torch()
    n2 = plan.N * plan.N
    _dev_f32(x, n2, "x")
    out = torch.empty(9 * n2, dtype=torch.float32, device=x.device) if out is None else _dev_f32(out, 9 * n2, "out")
    scratch = torch.empty(16 * n2, dtype=torch.float32, device=x.device)
    check(load().wp_sara_analysis(plan.handle, int(levels), _ptr(x), _ptr(out), _ptr(scratch), _stream(stream)),
          "wp_sara_analysis")
    return out


def sara_synthesis(plan: Plan, c, levels: int = 4, out=None, stream=None):
    """wp_sara_synthesis: the N*N image of [9, N, N] coefficients."""
    torch = _torch()
    n2 = plan.N * plan.N
    _dev_f32(c, 9 * n2, "c")
    out = torch.empty(n2, dtype=torch.float32, device=c.device) if out is None else _dev_f32(out, n2, "out")
    scratch = torch.empty(16 * n2, dtype=torch.float32, device=c.device)
    check(load().wp_sara_synthesis(plan.handle, int(levels), _ptr(c), _ptr(out), _ptr(scratch), _stream(stream)),
          "wp_sara_synthesis")
    return out


def sara_solve(plan: Plan, G: GMatrix, y, eps: float, nu: float, iters: int, rounds: int, levels: int = 4, x=None,
               stream=None):
    """wp_sara_solve: x (float32 N*N, zeros by default) is updated in place and returned."""
    torch = _torch()
    _dev_c64(y, G.M, "y")
    x = torch.zeros(plan.N * plan.N, dtype=torch.float32, device=y.device) if x is None else \
        _dev_f32(x, plan.N * plan.N, "x")
    d = G.desc()
    b = C.c_int64()
    check(load().wp_sara_workspace_bytes(plan.handle, C.byref(d), C.byref(b)), "wp_sara_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
    check(load().wp_sara_solve(plan.handle, C.byref(d), _ptr(y), float(eps), float(nu), int(iters), int(rounds),
                               int(levels), _ptr(x), _ptr(ws), _stream(stream)), "wp_sara_solve")
    x._wp_ws = ws
    return x


class Batch:
    """wp_batch_*: P problems sharing one plan, one persistent launch per sparse product."""

    def __init__(self, plan: Plan, Gs):
        self.plan = plan
        self.Gs = list(Gs)
        arr = (_lib.WpG * len(self.Gs))(*[G.desc() for G in self.Gs])
        h = C.c_void_p()
        check(load().wp_batch_create(C.byref(h), plan.handle, len(self.Gs), arr), "wp_batch_create")
        self._h = h
        self.M_total = sum(G.M for G in self.Gs)

    def shapes(self):
        m = C.c_int64()
        sh = (C.c_int * 6)()
        check(load().wp_batch_info(self._h, C.byref(m), sh), "wp_batch_info")
        return list(sh)

    def new_buffers(self):
        torch = _torch()
        P, N, Ng = len(self.Gs), self.plan.N, self.plan.Ng
        x = torch.zeros(P * N * N, dtype=torch.complex64, device="cuda")
        y = torch.zeros(self.M_total, dtype=torch.complex64, device="cuda")
        grids = torch.empty(P * Ng * Ng, dtype=torch.complex64, device="cuda")
        return x, y, grids

    def apply_Phi(self, x, y, grids, stream=None):
        check(load().wp_apply_Phi_batch(self._h, _ptr(x), _ptr(y), _ptr(grids), _stream(stream)),
              "wp_apply_Phi_batch")
        return y

    def apply_PhiT(self, y, x, grids, stream=None):
        check(load().wp_apply_PhiT_batch(self._h, _ptr(y), _ptr(x), _ptr(grids), _stream(stream)),
              "wp_apply_PhiT_batch")
        return x

    def autotune(self, x, y, grids, stream=None):
        best = (C.c_float * 2)()
        check(load().wp_batch_autotune(self._h, _ptr(x), _ptr(y), _ptr(grids), _stream(stream), best),
              "wp_batch_autotune")
        return list(best)

    def mode(self, degrid: int = -1, gather: int = -1):
        """wp_batch_mode: set (0 persistent, 1 flat, < 0 keep) and return (degrid, gather) modes."""
        d, g = C.c_int(), C.c_int()
        check(load().wp_batch_mode(self._h, int(degrid), int(gather), C.byref(d), C.byref(g)), "wp_batch_mode")
        return d.value, g.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().wp_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_f32n(t, n, name):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous float32 CUDA tensor with {n} elements")
    return t


class Mlp:
    """wp_mlp_*: the surrogate network (parameters, Adam moments and activations on the device)."""

    H, BOX, NOUT = 256, 32, 2048

    def __init__(self, max_batch: int = 8192):
        h = C.c_void_p()
        check(load().wp_mlp_create(C.byref(h), int(max_batch)), "wp_mlp_create")
        self._h = h
        self.max_batch = int(max_batch)

    @staticmethod
    def param_count() -> int:
        return int(load().wp_mlp_param_count())

    @property
    def handle(self):
        return self._h

    def set_params(self, params, w_top: float, s_out: float):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.param_count():
            raise ValueError(f"params: need {self.param_count()} floats")
        check(load().wp_mlp_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), float(w_top),
                                       float(s_out)), "wp_mlp_set_params")

    def get_params(self):
        import numpy as np
        p = np.empty(self.param_count(), dtype=np.float32)
        wt, so = C.c_double(), C.c_double()
        check(load().wp_mlp_get_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), C.byref(wt), C.byref(so)),
              "wp_mlp_get_params")
        return p, wt.value, so.value

    def features(self, plan: Plan, u, v, w, out=None, stream=None):
        torch = _torch()
        n = u.numel()
        for t, nm in ((u, "u"), (v, "v"), (w, "w")):
            _dev_f64(t, n, nm)
        out = torch.empty(3 * n, dtype=torch.float32, device="cuda") if out is None else _dev_f32n(out, 3 * n, "out")
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        check(load().wp_mlp_features(plan.handle, self._h, n, _ptr(u), _ptr(v), _ptr(w), _ptr(out), _ptr(err),
                                     _stream(stream)), "wp_mlp_features")
        if int(err.item()) != 0:
            raise WprojError(-1, "wp_mlp_features: a coordinate is not finite or lies outside the grid")
        return out

    def forward(self, feat, out=None, stream=None):
        torch = _torch()
        n = feat.numel() // 3
        _dev_f32n(feat, 3 * n, "feat")
        out = torch.empty(n * self.NOUT, dtype=torch.float32, device="cuda") if out is None else \
            _dev_f32n(out, n * self.NOUT, "out")
        check(load().wp_mlp_forward(self._h, n, _ptr(feat), _ptr(out), _stream(stream)), "wp_mlp_forward")
        return out

    def gradients(self, feat, target, grads=None, stream=None):
        torch = _torch()
        n = feat.numel() // 3
        _dev_f32n(feat, 3 * n, "feat")
        _dev_f32n(target, n * self.NOUT, "target")
        grads = torch.empty(self.param_count(), dtype=torch.float32, device="cuda") if grads is None else \
            _dev_f32n(grads, self.param_count(), "grads")
        loss = C.c_double()
        check(load().wp_mlp_gradients(self._h, n, _ptr(feat), _ptr(target), _ptr(grads), C.byref(loss),
                                      _stream(stream)), "wp_mlp_gradients")
        return grads, loss.value

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        check(load().wp_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
              "wp_mlp_adam_step")

    def train(self, feat, target, batch: int, epochs: int, lr_max: float, stream=None):
        n = feat.numel() // 3
        _dev_f32n(feat, 3 * n, "feat")
        _dev_f32n(target, n * self.NOUT, "target")
        hist = (C.c_double * int(epochs))()
        check(load().wp_mlp_train(self._h, n, _ptr(feat), _ptr(target), int(batch), int(epochs), float(lr_max), hist,
                                  _stream(stream)), "wp_mlp_train")
        return list(hist)

    @staticmethod
    def output_scale(plan: Plan) -> float:
        s = C.c_double()
        check(load().wp_mlp_output_scale(plan.handle, C.byref(s)), "wp_mlp_output_scale")
        return s.value

    def box_targets(self, plan: Plan, G: GMatrix, u, v, s_out: float, stream=None):
        torch = _torch()
        _dev_f64(u, G.M, "u")
        _dev_f64(v, G.M, "v")
        target = torch.empty(G.M * self.NOUT, dtype=torch.float32, device="cuda")
        lost = torch.empty(G.M, dtype=torch.float32, device="cuda")
        d = G.desc()
        check(load().wp_mlp_box_targets(plan.handle, C.byref(d), _ptr(u), _ptr(v), float(s_out), _ptr(target),
                                        _ptr(lost), _stream(stream)), "wp_mlp_box_targets")
        return target, lost

    def row_errors(self, plan: Plan, G: GMatrix, u, v, feat, stream=None):
        torch = _torch()
        _dev_f64(u, G.M, "u")
        _dev_f64(v, G.M, "v")
        _dev_f32n(feat, 3 * G.M, "feat")
        eps = torch.empty(G.M, dtype=torch.float32, device="cuda")
        d = G.desc()
        check(load().wp_mlp_row_errors(plan.handle, self._h, C.byref(d), _ptr(u), _ptr(v), _ptr(feat), _ptr(eps),
                                       _stream(stream)), "wp_mlp_row_errors")
        return eps

    def lattice_coords(self, plan: Plan, nw: int, nd: int, stream=None):
        """wp_mlp_lattice_coords: (u, v, w) of the check lattice's nw * nd * nd nodes (float64 CUDA)."""
        torch = _torch()
        n = int(nw) * int(nd) * int(nd)
        u, v, w = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
        check(load().wp_mlp_lattice_coords(plan.handle, self._h, int(nw), int(nd), _ptr(u), _ptr(v), _ptr(w),
                                           _stream(stream)), "wp_mlp_lattice_coords")
        return u, v, w

    def check_table(self, plan: Plan, E: float, nw: int = 257, nd: int = 33, stream=None):
        """The check lattice's table: its nodes' exact rows (wp_build_G_* on wp_mlp_lattice_coords) and
        wp_mlp_check_table.  Returns float32 CUDA [2 nw nd nd] (node errors, then kept energies)."""
        torch = _torch()
        u, v, w = self.lattice_coords(plan, nw, nd, stream)
        G = build_G(plan, u, v, w, E, transpose=False, stream=stream)
        feat = self.features(plan, u, v, w, stream=stream)
        table = torch.empty(2 * G.M, dtype=torch.float32, device="cuda")
        d = G.desc()
        check(load().wp_mlp_check_table(plan.handle, self._h, C.byref(d), int(nw), int(nd), _ptr(u), _ptr(v),
                                        _ptr(feat), _ptr(table), _stream(stream)), "wp_mlp_check_table")
        torch.cuda.synchronize()
        return table

    def row_check(self, plan: Plan, table, nw: int, nd: int, feat, stream=None):
        """wp_mlp_row_check: estimated row errors (float32 CUDA [n], caller order) from the table alone."""
        torch = _torch()
        n = feat.numel() // 3
        _dev_f32n(feat, 3 * n, "feat")
        _dev_f32n(table, 2 * int(nw) * int(nd) * int(nd), "table")
        est = torch.empty(n, dtype=torch.float32, device="cuda")
        check(load().wp_mlp_row_check(plan.handle, self._h, int(nw), int(nd), _ptr(table), n, _ptr(feat), _ptr(est),
                                      _stream(stream)), "wp_mlp_row_check")
        return est

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().wp_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """wp_surrogate_*: Phi / Phi^H with network rows where the per-row energy error is at most tol and exact
    fallback rows elsewhere.  Visibility vectors are in slot order (see slots())."""

    def __init__(self, plan: Plan, mlp: Mlp, u, v, w, eps=None, tol: float = 1e-3, stream=None):
        M = u.numel()
        for t, nm in ((u, "u"), (v, "v"), (w, "w")):
            _dev_f64(t, M, nm)
        if eps is not None:
            _dev_f32n(eps, M, "eps")
        h = C.c_void_p()
        mf = C.c_int64()
        check(load().wp_surrogate_create(C.byref(h), plan.handle, mlp.handle, M, _ptr(u), _ptr(v), _ptr(w), _ptr(eps),
                                         float(tol), C.byref(mf), _stream(stream)), "wp_surrogate_create")
        self._h = h
        self.plan = plan
        info = (C.c_int64 * 5)()
        check(load().wp_surrogate_info(h, info), "wp_surrogate_info")
        self.M, self.Ms, self.Mf, self.ncell = int(info[0]), int(info[1]), int(info[2]), int(info[3])
        self.groups = (int(info[4]) >> 32, int(info[4]) & 0xffffffff)

    def slots(self, stream=None):
        torch = _torch()
        out = torch.empty(self.M, dtype=torch.int32, device="cuda")
        check(load().wp_surrogate_slots(self._h, _ptr(out), _stream(stream)), "wp_surrogate_slots")
        return out

    def fallback_coords(self, stream=None):
        torch = _torch()
        u, v, w = (torch.empty(self.Mf, dtype=torch.float64, device="cuda") for _ in range(3))
        check(load().wp_surrogate_fallback_coords(self._h, _ptr(u), _ptr(v), _ptr(w), _stream(stream)),
              "wp_surrogate_fallback_coords")
        return u, v, w

    def degrid(self, grid, y=None, stream=None):
        torch = _torch()
        _dev_c64(grid, self.plan.Ng ** 2, "grid")
        y = torch.zeros(self.M, dtype=torch.complex64, device="cuda") if y is None else _dev_c64(y, self.M, "y")
        check(load().wp_surrogate_degrid(self.plan.handle, self._h, _ptr(grid), _ptr(y), _stream(stream)),
              "wp_surrogate_degrid")
        return y

    def grid_add(self, y, grid, stream=None):
        _dev_c64(y, self.M, "y")
        _dev_c64(grid, self.plan.Ng ** 2, "grid")
        check(load().wp_surrogate_grid_add(self.plan.handle, self._h, _ptr(y), _ptr(grid), _stream(stream)),
              "wp_surrogate_grid_add")
        return grid

    def _gf(self, Gf):
        if self.Mf == 0:
            return None
        if Gf is None:
            raise ValueError(f"{self.Mf} fallback rows need their exact G")
        return C.byref(Gf.desc())

    def apply_Phi(self, x, y=None, grid=None, Gf=None, stream=None):
        torch = _torch()
        N = self.plan.N
        _dev_c64(x, N * N, "x")
        y = torch.empty(self.M, dtype=torch.complex64, device="cuda") if y is None else _dev_c64(y, self.M, "y")
        grid = self.plan.new_grid() if grid is None else grid
        gf = self._gf(Gf)
        check(load().wp_surrogate_apply_Phi(self.plan.handle, self._h, gf, _ptr(x), _ptr(y), _ptr(grid),
                                            _stream(stream)), "wp_surrogate_apply_Phi")
        return y

    def apply_PhiT(self, y, x=None, grid=None, Gf=None, stream=None):
        torch = _torch()
        N = self.plan.N
        _dev_c64(y, self.M, "y")
        x = torch.empty(N * N, dtype=torch.complex64, device="cuda") if x is None else _dev_c64(x, N * N, "x")
        grid = self.plan.new_grid() if grid is None else grid
        gf = self._gf(Gf)
        check(load().wp_surrogate_apply_PhiT(self.plan.handle, self._h, gf, _ptr(y), _ptr(x), _ptr(grid),
                                             _stream(stream)), "wp_surrogate_apply_PhiT")
        return x

    def to_slots(self, y_caller, Gf=None, out=None, stream=None):
        torch = _torch()
        _dev_c64(y_caller, self.M, "y_caller")
        out = torch.empty(self.M, dtype=torch.complex64, device="cuda") if out is None else _dev_c64(out, self.M, "out")
        check(load().wp_surrogate_to_slots(self._h, self._gf(Gf), _ptr(y_caller), _ptr(out), _stream(stream)),
              "wp_surrogate_to_slots")
        return out

    def _solver_ws(self):
        torch = _torch()
        b = C.c_int64()
        check(load().wp_surrogate_solver_workspace_bytes(self.plan.handle, self._h, C.byref(b)),
              "wp_surrogate_solver_workspace_bytes")
        return torch.empty(b.value, dtype=torch.uint8, device="cuda")

    def power_norm2(self, x0, iters: int = 50, Gf=None, stream=None) -> float:
        ws = self._solver_ws()
        nu = C.c_double()
        check(load().wp_surrogate_power_norm2(self.plan.handle, self._h, self._gf(Gf), _ptr(x0), int(iters), _ptr(ws),
                                              C.byref(nu), _stream(stream)), "wp_surrogate_power_norm2")
        return nu.value

    def solve(self, y_slots, eps: float, nu: float, iters: int, levels: int = 4, x=None, Gf=None, stream=None):
        torch = _torch()
        N = self.plan.N
        _dev_c64(y_slots, self.M, "y_slots")
        x = torch.zeros(N * N, dtype=torch.float32, device="cuda") if x is None else x
        ws = self._solver_ws()
        check(load().wp_surrogate_solve(self.plan.handle, self._h, self._gf(Gf), _ptr(y_slots), float(eps), float(nu),
                                        int(iters), int(levels), _ptr(x), _ptr(ws), _stream(stream)),
              "wp_surrogate_solve")
        x._wp_ws = ws
        return x

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().wp_surrogate_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
