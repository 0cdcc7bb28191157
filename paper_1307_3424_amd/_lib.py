"""ctypes binding of libwproj.so: argument marshalling only.

Every computation happens in the HIP library; this module converts torch
tensors (device memory, streams) into the plain pointers and sizes of the C
ABI declared in include/wproj.h, and turns error codes into exceptions.  If
the library is missing it raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwproj.so")

WP_CHIRP_LINEAR, WP_CHIRP_EXACT = 0, 1
WP_TAPS_C64, WP_TAPS_BF16, WP_TAPS_I16 = 0, 1, 2
WP_APHYS_ONE, WP_APHYS_INV_N = 0, 1
WP_ORDER_CALLER, WP_ORDER_SORTED = 0, 1

STATUS = {0: "WP_OK", -1: "WP_EINVAL", -2: "WP_ENOMEM", -3: "WP_EHIP", -4: "WP_ECAPACITY",
          -5: "WP_EUNSUPPORTED"}

# every entry point declared in include/wproj.h, with its argument types
_vp, _i64, _i32, _d = C.c_void_p, C.c_int64, C.c_int, C.c_double
_pi64 = C.POINTER(C.c_int64)


class WpG(C.Structure):
    _fields_ = [("M", C.c_int64), ("nnz", C.c_int64), ("taps", C.c_int32), ("order", C.c_int32),
                ("rowptr", _vp), ("col", _vp), ("val", _vp), ("perm", _vp), ("work", _vp),
                ("n_work", C.c_int64), ("rscale", _vp), ("tcolptr", _vp), ("trow", _vp), ("tval", _vp),
                ("tblk", _vp), ("n_tblk", C.c_int64), ("frec", _vp), ("fdat", _vp), ("fbytes", C.c_int64)]


_PG = C.POINTER(WpG)

SIGNATURES = {
    "wp_last_error": ([], C.c_char_p),
    "wp_version": ([], C.c_char_p),
    "wp_plan_create": ([C.POINTER(_vp), _i32, _d, _i32, _d, _i32, _i32], _i32),
    "wp_plan_destroy": ([_vp], _i32),
    "wp_plan_info": ([_vp, _pi64, _pi64], _i32),
    "wp_plan_set_tuning": ([_vp, C.c_char_p, _i32], _i32),
    "wp_gather_table_size": ([_vp, _i64, _pi64], _i32),
    "wp_build_factor_bytes": ([_vp, _i64, _vp, _pi64, _vp], _i32),
    "wp_build_workspace_bytes": ([_vp, _i64, _pi64], _i32),
    "wp_build_G_count": ([_vp, _i64, _vp, _vp, _vp, _d, _vp, _pi64, _pi64, _vp], _i32),
    "wp_build_G_fill": ([_vp, _i64, _vp, _vp, _vp, _d, _vp, _PG, _vp], _i32),
    "wp_build_dde_workspace_bytes": ([_vp, _i64, _pi64], _i32),
    "wp_build_G_count_batch": ([_i32, _vp, _pi64, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _pi64, _pi64, _vp],
                               _i32),
    "wp_build_G_fill_batch": ([_i32, _vp, _pi64, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _vp, _vp], _i32),
    "wp_build_G_dde_count": ([_vp, _i64, _vp, _vp, _vp, _vp, _d, _vp, _pi64, _pi64, _vp], _i32),
    "wp_build_G_dde_fill": ([_vp, _i64, _vp, _vp, _vp, _vp, _d, _vp, _PG, _vp], _i32),
    "wp_apply_Phi": ([_vp, _PG, _vp, _vp, _vp, _vp], _i32),
    "wp_apply_PhiT": ([_vp, _PG, _vp, _vp, _vp, _vp], _i32),
    "wp_apply_Phi_noalloc": ([_vp, _PG, _vp, _vp, _vp], _i32),
    "wp_grid_forward": ([_vp, _vp, _vp, _vp], _i32),
    "wp_grid_adjoint": ([_vp, _vp, _vp, _vp], _i32),
    "wp_degrid": ([_vp, _PG, _vp, _vp, _vp], _i32),
    "wp_grid_scatter": ([_vp, _PG, _vp, _vp, _vp], _i32),
    "wp_grid_gather": ([_vp, _PG, _vp, _vp, _vp], _i32),
    "wp_to_sorted": ([_PG, _vp, _vp, _vp], _i32),
    "wp_to_caller": ([_PG, _vp, _vp, _vp], _i32),
    "wp_db8_filter": ([C.POINTER(C.c_double)], _i32),
    "wp_batch_create": ([C.POINTER(_vp), _vp, _i32, _PG], _i32),
    "wp_batch_destroy": ([_vp], _i32),
    "wp_batch_info": ([_vp, _pi64, C.POINTER(C.c_int)], _i32),
    "wp_apply_Phi_batch": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "wp_apply_PhiT_batch": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "wp_batch_autotune": ([_vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_float)], _i32),
    "wp_batch_mode": ([_vp, _i32, _i32, C.POINTER(C.c_int), C.POINTER(C.c_int)], _i32),
    "wp_mlp_param_count": ([], _i64),
    "wp_mlp_create": ([C.POINTER(_vp), _i32], _i32),
    "wp_mlp_destroy": ([_vp], _i32),
    "wp_mlp_set_params": ([_vp, C.POINTER(C.c_float), _d, _d], _i32),
    "wp_mlp_get_params": ([_vp, C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_double)], _i32),
    "wp_mlp_features": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "wp_mlp_forward": ([_vp, _i32, _vp, _vp, _vp], _i32),
    "wp_mlp_gradients": ([_vp, _i32, _vp, _vp, _vp, C.POINTER(C.c_double), _vp], _i32),
    "wp_mlp_adam_step": ([_vp, C.c_float, C.c_float, C.c_float, C.c_float, _vp], _i32),
    "wp_mlp_train": ([_vp, _i64, _vp, _vp, _i32, _i32, C.c_float, C.POINTER(C.c_double), _vp], _i32),
    "wp_mlp_output_scale": ([_vp, C.POINTER(C.c_double)], _i32),
    "wp_mlp_box_targets": ([_vp, _PG, _vp, _vp, _d, _vp, _vp, _vp], _i32),
    "wp_mlp_row_errors": ([_vp, _vp, _PG, _vp, _vp, _vp, _vp, _vp], _i32),
    "wp_mlp_lattice_coords": ([_vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "wp_mlp_check_table": ([_vp, _vp, _PG, _i32, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "wp_mlp_row_check": ([_vp, _vp, _i32, _i32, _vp, _i64, _vp, _vp, _vp], _i32),
    "wp_surrogate_create": ([C.POINTER(_vp), _vp, _vp, _i64, _vp, _vp, _vp, _vp, _d, _pi64, _vp], _i32),
    "wp_surrogate_destroy": ([_vp], _i32),
    "wp_surrogate_info": ([_vp, _pi64], _i32),
    "wp_surrogate_slots": ([_vp, _vp, _vp], _i32),
    "wp_surrogate_fallback_coords": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "wp_surrogate_degrid": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "wp_surrogate_grid_add": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "wp_surrogate_apply_Phi": ([_vp, _vp, _PG, _vp, _vp, _vp, _vp], _i32),
    "wp_surrogate_apply_PhiT": ([_vp, _vp, _PG, _vp, _vp, _vp, _vp], _i32),
    "wp_surrogate_to_slots": ([_vp, _PG, _vp, _vp, _vp], _i32),
    "wp_surrogate_solver_workspace_bytes": ([_vp, _vp, _pi64], _i32),
    "wp_surrogate_power_norm2": ([_vp, _vp, _PG, _vp, _i32, _vp, C.POINTER(C.c_double), _vp], _i32),
    "wp_surrogate_solve": ([_vp, _vp, _PG, _vp, _d, _d, _i32, _i32, _vp, _vp, _vp], _i32),
    "wp_dwt2": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "wp_idwt2": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "wp_solver_workspace_bytes": ([_vp, _PG, _pi64], _i32),
    "wp_power_norm2": ([_vp, _PG, _vp, _i32, _vp, C.POINTER(C.c_double), _vp], _i32),
    "wp_solve": ([_vp, _PG, _vp, _d, _d, _i32, _i32, _vp, _vp, _vp], _i32),
    "wp_dr_workspace_bytes": ([_vp, _PG, _pi64], _i32),
    "wp_dr_solve": ([_vp, _PG, _vp, _d, _d, _i32, _i32, _d, _i32, _vp, _vp, _vp], _i32),
    "wp_sara_analysis": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "wp_sara_synthesis": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "wp_sara_workspace_bytes": ([_vp, _PG, _pi64], _i32),
    "wp_sara_solve": ([_vp, _PG, _vp, _d, _d, _i32, _i32, _i32, _vp, _vp, _vp], _i32),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libwproj.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname: importing it first makes
        # the library bind to that runtime instead of loading a second one beside it
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise OSError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        lib = C.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


class WprojError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().wp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != 0:
        raise WprojError(status, where)
