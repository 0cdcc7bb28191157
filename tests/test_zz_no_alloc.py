"""wp_apply_Phi_noalloc (the entry point that allocates nothing) against wp_apply_Phi, through the C
ABI: two calls in a row on the same GPU, the second on a smaller problem (so the static grid holds
the first call's larger contents when the second runs), each equal to wp_apply_Phi's result on the
same input; the capacity limit rejects a larger grid before any launch."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402
from paper_1307_3424_amd import _lib  # noqa: E402


def _problem(N, M, seed):
    L = synth.fov_L()
    rng = np.random.default_rng(seed)
    u, v, w = synth.uvw(N, M, L, "gaussian", 0.25, synth.configs.w_for_support(24, 4, L), rng)
    x = synth.sky(N, 5, 10, np.random.default_rng(seed + 1))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = wp.Plan(N, L)
    G = wp.build_G(plan, t(u), t(v), t(w), 0.99, transpose=False)
    return plan, G, t(x.astype(np.complex64).ravel())


def _noalloc(plan, G, x, y):
    d = G.desc()
    st = wp.load().wp_apply_Phi_noalloc(plan.handle, C.byref(d), C.c_void_p(x.data_ptr()),
                                        C.c_void_p(y.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("order", [wp.WP_ORDER_CALLER, wp.WP_ORDER_SORTED])
def test_noalloc_phi_matches_apply_phi_twice(order):
    for N, M, seed in ((1024, 200000, 5), (64, 900, 6)):          # Ng = 2048 (the limit), then 128
        print(f"noalloc: N={N} M={M} order={order}", flush=True)
        plan, G, x = _problem(N, M, seed)
        G.order = order
        y_ref = wp.apply_Phi(plan, G, x)
        y = torch.full((G.M,), float("nan"), dtype=torch.complex64, device="cuda")
        assert _noalloc(plan, G, x, y) == 0, wp.load().wp_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)             # same kernels on the same input: identical bits
        wp.apply_Phi_noalloc(plan, G, x, y)     # the binding's wrapper of the same call
        assert torch.equal(y, y_ref)
        plan.close()


def test_noalloc_phi_rejects_large_grid():
    plan, G, x = _problem(64, 10, 7)
    big = wp.Plan(2048, synth.fov_L())                    # Ng = 4096 > 2048
    xb = torch.zeros(2048 * 2048, dtype=torch.complex64, device="cuda")
    y = torch.zeros(G.M, dtype=torch.complex64, device="cuda")
    st = _noalloc(big, G, xb, y)
    assert _lib.STATUS[st] == "WP_ECAPACITY" and b"Ng" in wp.load().wp_last_error()
    plan.close()
    big.close()
