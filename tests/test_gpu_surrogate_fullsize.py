"""The surrogate operator's products at the 2048-pixel form's full size (N = 2048, Ng = 4096,
M = 16 777 216, every visibility a network row of a seeded network) against the oracle's surrogate
rows on a seeded 4096-visibility sample, in the launch forms the benchmark times (the LDS-ring
degridding and gridding): degridding of a random grid on the sampled rows; gridding of visibilities
that are non-zero on the sampled rows only, compared over the whole grid.

Tolerances: the products take the grid values and the per-cell sums s_c in bfloat16 (relative
rounding 2^-9 per value, FP32 accumulation), against FP64 rows with the oracle rounding the hidden
layers and weights as the products do (`q=round_bf16`): per-row errors below 1e-2 of the row's
absolute sum, 3e-3 in norm.
"""
import numpy as np
import pytest

import synth
from oracle import surrogate as S
from oracle.wproj import Setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1307_3424_amd as wp  # noqa: E402

ROWS = 4096


def test_surrogate_products_full_size():
    wl = synth.workload(4)
    _, u, v, w = synth.workload_inputs(wl, with_sky=False)
    s = Setup(N=wl.N, L=wl.L)
    rows = synth.subset_rows(wl.M, ROWS, synth.rng_for(wl.seed, "subset"))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = wp.Plan(wl.N, wl.L, kb_W=wl.W)
    mlp = wp.Mlp(max_batch=8192)
    s_out = wp.Mlp.output_scale(plan)
    params = synth.mlp_init(wl.seed + 1)
    mlp.set_params(params, wl.w_top, s_out)
    net = S.from_packed(params, w_top=wl.w_top, s_out=s_out)
    print(f"full size {wl.name}: surrogate set-up for {wl.M} rows", flush=True)
    sur = wp.Surrogate(plan, mlp, t(u), t(v), t(w))
    assert sur.Ms == wl.M and sur.Mf == 0
    slot = sur.slots().cpu().numpy()
    pos = np.empty(wl.M, dtype=np.int64)
    pos[slot] = np.arange(wl.M)                      # slot of each caller index
    cols, taps = S.surrogate_rows(net, u[rows], v[rows], w[rows], s, q=S.round_bf16)
    Ng = s.Ng
    # degridding
    X = synth.random_complex(Ng * Ng, synth.rng_for(wl.seed, "y", 5)).astype(np.complex64)
    y = sur.degrid(t(X)).cpu().numpy()[pos[rows]]
    Xc = X.astype(np.complex128)[cols]
    y_ref = np.einsum("kp,kp->k", taps, Xc)
    scale = np.sum(np.abs(taps) * np.abs(Xc), axis=1)
    print(f"degrid: largest row error {np.max(np.abs(y - y_ref) / scale):.2e} of the row's absolute sum", flush=True)
    assert np.all(np.abs(y - y_ref) <= 1e-2 * scale)
    assert np.linalg.norm(y - y_ref) <= 3e-3 * np.linalg.norm(y_ref)
    # gridding of visibilities non-zero on the sampled rows only
    yv = synth.random_complex(ROWS, synth.rng_for(wl.seed, "y", 6))
    ys = np.zeros(wl.M, dtype=np.complex64)
    ys[pos[rows]] = yv
    g = torch.zeros(Ng * Ng, dtype=torch.complex64, device="cuda")
    got = sur.grid_add(t(ys), g).cpu().numpy()
    ref = np.zeros(Ng * Ng, dtype=np.complex128)
    np.add.at(ref, cols.ravel(), (np.conj(taps) * yv[:, None]).ravel())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"grid: relative error {err:.2e}; cells outside the sampled boxes "
          f"{np.count_nonzero(got[ref == 0])} non-zero", flush=True)
    assert err <= 3e-3
    assert np.count_nonzero(got[ref == 0]) == 0
    sur.close()
    mlp.close()
    plan.close()
