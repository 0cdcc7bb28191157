"""Surrogate operator on the GPU (wp_surrogate_*) against the oracle's surrogate operator
(oracle/surrogate.py), which builds every row's taps and multiplies them out plainly."""
import numpy as np
import pytest

from oracle import surrogate as S
from oracle import wproj
from synth import configs, generators as gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
W = pytest.importorskip("paper_1307_3424_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _coords(M, N, seed, frac_dense=0.5):
    """Half the visibilities Gaussian around the uv centre (several per cell, groups of many
    cells), half uniform (boxes that wrap around the grid edges)."""
    L = configs.workload(0).L
    rng = np.random.default_rng(seed)
    B = N / (2 * L)
    md = int(M * frac_dense)
    u = np.concatenate([np.clip(rng.normal(0, 0.06 * B, md), -0.99 * B, 0.99 * B), rng.uniform(-B, B, M - md)])
    v = np.concatenate([np.clip(rng.normal(0, 0.06 * B, md), -0.99 * B, 0.99 * B), rng.uniform(-B, B, M - md)])
    w_top = configs.w_for_support(24, 4, L)
    w = rng.uniform(0, w_top, M)
    return L, u, v, w, w_top


@pytest.fixture(scope="module")
def setup():
    N, M = 64, 3000
    L, u, v, w, w_top = _coords(M, N, 21)
    plan = W.Plan(N, L)
    mlp = W.Mlp(max_batch=1024)
    s_out = W.Mlp.output_scale(plan)
    params = gen.mlp_init(22)
    mlp.set_params(params, w_top, s_out)
    net = S.from_packed(params, w_top=w_top, s_out=s_out)
    s = wproj.Setup(N=N, L=L)
    yield dict(N=N, M=M, L=L, u=u, v=v, w=w, plan=plan, mlp=mlp, net=net, s=s)
    mlp.close()
    plan.close()


def _bf16_exact(shape, rng):
    """values exactly representable in bfloat16: small integers times powers of two"""
    return rng.integers(-64, 64, shape).astype(np.float64) * 2.0 ** rng.integers(-3, 3, shape)


def test_degrid_matches_oracle_on_bf16_exact_grids(setup):
    d = setup
    sur = W.Surrogate(d["plan"], d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]))
    assert sur.Ms == d["M"] and sur.Mf == 0
    assert sur.groups[0] > 1          # several degridding groups
    rng = np.random.default_rng(23)
    Ng = d["s"].Ng
    X = (_bf16_exact(Ng * Ng, rng) + 1j * _bf16_exact(Ng * Ng, rng))
    y = sur.degrid(_dev(X.astype(np.complex64))).cpu().numpy()
    slot = sur.slots().cpu().numpy()
    assert np.array_equal(np.sort(slot), np.arange(d["M"]))
    cols, t = S.surrogate_rows(d["net"], d["u"], d["v"], d["w"], d["s"], q=S.round_bf16)
    ref = np.einsum("kp,kp->k", t, X[cols])[slot]
    scale = np.sqrt(np.einsum("kp,kp->k", np.abs(t) ** 2, np.abs(X[cols]) ** 2))[slot]
    # box values are exact in bfloat16, so the rows agree to FP32 accumulation (~1e-6 of their
    # scale) except where one hidden activation rounds to the other bfloat16 neighbour on the
    # two sides (about 6% of rows; ~1e-3 of the row, as in the network's own parity test)
    rel = np.abs(y - ref) / scale
    assert rel.max() < 5e-3
    assert np.mean(rel > 2e-5) < 0.2
    assert np.linalg.norm(y - ref) <= 1e-3 * np.linalg.norm(ref)
    sur.close()


def test_degrid_forms_agree(setup):
    """The LDS-ring degridding (form 2, the default) reads the grid rounded to bfloat16, which is also
    what the register-staged form (1) feeds its products, and runs the same products in the same order;
    it sums the bias term b4 . box from the rounded grid and each visibility's dot product h . r in
    another order.  So on grids exact in bfloat16 the two differ by FP32 rounding only, and on general
    grids by at most 2^-9 of sum |b4| |X| per row and component more (the bias from the FP32 grid in
    form 1)."""
    d = setup
    plan = d["plan"]
    sur = W.Surrogate(plan, d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]))
    Ng = d["s"].Ng
    rng = np.random.default_rng(29)
    X = (_bf16_exact(Ng * Ng, rng) + 1j * _bf16_exact(Ng * Ng, rng)).astype(np.complex64)
    Xg = (rng.normal(size=Ng * Ng) + 1j * rng.normal(size=Ng * Ng)).astype(np.complex64)
    out = {}
    try:
        for form in (1, 2):
            plan.set_tuning("sur_degrid", form)
            out[form] = (sur.degrid(_dev(X)).cpu().numpy(), sur.degrid(_dev(Xg)).cpu().numpy())
    finally:
        plan.set_tuning("sur_degrid", 0)
    slot = sur.slots().cpu().numpy()
    cols, _ = S.surrogate_rows(d["net"], d["u"], d["v"], d["w"], d["s"], q=S.round_bf16)
    b4 = d["net"].b4.reshape(-1, 2)
    bmag = np.abs(b4[:, 0] + 1j * b4[:, 1]) * d["net"].s_out
    for k, (Xk, bf16_exact) in enumerate(((X, True), (Xg, False))):
        bsum = np.sum(bmag[None, :] * np.abs(Xk[cols]), axis=1)[slot]
        y1, y2 = out[1][k], out[2][k]
        bound = 2e-6 * np.abs(y1).max() + (1e-5 if bf16_exact else 2.0 ** -9 * np.sqrt(2.0) + 1e-5) * bsum
        assert np.all(np.abs(y1 - y2) <= bound), k
    sur.close()


def test_grid_add_matches_oracle_with_exact_cell_sums(setup):
    d = setup
    sur = W.Surrogate(d["plan"], d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]))
    slot = sur.slots().cpu().numpy()
    # one non-zero visibility per cell, values +-1, +-2: s_c = h_k y_k is exact in bfloat16
    cu, _ = S.nearest_cell(d["u"] * 2 * d["L"])
    cv, _ = S.nearest_cell(d["v"] * 2 * d["L"])
    _, first = np.unique(cv * 100000 + cu, return_index=True)
    rng = np.random.default_rng(24)
    yc = np.zeros(d["M"], dtype=np.complex128)
    yc[first] = rng.choice([-2.0, -1.0, 1.0, 2.0], first.size) + 1j * rng.choice([-2.0, -1.0, 1.0, 2.0], first.size)
    y_slot = yc[slot]
    Ng = d["s"].Ng
    grid = torch.zeros(Ng * Ng, dtype=torch.complex64, device="cuda")
    sur.grid_add(_dev(y_slot.astype(np.complex64)), grid)
    got = grid.cpu().numpy()
    cols, t = S.surrogate_rows(d["net"], d["u"], d["v"], d["w"], d["s"], q=S.round_bf16)
    ref = np.zeros(Ng * Ng, dtype=np.complex128)
    np.add.at(ref, cols.ravel(), (np.conj(t) * yc[:, None]).ravel())
    # s_c = h_k y_k is exact; differences come from FP32 sums and the hidden-layer rounding
    # boundary cases described in the degridding test
    assert np.linalg.norm(got - ref) <= 5e-4 * np.linalg.norm(ref)
    assert np.max(np.abs(got - ref)) <= 5e-3 * np.max(np.abs(ref))
    sur.close()


def test_grid_forms_agree(setup):
    """The LDS-ring gridding (form 2, the default: per-cell s in bfloat16, then 8 slices of 256 outputs
    per group of <= 128 cells) against the register-staged one (form 1, groups of <= 32 cells): the
    same bfloat16 products, summed in other groups, so they differ by the 32-bit fixed-point
    quantisation of each window (2^-22 of a group's largest output bound per contribution) and FP32
    rounding."""
    d = setup
    plan = d["plan"]
    sur = W.Surrogate(plan, d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]))
    Ng = d["s"].Ng
    rng = np.random.default_rng(31)
    yy = _dev((rng.normal(size=d["M"]) + 1j * rng.normal(size=d["M"])).astype(np.complex64))
    out = {}
    try:
        for form in (1, 2):
            plan.set_tuning("sur_grid", form)
            g = torch.zeros(Ng * Ng, dtype=torch.complex64, device="cuda")
            out[form] = sur.grid_add(yy, g).cpu().numpy()
    finally:
        plan.set_tuning("sur_grid", 0)
    g1, g2 = out[1], out[2]
    assert np.linalg.norm(g1 - g2) <= 1e-5 * np.linalg.norm(g1)
    assert np.max(np.abs(g1 - g2)) <= 1e-4 * np.max(np.abs(g1))
    sur.close()


def test_grid_short_groups_match_oracle(setup):
    """Sparse visibilities only (uniform over the band, few per cell): the default gridding's groups
    are cut short by their span, so most hold far fewer than 128 cells.  Their row blocks past the
    group read the zero row of the per-cell s and waves with no cell of the group skip the products;
    the sums must still match the oracle's rows and the register-staged form."""
    d = setup
    plan = d["plan"]
    M = 400
    L, u, v, w, _ = _coords(M, d["N"], 41, frac_dense=0.0)
    sur = W.Surrogate(plan, d["mlp"], _dev(u), _dev(v), _dev(w))
    slot = sur.slots().cpu().numpy()
    cu, _ = S.nearest_cell(u * 2 * L)
    cv, _ = S.nearest_cell(v * 2 * L)
    _, first = np.unique(cv * 100000 + cu, return_index=True)
    assert first.size > 300            # mostly one visibility per cell: sparse cells, short groups
    rng = np.random.default_rng(42)
    yc = np.zeros(M, dtype=np.complex128)
    yc[first] = rng.choice([-2.0, -1.0, 1.0, 2.0], first.size) + 1j * rng.choice([-2.0, -1.0, 1.0, 2.0], first.size)
    y_slot = _dev(yc[slot].astype(np.complex64))
    Ng = d["s"].Ng
    out = {}
    try:
        for form in (1, 2):
            plan.set_tuning("sur_grid", form)
            g = torch.zeros(Ng * Ng, dtype=torch.complex64, device="cuda")
            out[form] = sur.grid_add(y_slot, g).cpu().numpy()
    finally:
        plan.set_tuning("sur_grid", 0)
    cols, t = S.surrogate_rows(d["net"], u, v, w, d["s"], q=S.round_bf16)
    ref = np.zeros(Ng * Ng, dtype=np.complex128)
    np.add.at(ref, cols.ravel(), (np.conj(t) * yc[:, None]).ravel())
    got = out[2]
    assert np.linalg.norm(got - ref) <= 5e-4 * np.linalg.norm(ref)
    assert np.max(np.abs(got - ref)) <= 5e-3 * np.max(np.abs(ref))
    assert np.linalg.norm(out[1] - got) <= 1e-5 * np.linalg.norm(out[1])
    # nothing outside the union of the rows' boxes
    assert np.all(got[np.setdiff1d(np.arange(Ng * Ng), np.unique(cols))] == 0)
    sur.close()


def _fallback_setup(d, every=5):
    eps = np.zeros(d["M"], dtype=np.float32)
    eps[::every] = 1.0                  # these rows fail the check
    return eps


@pytest.mark.parametrize("fallback", [False, True])
def test_operator_and_adjoint_match_oracle(setup, fallback):
    d = setup
    ud, vd, wd = _dev(d["u"]), _dev(d["v"]), _dev(d["w"])
    eps = _fallback_setup(d) if fallback else None
    sur = W.Surrogate(d["plan"], d["mlp"], ud, vd, wd, eps=None if eps is None else _dev(eps), tol=0.5)
    Gf = None
    if fallback:
        assert sur.Mf == (d["M"] + 4) // 5
        fu, fv, fw = sur.fallback_coords()
        Gf = W.build_G(d["plan"], fu, fv, fw, 0.99)
        Gf.order = W.WP_ORDER_CALLER
    slot = sur.slots().cpu().numpy()
    use_exact = None if eps is None else eps > 0.5
    Gr = wproj.build_rows(d["u"], d["v"], d["w"], 0.99, d["s"])
    rng = np.random.default_rng(25)
    N = d["N"]
    x = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    y = sur.apply_Phi(_dev(x.astype(np.complex64).ravel()), Gf=Gf).cpu().numpy()
    ref = S.phi_s(d["net"], d["u"], d["v"], d["w"], x, d["s"], Gr, use_exact, q=S.round_bf16)[slot]
    # bfloat16 box values (relative rounding 2^-9) in the surrogate rows: ~1e-3 relative
    assert np.linalg.norm(y - ref) <= 3e-3 * np.linalg.norm(ref)
    if fallback:
        tail = slice(sur.Ms, None)      # exact rows: complex64 taps only
        assert np.linalg.norm(y[tail] - ref[tail]) <= 1e-5 * np.linalg.norm(ref[tail])
    yy = gen.random_complex(d["M"], rng)
    xa = sur.apply_PhiT(_dev(yy.astype(np.complex64)), Gf=Gf).cpu().numpy().reshape(N, N)
    yc = np.empty_like(yy)
    yc[slot] = yy
    refa = S.phi_s_adjoint(d["net"], d["u"], d["v"], d["w"], yc, d["s"], Gr, use_exact, q=S.round_bf16)
    assert np.linalg.norm(xa - refa) <= 3e-3 * np.linalg.norm(refa)
    # adjoint identity of the GPU pair
    lhs = np.vdot(yy, y)
    rhs = np.vdot(xa.ravel(), x.ravel())
    assert abs(lhs - rhs) <= 5e-3 * abs(lhs)
    sur.close()


def test_all_rows_fall_back(setup):
    d = setup
    eps = np.ones(d["M"], dtype=np.float32)
    sur = W.Surrogate(d["plan"], d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]), eps=_dev(eps), tol=1e-3)
    assert sur.Ms == 0 and sur.Mf == d["M"]
    fu, fv, fw = sur.fallback_coords()
    Gf = W.build_G(d["plan"], fu, fv, fw, 0.99)
    Gf.order = W.WP_ORDER_CALLER
    x = np.random.default_rng(26).normal(size=d["N"] ** 2).astype(np.complex64)
    y = sur.apply_Phi(_dev(x), Gf=Gf).cpu().numpy()
    yref = W.apply_Phi(d["plan"], Gf, _dev(x)).cpu().numpy()
    assert np.array_equal(y, yref)
    sur.close()


def test_single_visibility_and_crowded_cell(setup):
    d = setup
    plan, mlp = d["plan"], d["mlp"]
    one = [_dev(a[:1]) for a in (d["u"], d["v"], d["w"])]
    sur = W.Surrogate(plan, mlp, *one)
    assert sur.Ms == 1 and sur.ncell == 1
    Ng = d["s"].Ng
    X = np.zeros(Ng * Ng, dtype=np.complex64)
    X[::7] = 1.0
    y = sur.degrid(_dev(X)).cpu().numpy()
    cols, t = S.surrogate_rows(d["net"], d["u"][:1], d["v"][:1], d["w"][:1], d["s"], q=S.round_bf16)
    assert abs(y[0] - np.sum(t[0] * X[cols[0]])) <= 1e-5 * np.sum(np.abs(t[0]))
    sur.close()
    # many visibilities in one cell (one degridding group, one gridding group)
    M = 12801
    same = [_dev(np.full(M, a[0])) for a in (d["u"], d["v"], d["w"])]
    sur = W.Surrogate(plan, mlp, *same)
    assert sur.ncell == 1 and sur.groups == (1, 1)
    y = sur.degrid(_dev(X)).cpu().numpy()
    ref = np.sum(t[0] * X[cols[0]])
    assert np.all(y == y[0])
    assert abs(y[0] - ref) <= 1e-5 * np.sum(np.abs(t[0]))
    yy = np.full(M, 1.0 + 0.5j, dtype=np.complex64)
    g = torch.zeros(Ng * Ng, dtype=torch.complex64, device="cuda")
    got = sur.grid_add(_dev(yy), g).cpu().numpy()
    refg = np.zeros(Ng * Ng, dtype=np.complex128)
    np.add.at(refg, cols[0], np.conj(t[0]) * (M * (1.0 + 0.5j)))
    # the cell sum s_c = M h y is rounded to bfloat16 once: relative 2^-9
    assert np.linalg.norm(got - refg) <= 4e-3 * np.linalg.norm(refg)
    sur.close()


def test_to_slots_with_sorted_fallback(setup):
    d = setup
    eps = _fallback_setup(d, every=3)
    sur = W.Surrogate(d["plan"], d["mlp"], _dev(d["u"]), _dev(d["v"]), _dev(d["w"]), eps=_dev(eps), tol=0.5)
    fu, fv, fw = sur.fallback_coords()
    Gf = W.build_G(d["plan"], fu, fv, fw, 0.99)
    Gf.order = W.WP_ORDER_SORTED
    yc = gen.random_complex(d["M"], np.random.default_rng(27)).astype(np.complex64)
    ys = sur.to_slots(_dev(yc), Gf=Gf).cpu().numpy()
    slot = sur.slots().cpu().numpy()
    perm = Gf.perm.cpu().numpy()
    Ms = sur.Ms
    assert np.array_equal(ys[:Ms], yc[slot[:Ms]])
    assert np.array_equal(ys[Ms:], yc[slot[Ms + perm]])
    sur.close()


def test_surrogate_solve_matches_oracle():
    import synth
    from oracle import metrics, solver
    wl = synth.workload(0)
    x, u, v, w = synth.workload_inputs(wl)
    s = wproj.Setup(N=wl.N, L=wl.L)
    plan = W.Plan(wl.N, wl.L)
    mlp = W.Mlp(max_batch=1024)
    s_out = W.Mlp.output_scale(plan)
    params = gen.mlp_init(31)
    mlp.set_params(params, wl.w_top, s_out)
    net = S.from_packed(params, w_top=wl.w_top, s_out=s_out)
    rows_eps = np.zeros(wl.M, dtype=np.float32)
    rows_eps[::3] = 1.0
    use_exact = rows_eps > 0.5
    Gr = wproj.build_rows(u, v, w, wl.E, s)
    A = lambda z: S.phi_s(net, u, v, w, z, s, Gr, use_exact, q=S.round_bf16)
    AH = lambda r: S.phi_s_adjoint(net, u, v, w, r, s, Gr, use_exact, q=S.round_bf16)
    y0 = A(x)
    sig = metrics.noise_sigma(y0, wl.snr_in_db)
    y = y0 + synth.noise(wl.M, sig, synth.rng_for(wl.seed, "noise"))
    eps = metrics.l2_ball_radius(sig, wl.M)
    x0 = synth.rng_for(wl.seed, "x").normal(size=(wl.N, wl.N))
    sur = W.Surrogate(plan, mlp, _dev(u), _dev(v), _dev(w), eps=_dev(rows_eps), tol=0.5)
    fu, fv, fw = sur.fallback_coords()
    Gf = W.build_G(plan, fu, fv, fw, wl.E)
    Gf.order = W.WP_ORDER_SORTED
    nu_ref = solver.power_norm2(A, AH, x0, 30)
    nu_gpu = sur.power_norm2(_dev(x0.astype(np.float32).ravel()), 30, Gf=Gf)
    # bfloat16 box values and cell sums in the surrogate rows: ~1e-3 per application
    assert abs(nu_gpu - nu_ref) / nu_ref < 1e-2
    ys = sur.to_slots(_dev(y.astype(np.complex64)), Gf=Gf)
    x5 = sur.solve(ys, eps, nu_ref, 5, Gf=Gf).cpu().numpy().reshape(wl.N, wl.N)
    x5_ref = solver.solve(y, A, AH, (wl.N, wl.N), eps, nu_ref, 5)
    assert np.linalg.norm(x5 - x5_ref) / np.linalg.norm(x5_ref) < 1e-2
    sur.close()
    mlp.close()
