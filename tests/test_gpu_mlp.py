"""Surrogate network on the GPU (wp_mlp_*) against the oracle's network with the same
bfloat16 rounding points (oracle/surrogate.py)."""
import numpy as np
import pytest

from oracle import surrogate as S
from oracle import wproj
from synth import configs, generators as gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
W = pytest.importorskip("paper_1307_3424_amd")


def _feat(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)], 1).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def mlp():
    m = W.Mlp(max_batch=1024)
    yield m
    m.close()


def _set(m, seed, w_top=1.0, s_out=1.0):
    p = gen.mlp_init(seed)
    m.set_params(p, w_top, s_out)
    return p


@pytest.mark.parametrize("n", [512, 200, 1])
def test_forward_matches_oracle(mlp, n):
    p = _set(mlp, 1)
    X = _feat(n, 2)
    out = mlp.forward(_dev(X.ravel())).cpu().numpy().reshape(n, -1)
    ref, _ = S.forward(S.from_packed(p), X.astype(np.float64), q=S.round_bf16)
    # FP32 sums (relative error ~1.6e-7 per pre-activation) against FP64: an activation whose
    # value lies that close to a bfloat16 rounding boundary rounds the other way on one side
    # (probability ~8e-5 each, ~6% of rows over 768 activations); one such step of 2^-8 moves
    # the row's outputs by ~1e-3 relative.  Rows without one agree to ~1e-6.
    rel = np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert rel.max() < 3e-3
    assert np.mean(rel > 1e-5) < 0.2
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 5e-4


def test_gradients_match_oracle(mlp):
    n = 512
    p = _set(mlp, 3)
    X = _feat(n, 4)
    T = np.random.default_rng(5).normal(size=(n, 2048)).astype(np.float32) * 0.05
    g_gpu, loss = mlp.gradients(_dev(X.ravel()), _dev(T.ravel()))
    g_gpu = g_gpu.cpu().numpy()
    net = S.from_packed(p)
    o, cache = S.forward(net, X.astype(np.float64), q=S.round_bf16)
    l_ref, dO = S.mse_loss(o, T.astype(np.float64))
    g_ref = S.backward(net, cache, dO, q=S.round_bf16)
    assert abs(loss - l_ref) <= 1e-5 * l_ref
    g_dev = S.from_packed(g_gpu)
    for k in net.NAMES:
        a, b = getattr(g_dev, k), g_ref[k]
        # same bfloat16 boundary effect as the forward test, summed over the batch
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b), k


def test_forward_and_gradients_match_fp64_network(mlp):
    """Against the plain FP64 network (no rounding model): the bfloat16 products with FP32
    accumulation stay within P12's 1e-2 relative error, outputs and every parameter's gradient."""
    n = 512
    p = _set(mlp, 15)
    X = _feat(n, 16)
    T = np.random.default_rng(17).normal(size=(n, 2048)).astype(np.float32) * 0.05
    net = S.from_packed(p)
    out = mlp.forward(_dev(X.ravel())).cpu().numpy().reshape(n, -1)
    o, cache = S.forward(net, X.astype(np.float64))
    e_out = np.linalg.norm(out - o) / np.linalg.norm(o)
    g_gpu, loss = mlp.gradients(_dev(X.ravel()), _dev(T.ravel()))
    l_ref, dO = S.mse_loss(o, T.astype(np.float64))
    g_ref = S.backward(net, cache, dO)
    g_dev = S.from_packed(g_gpu.cpu().numpy())
    e_grad = {k: float(np.linalg.norm(getattr(g_dev, k) - g_ref[k]) / np.linalg.norm(g_ref[k])) for k in net.NAMES}
    print(f"fp64 network: output rel err {e_out:.2e}, loss rel err {abs(loss - l_ref) / l_ref:.2e}, "
          f"gradients {e_grad}", flush=True)
    assert e_out < 1e-2
    assert abs(loss - l_ref) < 1e-2 * l_ref
    for k, e in e_grad.items():
        assert e < 1e-2, k


def test_adam_step_matches_oracle(mlp):
    n = 256
    p = _set(mlp, 6)
    X = _feat(n, 7)
    T = np.random.default_rng(8).normal(size=(n, 2048)).astype(np.float32) * 0.05
    net = S.from_packed(p)
    st = S.adam_init(net)
    for it in range(3):
        before = S.from_packed(mlp.get_params()[0])
        g_gpu, _ = mlp.gradients(_dev(X.ravel()), _dev(T.ravel()))
        mlp.adam_step(2e-3)
        # the oracle's Adam on the device's parameters and gradients isolates the update
        for k in net.NAMES:
            setattr(net, k, getattr(before, k))
        S.adam_step(net, S.from_packed(g_gpu.cpu().numpy()).params(), st, lr=2e-3)
        got = S.from_packed(mlp.get_params()[0])
        for k in net.NAMES:
            a, b = getattr(got, k), getattr(net, k)
            assert np.max(np.abs(a - b)) <= 2e-6 * (np.max(np.abs(b)) + 2e-3), (it, k)


def test_training_fits_a_teacher(mlp):
    n = 4096
    _set(mlp, 9)
    X = _feat(n, 10)
    teacher = S.from_packed(gen.mlp_init(11))
    T, _ = S.forward(teacher, X.astype(np.float64))
    T = (T / np.std(T)).astype(np.float32)
    hist = mlp.train(_dev(X.ravel()), _dev(T.ravel()), batch=512, epochs=40, lr_max=2e-3)
    assert hist[-1] < 0.1 * hist[0], hist[::8]
    assert all(np.isfinite(hist))


def _vis(M, N, seed, support=24):
    L = configs.workload(0).L
    rng = np.random.default_rng(seed)
    B = N / (2 * L)
    u = rng.uniform(-B, B, M)
    v = rng.uniform(-B, B, M)
    w_top = configs.w_for_support(support, 4, L)
    w = rng.uniform(0, w_top, M)
    return L, u, v, w, w_top


def test_features_match_oracle(mlp):
    N = 64
    L, u, v, w, w_top = _vis(300, N, 12)
    plan = W.Plan(N, L)
    _set(mlp, 1, w_top=w_top)
    f = mlp.features(plan, _dev(u), _dev(v), _dev(w)).cpu().numpy().reshape(-1, 3)
    s = wproj.Setup(N=N, L=L)
    _, du = S.nearest_cell(u / (1 / (2 * L)))
    _, dv = S.nearest_cell(v / (1 / (2 * L)))
    ref = S.features(w, du, dv, w_top)
    assert np.max(np.abs(f - ref)) < 1e-6
    # outside the grid: the error flag
    bad = u.copy()
    bad[3] = 10 * N / (2 * L)
    with pytest.raises(W.WprojError):
        mlp.features(plan, _dev(bad), _dev(v), _dev(w))
    plan.close()
    del s


@pytest.mark.parametrize("order", [W.WP_ORDER_CALLER, W.WP_ORDER_SORTED])
def test_box_targets_and_row_errors_match_oracle(mlp, order):
    N, M = 64, 240
    L, u, v, w, w_top = _vis(M, N, 13)
    plan = W.Plan(N, L)
    ud, vd, wd = _dev(u), _dev(v), _dev(w)
    G = W.build_G(plan, ud, vd, wd, 0.99, transpose=False)
    G.order = order
    s_out = 0.02
    target, lost = mlp.box_targets(plan, G, ud, vd, s_out)
    s = wproj.Setup(N=N, L=L)
    Gr = wproj.build_rows(u, v, w, 0.99, s)
    cols, t_ref, lost_ref = S.exact_rows_in_box(Gr, u, v, s)
    tg = target.cpu().numpy().reshape(M, -1, 2)
    tg = (tg[..., 0] + 1j * tg[..., 1]) * s_out
    assert np.max(lost.cpu().numpy()) == 0.0 and np.max(lost_ref) == 0.0
    assert np.max(np.abs(tg - t_ref)) <= 1e-5 * np.max(np.abs(t_ref))
    # per-row energy error of a random network (scaled so the errors are O(1))
    p = _set(mlp, 14, w_top=w_top, s_out=s_out)
    feat = mlp.features(plan, ud, vd, wd)
    eps = mlp.row_errors(plan, G, ud, vd, feat).cpu().numpy()
    net = S.from_packed(p, w_top=w_top, s_out=s_out)
    eps_ref = S.row_errors(net, u, v, w, Gr, s, q=S.round_bf16)
    np.testing.assert_allclose(eps, eps_ref, rtol=2e-3)
    plan.close()
