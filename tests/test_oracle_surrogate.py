"""Pins of the surrogate oracle (oracle/surrogate.py) against facts outside it."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from oracle import wproj
from synth import generators as gen


def test_gelu_odd_part_and_limits():
    x = np.linspace(-6, 6, 241)
    # x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x)) = x
    assert np.max(np.abs(S.gelu(x) - S.gelu(-x) - x)) < 1e-14
    assert S.gelu(0.0) == 0.0
    assert abs(S.gelu(30.0) - 30.0) < 1e-12 and abs(S.gelu(-30.0)) < 1e-12
    # Phi(1) for the standard normal, from the error function's series at 1/sqrt(2)
    z = 1.0 / np.sqrt(2.0)
    erf_series = 2.0 / np.sqrt(np.pi) * sum((-1) ** n * z ** (2 * n + 1) / (float(math.factorial(n)) * (2 * n + 1))
                                             for n in range(30))
    assert abs(S.gelu(1.0) - 0.5 * (1.0 + erf_series)) < 1e-14
    for v in (-2.3, -0.4, 0.0, 0.7, 3.1):
        assert abs(S.gelu(v) - S.gelu_scalar(v)) < 1e-15


def test_gelu_grad_is_the_derivative():
    x = np.linspace(-5, 5, 101)
    h = 1e-5
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(S.gelu_grad(x) - fd)) < 1e-9
    assert abs(S.gelu_grad(0.0) - 0.5) < 1e-15


def _tiny_net(seed=3, H=7, n_out=10):
    rng = np.random.default_rng(seed)
    return S.init_net(rng, H=H, n_out=n_out), rng


def test_backward_matches_central_differences():
    net, rng = _tiny_net()
    X = rng.uniform(-1, 1, (5, 3))
    T = rng.normal(size=(5, 10))
    o, cache = S.forward(net, X)
    _, dO = S.mse_loss(o, T)
    g = S.backward(net, cache, dO)
    h = 1e-6
    for name in net.NAMES:
        P = getattr(net, name)
        for idx in list(np.ndindex(P.shape))[:: max(1, P.size // 12)]:
            keep = P[idx]
            P[idx] = keep + h
            lp = S.mse_loss(S.forward(net, X)[0], T)[0]
            P[idx] = keep - h
            lm = S.mse_loss(S.forward(net, X)[0], T)[0]
            P[idx] = keep
            fd = (lp - lm) / (2 * h)
            assert abs(g[name][idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (name, idx, g[name][idx], fd)


def test_saturated_network_is_a_composed_affine_map():
    rng = np.random.default_rng(5)
    H, n_out = 6, 8
    X = rng.uniform(0.5, 1.0, (4, 3))
    W1 = rng.uniform(1, 2, (H, 3)); b1 = np.full(H, 10.0)
    W2 = rng.uniform(0, 1, (H, H)); b2 = np.full(H, 10.0)
    W3 = rng.uniform(0, 1, (H, H)); b3 = np.full(H, 10.0)
    W4 = rng.normal(size=(n_out, H)); b4 = rng.normal(size=n_out)
    net = S.Net(W1, b1, W2, b2, W3, b3, W4, b4)
    # every pre-activation >= 10, where gelu(z) = z to double precision
    M = W4 @ W3 @ W2 @ W1
    c = W4 @ (W3 @ (W2 @ b1 + b2) + b3) + b4
    o, _ = S.forward(net, X)
    assert np.max(np.abs(o - (X @ M.T + c))) < 1e-10 * np.max(np.abs(o))
    # every unit off: the output is the last bias
    off = S.Net(W1, -b1 - 20, W2, -b2 - 20, W3, -b3 - 20, W4, b4)
    o2, _ = S.forward(off, X)
    assert np.max(np.abs(o2 - b4)) < 1e-12


def test_adam_first_step_is_lr_sign():
    net, rng = _tiny_net(7)
    st = S.adam_init(net)
    before = net.copy()
    g = {k: rng.normal(size=p.shape) for k, p in net.params().items()}
    S.adam_step(net, g, st, lr=1e-3, eps=0.0)
    for k in net.NAMES:
        np.testing.assert_allclose(getattr(net, k), getattr(before, k) - 1e-3 * np.sign(g[k]), rtol=0, atol=1e-15)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    S.adam_step(net, g, st, lr=1e-3, eps=0.0)
    for k in net.NAMES:
        np.testing.assert_allclose(getattr(net, k), getattr(before, k) - 2e-3 * np.sign(g[k]), rtol=0, atol=1e-14)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(11)
    x = rng.normal(size=4096).astype(np.float32) * np.float32(1e3) ** rng.integers(-3, 3, 4096)
    # exact ties: low 16 bits 0x8000, even and odd upper halves
    bits = (rng.integers(0x3F000000 >> 16, 0x47000000 >> 16, 512).astype(np.uint32) << 16) | np.uint32(0x8000)
    x = np.concatenate([x, bits.view(np.float32), -bits.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(S.round_bf16(x), ref)


def test_nearest_cell():
    c, d = S.nearest_cell(np.array([2.5, 2.49, -0.5, -0.51, 0.0, 7.25]))
    assert list(c) == [3, 2, 0, -1, 0, 7]
    assert np.all(d >= -0.5) and np.all(d < 0.5)
    np.testing.assert_allclose(c + d, [2.5, 2.49, -0.5, -0.51, 0.0, 7.25], rtol=0, atol=1e-15)


def _small_problem(M=40, N=64, w_frac=0.5, seed=2):
    from synth import configs
    L = configs.workload(0).L
    s = wproj.Setup(N=N, L=L, W=4)
    rng = np.random.default_rng(seed)
    B = N / (2 * L)
    # keep the boxes away from nothing in particular: wrap-around is part of the definition
    u = rng.uniform(-B, B, M)
    v = rng.uniform(-B, B, M)
    w_top = configs.w_for_support(24, 4, L)
    w = rng.uniform(0, w_frac * w_top, M)
    return s, u, v, w, w_top


def test_exact_taps_in_the_box_reproduce_the_sparse_operator():
    s, u, v, w, _ = _small_problem()
    G = wproj.build_rows(u, v, w, 0.99, s)
    cols, t, lost = S.exact_rows_in_box(G, u, v, s)
    assert np.max(lost) == 0.0          # supports <= 24 cells fit the 32-cell box
    rng = np.random.default_rng(4)
    x = rng.normal(size=(s.N, s.N)) + 1j * rng.normal(size=(s.N, s.N))
    y = wproj.phi(G, x, s)
    ys = S.phi_rows(cols, t, x, s)
    assert np.max(np.abs(ys - y)) <= 1e-12 * np.max(np.abs(y))
    yy = gen.random_complex(len(u), np.random.default_rng(9))
    xa = wproj.phi_adjoint(G, yy, s)
    xs = S.phi_rows_adjoint(cols, t, yy, s)
    assert np.max(np.abs(xs - xa)) <= 1e-12 * np.max(np.abs(xa))
    # energy error of the exact box is zero, of an empty box is one
    for k in range(5):
        a, b = G.indptr[k], G.indptr[k + 1]
        cu, _ = S.nearest_cell(u[k] / (1 / (2 * s.L)))
        cv, _ = S.nearest_cell(v[k] / (1 / (2 * s.L)))
        tb = t[k].reshape(S.BOX, S.BOX)
        assert S.energy_error(tb, G.indices[a:b], G.data[a:b], int(cu), int(cv), s.Ng) == 0.0
        assert abs(S.energy_error(0 * tb, G.indices[a:b], G.data[a:b], int(cu), int(cv), s.Ng) - 1.0) < 1e-14


def test_surrogate_adjoint_identity_with_fallback_rows():
    s, u, v, w, w_top = _small_problem(M=30)
    net = S.init_net(np.random.default_rng(1), H=16, s_out=0.05, w_top=w_top)
    G = wproj.build_rows(u, v, w, 0.99, s)
    use_exact = np.zeros(len(u), dtype=bool)
    use_exact[::4] = True
    rng = np.random.default_rng(8)
    x = rng.normal(size=(s.N, s.N)) + 1j * rng.normal(size=(s.N, s.N))
    y = gen.random_complex(len(u), rng)
    for q in (S._ident, S.round_bf16):
        lhs = np.vdot(y, S.phi_s(net, u, v, w, x, s, G, use_exact, q=q))
        rhs = np.vdot(S.phi_s_adjoint(net, u, v, w, y, s, G, use_exact, q=q), x)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # all rows exact: the exact operator
    np.testing.assert_allclose(S.phi_s(net, u, v, w, x, s, G, np.ones(len(u), bool)), wproj.phi(G, x, s),
                               rtol=0, atol=1e-12 * np.max(np.abs(wproj.phi(G, x, s))))


def test_row_errors_definition():
    s, u, v, w, w_top = _small_problem(M=6)
    net = S.init_net(np.random.default_rng(2), H=8, s_out=0.01, w_top=w_top)
    G = wproj.build_rows(u, v, w, 0.99, s)
    e = S.row_errors(net, u, v, w, G, s)
    cols, t = S.surrogate_rows(net, u, v, w, s)
    cols_x, tx, _ = S.exact_rows_in_box(G, u, v, s)
    assert np.array_equal(cols, cols_x)
    ref = np.sum(np.abs(t - tx) ** 2, axis=1) / np.array([np.sum(np.abs(G.data[G.indptr[k]:G.indptr[k + 1]]) ** 2)
                                                          for k in range(len(u))])
    np.testing.assert_allclose(e, ref, rtol=1e-12)
