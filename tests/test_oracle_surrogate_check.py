"""Pins of the oracle's run-time row check (oracle/surrogate.py: lattice_coords, check_table,
check_estimate) against what the mathematics fixes, on the CPU:

* a row's energy before sparsifying is (sum over its window of KB^2)^2 at every w (shifted chirp
  spectra are orthonormal: the chirp has unit modulus on the padded grid), so a node's kept energy K
  lies in [E T, T] with T from that closed form;
* at a lattice node the estimate's energy term is the reverse triangle inequality's bound, never above
  the node's true error, and the estimate is at least the true error there (the corner maximum
  includes the node itself);
* rows outside the lattice (w above the trained range) get +infinity;
* the lattice's last offset node keeps the centre cell as its nearest.
"""
import numpy as np

import synth
from oracle import kb, surrogate as S, wproj
from oracle.wproj import Setup

N = 64


def _setup():
    L = synth.fov_L()
    s = Setup(N=N, L=L)
    w_top = synth.configs.w_for_support(24, 4, L)
    net = S.from_packed(synth.mlp_init(21), w_top=w_top, s_out=0.02)
    return s, net, w_top


def _T(ut, vt, s):
    tu = kb.kb_taps(ut, s.W, s.beta)[1]
    tv = kb.kb_taps(vt, s.W, s.beta)[1]
    return float(np.sum(np.asarray(tu) ** 2) * np.sum(np.asarray(tv) ** 2))


def test_lattice_nodes_keep_the_centre_cell():
    s, net, w_top = _setup()
    u, v, w = S.lattice_coords(3, 5, w_top, s)
    cell = 1 / (2 * s.L)
    c, d = S.nearest_cell(u / cell)
    assert np.all(c == 0) and d.min() == -0.5 and d.max() < 0.5
    assert w.min() == 0.0 and w.max() == w_top


def test_table_kept_energy_within_closed_form_bounds():
    s, net, w_top = _setup()
    E = 0.9
    eps, K = S.check_table(net, E, 3, 3, s)
    u, v, w = S.lattice_coords(3, 3, w_top, s)
    cell = 1 / (2 * s.L)
    for k in range(u.size):
        T = _T(u[k] / cell, v[k] / cell, s)
        assert E * T * (1 - 1e-9) <= K[k] <= T * (1 + 1e-9), k


def test_estimate_bounds_true_error_at_nodes():
    s, net, w_top = _setup()
    E = 0.99
    nw, nd = 3, 3
    eps, K = S.check_table(net, E, nw, nd, s)
    u, v, w = S.lattice_coords(nw, nd, w_top, s)
    est = S.check_estimate(net, u, v, w, eps, K, nw, nd, s)
    assert np.all(est >= eps * (1 - 1e-12))
    # the energy term alone never exceeds the true error (a table with zero node errors isolates it)
    lb = S.check_estimate(net, u, v, w, np.zeros_like(eps), K, nw, nd, s)
    assert np.all(lb <= eps * (1 + 1e-9))
    G = wproj.build_rows(u, v, w, E, s)
    assert np.allclose(K, np.asarray(abs(G).power(2).sum(axis=1)).ravel(), rtol=1e-12)


def test_estimate_infinite_outside_the_lattice():
    s, net, w_top = _setup()
    nw, nd = 3, 3
    eps, K = np.zeros(nw * nd * nd), np.ones(nw * nd * nd)
    cell = 1 / (2 * s.L)
    u = np.array([0.1, 0.2]) * cell
    v = np.array([-0.3, 0.4]) * cell
    w = np.array([0.5 * w_top, 1.5 * w_top])
    est = S.check_estimate(net, u, v, w, eps, K, nw, nd, s)
    assert np.isfinite(est[0]) and est[1] == np.inf
