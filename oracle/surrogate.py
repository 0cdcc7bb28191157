"""Learned surrogate of the sparsified w-projection rows, in FP64.

Test infrastructure (see the package header).

Each row of G (Section 3.1 with the energy rule of Section 3.2) depends on
the visibility only through its w and the fractional position of (u~, v~)
relative to the grid: the row of a visibility at u~ = c + du is the row of a
visibility at du shifted by c cells.  The surrogate maps (w, du, dv) to the
row's taps in a fixed box of grid cells around the nearest cell:

* nearest cell c = floor(u~ + 1/2), offset du = u~ - c in [-1/2, 1/2);
* the box is BOX x BOX cells (BOX = 32); box position (oy, ox) is grid cell
  ((c_v + Ng/2 + oy - BOX/2) mod Ng, (c_u + Ng/2 + ox - BOX/2) mod Ng)
  (grid index q = c + Ng/2 holds coordinate c, as in geometry.py);
* the network is an MLP 3 -> H -> H -> H -> 2 BOX^2 with GELU after the
  three hidden layers: a_1 = gelu(W1 f + b1), a_l = gelu(W_l a_{l-1} + b_l),
  o = W4 a_3 + b4, with input features f = (2 w / w_top - 1, 2 du, 2 dv);
* taps: t(oy, ox) = s_out (o[2 p] + i o[2 p + 1]), p = BOX oy + ox, with a
  fixed output scale s_out;
* gelu(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 (the exact form, not the
  tanh approximation).

Surrogate operator: y_k = sum over box cells of t_k(cell) X[cell] for a row
that passes the per-row check, the exact sparsified row otherwise; the
adjoint scatters conj(t_k) y_k back onto the box.  The per-row check is the
energy of the difference between the surrogate taps and the exact sparsified
row, relative to the energy of that row:
    eps_k = ||t_k - g_k||^2 / ||g_k||^2
(entries of g_k outside the box count in full); rows with eps_k above the
tolerance use the exact row.

Training: mean squared error over the 2 BOX^2 outputs against the exact
sparsified rows divided by s_out, Adam (Kingma & Ba 2015) with bias
correction.  Mixed precision is modelled by an optional rounding applied to
both operands of every matrix product except the first layer's (K = 3):
forward products W_l a_{l-1} (l = 2..4), backward products dZ_l W_l and
dZ_l^T a_{l-1}.  Sums, biases, GELU and its derivative stay unrounded.

Pins (tests/test_oracle_surrogate.py): GELU odd-part identity and limits,
backward against central finite differences of the loss for every
parameter, the network reducing to a composed affine map when every hidden
unit is saturated on, the first Adam step equal to lr sign(g), bfloat16
rounding against torch's conversion, exact taps in the box reproducing the
pinned sparse operator, and the adjoint identity of the surrogate operator.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import erf, sqrt

import numpy as np
from scipy.special import erf as _erf_vec

from . import geometry as geo

BOX = 32
HIDDEN = 256
N_OUT = 2 * BOX * BOX


# ----------------------------------------------------------------------------- rounding

def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via float32; returns float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


# ----------------------------------------------------------------------------- GELU

def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + _erf_vec(x / sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + _erf_vec(x / sqrt(2.0))) + x * np.exp(-0.5 * x * x) / sqrt(2.0 * np.pi)


def gelu_scalar(x: float) -> float:
    return 0.5 * x * (1.0 + erf(x / sqrt(2.0)))


# ----------------------------------------------------------------------------- network

@dataclass
class Net:
    W1: np.ndarray   # [H, 3]
    b1: np.ndarray   # [H]
    W2: np.ndarray   # [H, H]
    b2: np.ndarray
    W3: np.ndarray   # [H, H]
    b3: np.ndarray
    W4: np.ndarray   # [2 BOX^2, H]
    b4: np.ndarray   # [2 BOX^2]
    s_out: float = 1.0
    w_top: float = 1.0

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")

    def params(self):
        return {k: getattr(self, k) for k in self.NAMES}

    def copy(self) -> "Net":
        return Net(**{k: np.array(v, dtype=np.float64) for k, v in self.params().items()},
                   s_out=self.s_out, w_top=self.w_top)


def init_net(rng: np.random.Generator, H: int = HIDDEN, n_out: int = N_OUT, s_out: float = 1.0,
             w_top: float = 1.0) -> Net:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    def lin(n, k):
        a = 1.0 / sqrt(k)
        return rng.uniform(-a, a, (n, k)), rng.uniform(-a, a, n)
    W1, b1 = lin(H, 3)
    W2, b2 = lin(H, H)
    W3, b3 = lin(H, H)
    W4, b4 = lin(n_out, H)
    return Net(W1, b1, W2, b2, W3, b3, W4, b4, s_out=s_out, w_top=w_top)


def features(w, du, dv, w_top: float) -> np.ndarray:
    """[n, 3] inputs (2 w / w_top - 1, 2 du, 2 dv)."""
    return np.stack([2.0 * np.asarray(w, dtype=np.float64) / w_top - 1.0,
                     2.0 * np.asarray(du, dtype=np.float64), 2.0 * np.asarray(dv, dtype=np.float64)], axis=1)


def forward(net: Net, X: np.ndarray, q=_ident):
    """Outputs o [n, n_out] and the cache for backward.  X: [n, 3]."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ net.W1.T + net.b1
    a1 = gelu(z1)
    z2 = q(a1) @ q(net.W2).T + net.b2
    a2 = gelu(z2)
    z3 = q(a2) @ q(net.W3).T + net.b3
    a3 = gelu(z3)
    o = q(a3) @ q(net.W4).T + net.b4
    return o, dict(X=X, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3)


def hidden(net: Net, X: np.ndarray, q=_ident) -> np.ndarray:
    """a_3, the last hidden layer [n, H]."""
    return forward(net, X, q)[1]["a3"]


def mse_loss(o: np.ndarray, T: np.ndarray):
    """(loss, dL/do) with loss = mean over all entries of (o - T)^2."""
    d = o - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(net: Net, cache, dO: np.ndarray, q=_ident):
    """Gradients of the loss with respect to every parameter, given dL/do."""
    g = {}
    g["W4"] = q(dO).T @ q(cache["a3"])
    g["b4"] = dO.sum(axis=0)
    dz3 = (q(dO) @ q(net.W4)) * gelu_grad(cache["z3"])
    g["W3"] = q(dz3).T @ q(cache["a2"])
    g["b3"] = dz3.sum(axis=0)
    dz2 = (q(dz3) @ q(net.W3)) * gelu_grad(cache["z2"])
    g["W2"] = q(dz2).T @ q(cache["a1"])
    g["b2"] = dz2.sum(axis=0)
    dz1 = (q(dz2) @ q(net.W2)) * gelu_grad(cache["z1"])
    g["W1"] = dz1.T @ cache["X"]
    g["b1"] = dz1.sum(axis=0)
    return g


@dataclass
class AdamState:
    m: dict
    v: dict
    t: int = 0


def adam_init(net: Net) -> AdamState:
    return AdamState({k: np.zeros_like(p) for k, p in net.params().items()},
                     {k: np.zeros_like(p) for k, p in net.params().items()}, 0)


def adam_step(net: Net, grads: dict, st: AdamState, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam update in place (Kingma & Ba 2015, with bias correction)."""
    st.t += 1
    c1 = 1.0 - beta1 ** st.t
    c2 = 1.0 - beta2 ** st.t
    for k in net.NAMES:
        gk = grads[k]
        st.m[k] = beta1 * st.m[k] + (1.0 - beta1) * gk
        st.v[k] = beta2 * st.v[k] + (1.0 - beta2) * gk * gk
        mh = st.m[k] / c1
        vh = st.v[k] / c2
        setattr(net, k, getattr(net, k) - lr * mh / (np.sqrt(vh) + eps))


# ----------------------------------------------------------------------------- box geometry

def nearest_cell(gt):
    """(c, d): c = floor(g + 1/2) (integer), d = g - c in [-1/2, 1/2)."""
    gt = np.asarray(gt, dtype=np.float64)
    c = np.floor(gt + 0.5)
    return c.astype(np.int64), gt - c


def box_columns(cu: int, cv: int, Ng: int) -> np.ndarray:
    """Flattened grid indices of the BOX x BOX box, in (oy, ox) order."""
    o = np.arange(BOX) - BOX // 2
    qv = (cv + Ng // 2 + o) % Ng
    qu = (cu + Ng // 2 + o) % Ng
    return (qv[:, None] * Ng + qu[None, :]).ravel()


def taps(net: Net, w, du, dv, q=_ident) -> np.ndarray:
    """Surrogate taps [n, BOX, BOX] (complex)."""
    o, _ = forward(net, features(w, du, dv, net.w_top), q)
    o = o.reshape(-1, BOX, BOX, 2)
    return net.s_out * (o[..., 0] + 1j * o[..., 1])


def exact_box(G_row_cols: np.ndarray, G_row_vals: np.ndarray, cu: int, cv: int, Ng: int):
    """Dense BOX x BOX box of one exact sparsified row, and the row energy outside the box."""
    cols = box_columns(cu, cv, Ng)
    pos = {int(c): i for i, c in enumerate(cols)}
    box = np.zeros(BOX * BOX, dtype=np.complex128)
    outside = 0.0
    for c, val in zip(G_row_cols, G_row_vals):
        i = pos.get(int(c))
        if i is None:
            outside += abs(val) ** 2
        else:
            box[i] = val
    return box.reshape(BOX, BOX), outside


def energy_error(t_box: np.ndarray, G_row_cols, G_row_vals, cu: int, cv: int, Ng: int) -> float:
    """||t - g||^2 / ||g||^2 for one row (g: exact sparsified row, entries outside the box count in full)."""
    gb, outside = exact_box(G_row_cols, G_row_vals, cu, cv, Ng)
    num = float(np.sum(np.abs(t_box - gb) ** 2)) + outside
    den = float(np.sum(np.abs(np.asarray(G_row_vals)) ** 2))
    return num / den


# ----------------------------------------------------------------------------- operator

def _cells(u, v, s):
    ut = np.asarray(u, dtype=np.float64) / geo.cell_size(s.N, s.L, s.sigma)
    vt = np.asarray(v, dtype=np.float64) / geo.cell_size(s.N, s.L, s.sigma)
    cu, du = nearest_cell(ut)
    cv, dv = nearest_cell(vt)
    return cu, du, cv, dv


def surrogate_rows(net: Net, u, v, w, s, q=_ident):
    """(box columns [n, BOX^2], taps [n, BOX^2]) of every visibility."""
    cu, du, cv, dv = _cells(u, v, s)
    t = taps(net, w, du, dv, q).reshape(len(cu), -1)
    cols = np.stack([box_columns(int(a), int(b), s.Ng) for a, b in zip(cu, cv)])
    return cols, t


def phi_rows(cols, t, x, s, exact_rows=None, use_exact=None) -> np.ndarray:
    """y = G_s F Z A x for rows given as box columns and taps [n, BOX^2].

    exact_rows: scipy CSR with one row per visibility (caller order), used only
    where use_exact is true.
    """
    from .wproj import grid_forward
    X = grid_forward(x, s).ravel()
    y = np.einsum("kp,kp->k", t, X[cols])
    if use_exact is not None and np.any(use_exact):
        idx = np.nonzero(use_exact)[0]
        y[idx] = exact_rows[idx] @ X
    return y


def phi_rows_adjoint(cols, t, y, s, exact_rows=None, use_exact=None) -> np.ndarray:
    """x = A Z^H F^H G_s^H y for rows given as box columns and taps."""
    from .wproj import grid_adjoint
    y = np.asarray(y, dtype=np.complex128)
    keep = np.ones(len(y), dtype=bool)
    if use_exact is not None:
        keep &= ~np.asarray(use_exact, dtype=bool)
    Xp = np.zeros(s.Ng * s.Ng, dtype=np.complex128)
    np.add.at(Xp, cols[keep].ravel(), (np.conj(t[keep]) * y[keep, None]).ravel())
    if use_exact is not None and np.any(use_exact):
        idx = np.nonzero(use_exact)[0]
        Xp += exact_rows[idx].conj().T @ y[idx]
    return grid_adjoint(Xp.reshape(s.Ng, s.Ng), s)


def phi_s(net: Net, u, v, w, x, s, exact_rows=None, use_exact=None, q=_ident) -> np.ndarray:
    """Surrogate Phi: network taps, exact rows where use_exact[k]."""
    cols, t = surrogate_rows(net, u, v, w, s, q)
    return phi_rows(cols, t, x, s, exact_rows, use_exact)


def phi_s_adjoint(net: Net, u, v, w, y, s, exact_rows=None, use_exact=None, q=_ident) -> np.ndarray:
    """Surrogate Phi^H: network taps, exact rows where use_exact[k]."""
    cols, t = surrogate_rows(net, u, v, w, s, q)
    return phi_rows_adjoint(cols, t, y, s, exact_rows, use_exact)


def exact_rows_in_box(G, u, v, s):
    """(box columns, taps, energy outside the box) of exact sparsified rows G (caller order)."""
    cu, _, cv, _ = _cells(u, v, s)
    cols = np.stack([box_columns(int(a), int(b), s.Ng) for a, b in zip(cu, cv)])
    t = np.empty((len(cu), BOX * BOX), dtype=np.complex128)
    lost = np.empty(len(cu))
    for k in range(len(cu)):
        a, b = G.indptr[k], G.indptr[k + 1]
        bx, lost[k] = exact_box(G.indices[a:b], G.data[a:b], int(cu[k]), int(cv[k]), s.Ng)
        t[k] = bx.ravel()
    return cols, t, lost


def row_errors(net: Net, u, v, w, G, s, q=_ident) -> np.ndarray:
    """eps_k of every visibility against the exact sparsified rows G (caller order)."""
    cu, du, cv, dv = _cells(u, v, s)
    t = taps(net, w, du, dv, q)
    out = np.empty(len(cu))
    for k in range(len(cu)):
        a, b = G.indptr[k], G.indptr[k + 1]
        out[k] = energy_error(t[k], G.indices[a:b], G.data[a:b], int(cu[k]), int(cv[k]), s.Ng)
    return out


def from_packed(p, w_top: float = 1.0, s_out: float = 1.0, H: int = HIDDEN, n_out: int = N_OUT) -> Net:
    """Net from a flat parameter vector in the order W1 [H,3], b1, W2 [H,H], b2, W3, b3, W4 [n_out,H], b4."""
    p = np.asarray(p, dtype=np.float64)
    shapes = [(H, 3), (H,), (H, H), (H,), (H, H), (H,), (n_out, H), (n_out,)]
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(p[o:o + n].reshape(sh))
        o += n
    if o != p.size:
        raise ValueError(f"expected {o} parameters, got {p.size}")
    return Net(*out, s_out=s_out, w_top=w_top)


def to_packed(net: Net) -> np.ndarray:
    return np.concatenate([getattr(net, k).ravel() for k in net.NAMES])


# ----------------------------------------------------------------------------- run-time check

def lattice_coords(nw: int, nd: int, w_top: float, s):
    """(u, v, w) of the check lattice's nodes, node i = (iw nd + iv) nd + iu: w = w_top iw / (nw - 1),
    offsets -1/2 + j / (nd - 1) cells from the centre cell, the last one 2^-20 cells below +1/2 (so
    that it keeps the centre cell as its nearest)."""
    cell = geo.cell_size(s.N, s.L, s.sigma)
    off = -0.5 + np.arange(nd) / (nd - 1.0)
    off[-1] = 0.5 - 2.0 ** -20
    iw, iv, iu = np.meshgrid(np.arange(nw), np.arange(nd), np.arange(nd), indexing="ij")
    return off[iu.ravel()] * cell, off[iv.ravel()] * cell, w_top * iw.ravel() / (nw - 1.0)


def check_table(net: Net, E: float, nw: int, nd: int, s, q=_ident):
    """(node errors, node kept energies) of the check lattice: the network's row error against the
    exact sparsified row of every node (Section 3.2's energy rule), and that row's kept energy."""
    from .wproj import build_rows
    u, v, w = lattice_coords(nw, nd, net.w_top, s)
    G = build_rows(u, v, w, E, s)
    eps = row_errors(net, u, v, w, G, s, q)
    K = np.asarray(G.multiply(G.conj()).sum(axis=1)).ravel().real
    return eps, K


def check_estimate(net: Net, u, v, w, table_eps, table_K, nw: int, nd: int, s, q=_ident) -> np.ndarray:
    """Run-time estimate of each network row's error from the lattice alone (no exact row):
    max(largest node error of the lattice cell holding (w, du, dv),
        (| ||t|| - sqrt(K) | / sqrt(K))^2), K = trilinear interpolation of the nodes' kept energies
    (the second term is the reverse triangle inequality's lower bound on ||t - g||^2 / ||g||^2 when
    K = ||g||^2); +inf outside the lattice."""
    cu, du, cv, dv = _cells(u, v, s)
    t = taps(net, w, du, dv, q).reshape(len(cu), -1)
    tn = np.sqrt(np.sum(np.abs(t) ** 2, axis=1))
    f = features(w, du, dv, net.w_top)
    wf = 0.5 * (f[:, 0] + 1.0) * (nw - 1)
    uf = (0.5 * f[:, 1] + 0.5) * (nd - 1)
    vf = (0.5 * f[:, 2] + 0.5) * (nd - 1)
    out = np.full(len(cu), np.inf)
    e_node = np.asarray(table_eps).reshape(nw, nd, nd)
    K_node = np.asarray(table_K).reshape(nw, nd, nd)
    for k in range(len(cu)):
        if not (0 <= wf[k] <= nw - 1 and 0 <= uf[k] <= nd - 1 and 0 <= vf[k] <= nd - 1):
            continue
        iw, iu, iv = min(int(wf[k]), nw - 2), min(int(uf[k]), nd - 2), min(int(vf[k]), nd - 2)
        tw, tu, tv = wf[k] - iw, uf[k] - iu, vf[k] - iv
        corner = e_node[iw:iw + 2, iv:iv + 2, iu:iu + 2]
        wgt = np.einsum("a,b,c->abc", [1 - tw, tw], [1 - tv, tv], [1 - tu, tu])
        K = float(np.sum(wgt * K_node[iw:iw + 2, iv:iv + 2, iu:iu + 2]))
        lb = (tn[k] - np.sqrt(K)) ** 2 / K if K > 0 else np.inf
        out[k] = max(float(corner.max()), lb)
    return out
