"""Shared helpers of the GPU parity tests: oracle rows built in a process pool, and the rounding
model that bounds the error of bfloat16 taps."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np
import scipy.sparse as sp

from oracle import wproj

# bfloat16 keeps 8 significant bits: round-to-nearest-even leaves a relative error of at most
# u = 2^-8 in each of a tap's two components (half a unit in the last place of 2^-7).
BF16_U = 2.0 ** -8


def pool_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_rows(u, v, w, E, s, rows, workers=None):
    """The oracle's sparsified rows of the visibilities `rows` (in that order), built in a pool of
    processes; scipy CSR with one row per selected visibility."""
    workers = workers or pool_workers()
    rows = np.asarray(rows)
    chunks = [c for c in np.array_split(rows, workers * 4) if c.size]
    if len(chunks) <= 1 or workers == 1:
        return wproj.build_rows(u, v, w, E, s, rows=rows)
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(wproj.build_rows_csr_parts, [(u[c], v[c], w[c], E, s, None) for c in chunks])
    return sp.vstack([sp.csr_matrix((d, i, p), shape=(n, s.Ng * s.Ng)) for p, i, d, n in parts]).tocsr()


def relerr(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def bf16_rms_bound(G, vec, adjoint: bool, ref) -> float:
    """Expected relative error of the product G vec (adjoint: G^H vec) when every tap of G is rounded
    to bfloat16 pairs, under the rounding model: each component's error is uniform within half a unit
    in the last place (at most u |component|, variance at most u^2 component^2 / 3) and independent
    across taps.  Then E ||delta||^2 <= (u^2 / 3) sum_k sum_j |G_kj|^2 |vec_j|^2 (summed over the
    product's outputs), and the bound is the square root of that over ||ref|| (the exact product)."""
    A2 = abs(G).power(2) if sp.issparse(G) else np.abs(G) ** 2
    p2 = np.abs(np.asarray(vec)) ** 2
    tot = float((A2.T @ p2).sum()) if adjoint else float((A2 @ p2).sum())
    return BF16_U / np.sqrt(3.0) * np.sqrt(tot) / float(np.linalg.norm(ref))


def oracle_row_window(args):
    """One oracle row (the literal construction: the whole Ng x Ng row) around its visibility's cell:
    (first v cell, first u cell, energies and values on a (2 half) x (2 half) window of cells,
    tau, number of kept cells outside the window).  Worker form for process pools."""
    ut, vt, w, E, s, half = args
    g = wproj.kernel_row(ut, vt, w, s)
    m = (g * g.conj()).real
    tau, _ = wproj.energy_threshold(m, E)
    Ng = s.Ng
    cv = int(np.floor(vt + 0.5)) + Ng // 2 - half
    cu = int(np.floor(ut + 0.5)) + Ng // 2 - half
    rv = (cv + np.arange(2 * half)) % Ng
    ru = (cu + np.arange(2 * half)) % Ng
    mw = m[np.ix_(rv, ru)]
    gw = g[np.ix_(rv, ru)]
    outside = int((m >= tau).sum() - (mw >= tau).sum())
    return cv, cu, mw, gw, tau, outside
