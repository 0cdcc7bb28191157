"""Pins of the paper-form operator C-hat (Eq. 8) against the numbers Section 3.2 prints (CPU only)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import paper_form

L = synth.fov_L()
GOLD = os.path.join(os.path.dirname(__file__), "golden", "nnz_fraction_section3_2.json")


def test_full_rows_have_unit_energy():
    for wd in (0.0, 0.3, 1.0):
        g = paper_form.chirp_row(wd, 32, L)
        assert abs(np.sum(np.abs(g) ** 2) - 1.0) < 1e-12


def test_constant_w_chat_is_unitary():
    """All (2N)^2 shifted rows at one w form a unitary matrix (norm-preserving convolution, Section 2.3)."""
    N = 6
    Ng = 2 * N
    C = np.stack([paper_form.shifted_row(0.7, a, b, N, L).ravel() for a in range(Ng) for b in range(Ng)])
    assert np.abs(C.conj().T @ C - np.eye(Ng * Ng)).max() < 1e-12


def test_nonzero_fraction_matches_printed_values():
    gold = json.load(open(GOLD))
    wd = (np.arange(100) + 0.5) / 100          # quantiles of U(0, 1): the expectation over w_d
    N = gold["setup"]["N"]
    for E, (lo, hi) in gold["accept"].items():
        frac = paper_form.nnz_fraction(wd, float(E), N, L)
        assert lo <= frac <= hi, (E, frac)


def test_w_zero_row_is_a_single_entry():
    g = paper_form.chirp_row(0.0, 16, L)
    m = np.abs(g) ** 2
    assert np.count_nonzero(m > 1e-20) == 1 and abs(m.max() - 1) < 1e-12
