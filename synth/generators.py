"""Seeded random draws: sky images, baselines (u, v, w) and visibility noise.

All draws use NumPy's PCG64 generator seeded with [form seed, stream id], so
the sky, the baselines and the noise of one form are independent streams and
each can be regenerated on its own.

* Sky: Gaussian blobs (sigma ~ U[1, 4] px, amplitude ~ LogNormal(0, 1)) plus
  point sources at uniform pixels (amplitude ~ LogNormal(0, 1)); non-negative.
  These stand in for the paper's M31 and 30 Doradus test images (Section 4.1),
  which are not available here.
* Baselines: (u, v) uniform in [-B, B)^2 or isotropic Gaussian with
  sigma = s*B truncated to the band (redrawn until |u|, |v| < B), and
  w ~ U[0, w_top], following the uniform random sampling of Section 4.1.
* Noise: i.i.d. complex Gaussian, sigma split equally between real and
  imaginary parts (Section 4.1).
"""
from __future__ import annotations

import numpy as np

_STREAM = {"sky": 1, "uvw": 2, "noise": 3, "x": 4, "y": 5, "subset": 6, "mlp": 7, "train": 8, "sweep": 9}


def rng_for(seed: int, stream: str, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(seed), _STREAM[stream], int(sub)])


def sky(N: int, n_blobs: int, n_points: int, rng: np.random.Generator) -> np.ndarray:
    """Non-negative N x N sky, float64, indexed [m, l] (row = v axis)."""
    img = np.zeros((N, N), dtype=np.float64)
    ii, jj = np.mgrid[0:N, 0:N].astype(np.float64)
    for _ in range(n_blobs):
        cy, cx = rng.uniform(0, N, size=2)
        s = rng.uniform(1.0, 4.0)
        a = rng.lognormal(0.0, 1.0)
        img += a * np.exp(-((ii - cy) ** 2 + (jj - cx) ** 2) / (2.0 * s * s))
    for _ in range(n_points):
        py, px = rng.integers(0, N, size=2)
        img[py, px] += rng.lognormal(0.0, 1.0)
    return img


def _truncated_gauss(rng, sigma, B, n):
    out = rng.normal(0.0, sigma, size=n)
    bad = np.abs(out) >= B
    while bad.any():
        out[bad] = rng.normal(0.0, sigma, size=int(bad.sum()))
        bad = np.abs(out) >= B
    return out


def uvw(N: int, M: int, L: float, dist: str, sigma_frac: float, w_top: float,
        rng: np.random.Generator):
    """Baseline coordinates in wavelengths, float64 arrays of length M."""
    B = N / (2.0 * L)
    if dist == "uniform":
        u = rng.uniform(-B, B, size=M)
        v = rng.uniform(-B, B, size=M)
    elif dist == "gaussian":
        u = _truncated_gauss(rng, sigma_frac * B, B, M)
        v = _truncated_gauss(rng, sigma_frac * B, B, M)
    else:
        raise ValueError(f"unknown uv distribution {dist!r}")
    w = rng.uniform(0.0, w_top, size=M)
    return u, v, w


def noise(M: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian noise with E|n|^2 = sigma^2."""
    return sigma * (rng.normal(size=M) + 1j * rng.normal(size=M)) / np.sqrt(2.0)


def subset_rows(M: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Sorted random subset of k distinct row indices out of M."""
    k = min(k, M)
    return np.sort(rng.choice(M, size=k, replace=False))


def workload_inputs(wl, with_sky: bool = True):
    """(sky, u, v, w) of a workload description (see configs.Workload)."""
    u, v, w = uvw(wl.N, wl.M, wl.L, wl.uv, wl.uv_sigma, wl.w_top, rng_for(wl.seed, "uvw"))
    x = sky(wl.N, wl.n_blobs, wl.n_points, rng_for(wl.seed, "sky")) if with_sky else None
    return x, u, v, w


def random_complex(shape, rng: np.random.Generator) -> np.ndarray:
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def mlp_init(seed: int, hidden: int = 256, n_out: int = 2048) -> np.ndarray:
    """Packed float32 initial parameters of the surrogate network, layers 3 -> hidden -> hidden ->
    hidden -> n_out: every weight and bias uniform in +-1/sqrt(fan_in), drawn layer by layer
    (W then b) in the order W1, b1, W2, b2, W3, b3, W4, b4 (row-major, W_l is [out, in])."""
    rng = np.random.default_rng(seed)
    parts = []
    for n, k in ((hidden, 3), (hidden, hidden), (hidden, hidden), (n_out, hidden)):
        a = 1.0 / np.sqrt(k)
        parts.append(rng.uniform(-a, a, n * k))
        parts.append(rng.uniform(-a, a, n))
    return np.concatenate(parts).astype(np.float32)


def training_positions(wl, n: int, rng: np.random.Generator):
    """(u, v, w) of n training visibilities: w ~ U[0, w_top), offsets du, dv ~ U[-1/2, 1/2) cells
    from the grid's centre cell (u = du / (2L) wavelengths)."""
    cell = 1.0 / (2.0 * wl.L)
    w = rng.uniform(0.0, wl.w_top, n)
    du = rng.uniform(-0.5, 0.5, n)
    dv = rng.uniform(-0.5, 0.5, n)
    return du * cell, dv * cell, w
