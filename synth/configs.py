"""Workload recipes (sizes, distributions, seeds) for the five benchmark forms.

Every number here is either a size stated by the workload description or a
geometric constant of the paper's set-up (Section 4.1).  The upper end of the
w distribution is stated through the chirp's bandwidth on the padded grid:

* the linear chirp exp(i pi w (l^2 + m^2)) has instantaneous frequency w*l;
  sampled on the padded grid (l in [-L, L), cell 1/(2L) in u) it spans
  4 w L^2 grid cells, and the Kaiser-Bessel window adds W cells, so a kernel
  support of S cells corresponds to w = (S - W) / (4 L^2);
* the tiny form instead states that the chirp's bandwidth over the field of
  view (2 w L^2 cells) is half of the padded grid (N cells), i.e.
  w = N / (2 L^2) -- the paper's maximal modulation w_d = 1 of Section 4.1
  expressed on this grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

THETA_DEG = 2.0          # opening angle of the field of view (Section 4.1)
BASE_SEED = 20130712     # seeds are BASE_SEED + form index


def fov_L(theta_deg: float = THETA_DEG) -> float:
    """Planar field of view L = 2 sin(theta / 2) (Section 4.1)."""
    return 2.0 * math.sin(math.radians(theta_deg) / 2.0)


def band_limit(N: int, L: float) -> float:
    """Band limit B = N / (2 L) of an N-pixel image over a field L (Section 4.1)."""
    return N / (2.0 * L)


def w_for_support(S: float, W: int, L: float) -> float:
    """w at which the padded-grid chirp plus the KB window spans S cells."""
    return (S - W) / (4.0 * L * L)


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    N: int
    M: int
    uv: str                  # "uniform" in [-B, B)^2, or "gaussian" (isotropic, truncated to the band)
    uv_sigma: float          # Gaussian sigma as a fraction of B (ignored for "uniform")
    w_top: float             # w ~ U[0, w_top] (wavelengths)
    E: float = 0.99          # preserved energy fraction (Section 3.2)
    W: int = 4               # Kaiser-Bessel support in grid cells
    sigma: float = 2.0       # grid oversampling
    n_blobs: int = 10
    n_points: int = 20
    iters: int = 0           # solver iterations of the form (0: none)
    snr_in_db: float = 30.0  # input SNR (Section 4.1)
    theta_deg: float = THETA_DEG
    taps: str = "c64"        # "c64" or "bf16"
    channels: Optional[Tuple[int, ...]] = None  # batched form: per-channel visibility counts
    w_scale: Optional[Tuple[float, ...]] = None  # batched form: per-channel w_top multipliers
    train_samples: int = 0   # surrogate form: exact rows the network is trained on

    @property
    def L(self) -> float:
        return fov_L(self.theta_deg)

    @property
    def Ng(self) -> int:
        return int(round(self.sigma * self.N))

    @property
    def B(self) -> float:
        return band_limit(self.N, self.L)

    @property
    def seed(self) -> int:
        return BASE_SEED + self.index

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


def _batched_counts(n_channels: int = 48, lo: float = 5e4, hi: float = 2e6):
    import numpy as np
    rng = np.random.default_rng([BASE_SEED + 3, 99])
    m = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_channels))
    return tuple(int(round(x)) for x in m)


def _make():
    L = fov_L()
    cfg = {}
    cfg[0] = Workload(name="tiny-64-fp64", index=0, N=64, M=820, uv="uniform", uv_sigma=0.0,
                      w_top=64 / (2.0 * L * L), n_blobs=10, n_points=20, iters=200)
    cfg[1] = Workload(name="plain-256-fp32", index=1, N=256, M=32768, uv="gaussian", uv_sigma=0.25,
                      w_top=w_for_support(32, 4, L), n_blobs=33, n_points=67, iters=500)
    cfg[2] = Workload(name="precision-1024", index=2, N=1024, M=4194304, uv="gaussian", uv_sigma=0.25,
                      w_top=w_for_support(64, 4, L), n_blobs=33, n_points=67, taps="bf16")
    counts = _batched_counts()
    cfg[3] = Workload(name="batched-48x512", index=3, N=512, M=sum(counts), uv="gaussian", uv_sigma=0.25,
                      w_top=w_for_support(32, 4, L) / 2.0, n_blobs=33, n_points=67,
                      channels=counts, w_scale=tuple(1.0 + c / 47.0 for c in range(48)))
    cfg[4] = Workload(name="surrogate-2048", index=4, N=2048, M=16777216, uv="gaussian", uv_sigma=0.25,
                      w_top=w_for_support(32, 4, L), n_blobs=33, n_points=67, iters=200,
                      train_samples=2_000_000)
    return cfg


CONFIGS = _make()


def workload(i: int) -> Workload:
    return CONFIGS[i]
