"""Quality metrics of Section 4.1.

Test infrastructure (see the package header).

* SNR_out = 20 log10(sigma(x) / sigma(x - x_rec)), sigma = standard deviation.
* Input noise: the paper sets sigma(n) = 10^(-SNR_in/20) sigma(x).  Because
  that presumes a unit-scale operator, the noise here is set in the
  visibility domain, sigma_n = 10^(-SNR_in/20) rms(Phi x), with the l2-ball
  radius eps^2 = sigma_n^2 (M + 2 sqrt(M)) (mean plus two standard deviations
  of ||n||^2 for complex Gaussian noise).  Parity unpinned against the
  paper's printed SNRs, which need its test images.
"""
from __future__ import annotations

import numpy as np


def snr_out(x: np.ndarray, x_rec: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    return float(20.0 * np.log10(np.std(x) / np.std(x - np.asarray(x_rec, dtype=np.float64))))


def noise_sigma(y_clean: np.ndarray, snr_in_db: float = 30.0) -> float:
    rms = np.sqrt(np.mean(np.abs(y_clean) ** 2))
    return float(10.0 ** (-snr_in_db / 20.0) * rms)


def l2_ball_radius(sigma_n: float, M: int) -> float:
    return float(np.sqrt(sigma_n ** 2 * (M + 2.0 * np.sqrt(M))))
