"""Seeded synthetic inputs for the sparse w-projection operator.

This package holds only workload recipes and random draws: sky images,
baseline coordinates (u, v, w) and noise.  It contains none of the method's
arithmetic (no chirp, no kernel, no FFT, no sparsification), so both the
FP64 oracle and the HIP path may take their inputs from here.

The geometry constants follow the experimental set-up of the paper
(Section 4.1): opening angle theta = 2 degrees, planar field of view
L = 2 sin(theta/2), band limit B = N / (2L).
"""
from .configs import CONFIGS, Workload, fov_L, band_limit, workload
from .generators import (sky, uvw, noise, subset_rows, rng_for, workload_inputs, random_complex, mlp_init,
                         training_positions)

__all__ = ["CONFIGS", "Workload", "fov_L", "band_limit", "workload", "mlp_init", "training_positions",
           "sky", "uvw", "noise", "subset_rows", "rng_for", "workload_inputs", "random_complex"]
