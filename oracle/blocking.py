"""Blocking estimate of the statistical uncertainty (Sec. III, Eq. uncertainty).

Test infrastructure: part of the FP64 oracle.

The N post-burn-in per-step values I'_n are cut into N/N_b blocks of N_b
consecutive steps; sigma_N^2 is the mean squared deviation of the block means
from I_N (divided by the number of blocks, as printed), and the uncertainty
of I_N is sigma_N / sqrt(N / N_b).  An incomplete last block is dropped.
"""
from __future__ import annotations

import numpy as np


def blocking(values, n_b: int = 100):
    """Return (I_N, sigma_bar_N) of a 1-D series of per-step estimates."""
    v = np.asarray(values, dtype=float)
    n_blocks = v.shape[0] // n_b
    if n_blocks < 2:
        raise ValueError("need at least two complete blocks")
    v = v[: n_blocks * n_b]
    I_N = float(v.mean())
    block_means = v.reshape(n_blocks, n_b).mean(axis=1)
    sigma2 = float(np.mean((block_means - I_N) ** 2))
    return I_N, float(np.sqrt(sigma2) / np.sqrt(n_blocks))
