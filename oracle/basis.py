"""Basis-function values (Sec. II, Eq. (C) and the text after it).

Test infrastructure: part of the FP64 oracle.

A component basis function is a Cartesian primitive Gaussian
chi_mu(r) = N_mu (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-zeta_mu |r-A|^2)
(the paper allows any basis function; the inputs carry N_mu).
"""
from __future__ import annotations

import numpy as np


def basis_values(points: np.ndarray, prim_xyz: np.ndarray, prim_exp: np.ndarray,
                 prim_lxyz: np.ndarray, prim_norm: np.ndarray) -> np.ndarray:
    """chi_mu(r) for points [P, 3] -> [P, n_b] (float64)."""
    pts = np.asarray(points, dtype=float)
    d = pts[:, None, :] - prim_xyz[None, :, :]          # [P, n_b, 3]
    r2 = np.sum(d * d, axis=-1)
    poly = np.ones(r2.shape)
    for ax in range(3):
        poly = poly * d[..., ax] ** prim_lxyz[None, :, ax]
    return prim_norm[None, :] * poly * np.exp(-prim_exp[None, :] * r2)
