"""Importance-sampling weights of the MC-MP2 estimator (Sec. III).

Test infrastructure: part of the FP64 oracle.

* Eq. basisSet: g(r) = sum_I [c1 N(z1) exp(-z1 |r-R_I|^2) + c2 N(z2) exp(-z2 |r-R_I|^2)],
  N(z) the normalisation of a primitive s Gaussian, read as the unit-L2
  constant (2 z / pi)^(3/4) (the paper does not print it).
* Electron-pair weight: w(r1, r2) = g(r1) g(r2) / (N_g r12).
* N_g = double integral of g(r1) g(r2) / r12, evaluated analytically: every
  term is a two-centre Coulomb integral of s Gaussians,
  int int exp(-a |r1-A|^2) exp(-b |r2-B|^2) / r12 = 2 pi^(5/2) / (a b sqrt(a+b)) F0(a b/(a+b) |A-B|^2),
  with F0(T) = (1/2) sqrt(pi/T) erf(sqrt(T)), F0(0) = 1.
* Eq. tauWeight: w(tau) = lambda exp(-lambda tau), lambda = 2 (eps_LUMO - eps_HOMO).
"""
from __future__ import annotations

import math

import numpy as np


def s_norm(zeta):
    """Unit-L2 normalisation of exp(-zeta r^2)."""
    return (2.0 * np.asarray(zeta, dtype=float) / math.pi) ** 0.75


def g_values(points: np.ndarray, nuc_xyz: np.ndarray, wfn: np.ndarray) -> np.ndarray:
    """Eq. basisSet at points [..., 3] -> [...]."""
    pts = np.asarray(points, dtype=float)
    out = np.zeros(pts.shape[:-1])
    for I in range(nuc_xyz.shape[0]):
        c1, z1, c2, z2 = wfn[I]
        d = pts - nuc_xyz[I]
        r2 = np.sum(d * d, axis=-1)
        out = out + c1 * s_norm(z1) * np.exp(-z1 * r2) + c2 * s_norm(z2) * np.exp(-z2 * r2)
    return out


def boys_f0(T: float) -> float:
    """F0(T) = int_0^1 exp(-T t^2) dt."""
    if T < 1e-14:
        return 1.0 - T / 3.0
    return 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))


def coulomb_ss(a: float, b: float, RAB2: float) -> float:
    """int int exp(-a|r1-A|^2) exp(-b|r2-B|^2)/r12 for |A-B|^2 = RAB2."""
    return 2.0 * math.pi ** 2.5 / (a * b * math.sqrt(a + b)) * boys_f0(a * b / (a + b) * RAB2)


def n_g(nuc_xyz: np.ndarray, wfn: np.ndarray) -> float:
    """Normalisation N_g of the electron-pair weight (Sec. III)."""
    terms = []
    for I in range(nuc_xyz.shape[0]):
        for (cI, zI) in ((wfn[I, 0], wfn[I, 1]), (wfn[I, 2], wfn[I, 3])):
            terms.append((nuc_xyz[I], cI * s_norm(zI), zI))
    total = 0.0
    for A, ca, za in terms:
        for B, cb, zb in terms:
            R2 = float(np.sum((A - B) ** 2))
            total += ca * cb * coulomb_ss(za, zb, R2)
    return total


def pair_weight(r1: np.ndarray, r2: np.ndarray, nuc_xyz, wfn, Ng: float) -> np.ndarray:
    """w(r1, r2) = g(r1) g(r2) / (N_g r12) for arrays of points [..., 3]."""
    r12 = np.sqrt(np.sum((np.asarray(r1) - np.asarray(r2)) ** 2, axis=-1))
    return g_values(r1, nuc_xyz, wfn) * g_values(r2, nuc_xyz, wfn) / (Ng * r12)


def tau_lambda(eps: np.ndarray, n_occ: int) -> float:
    """lambda = 2 (eps_LUMO - eps_HOMO)."""
    eps = np.asarray(eps, dtype=float)
    return 2.0 * (float(eps[n_occ:].min()) - float(eps[:n_occ].max()))


def tau_weight(tau, lam: float):
    """Eq. tauWeight."""
    return lam * np.exp(-lam * np.asarray(tau, dtype=float))
