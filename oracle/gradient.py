"""Gradients of the per-step estimate with respect to spinor energies and
coefficients, by reverse-mode differentiation of the oracle's own forward.

Test infrastructure: part of the FP64 oracle.

The quantity differentiated is the per-step value of Eq. redundant averaged
over the step's tau samples, at fixed walkers, fixed tau and fixed lambda
(lambda is a sampling parameter; the estimator is unbiased for any fixed
lambda, so holding it fixed gives an unbiased gradient of E2).

Complex convention: dE/dC = dE/dRe C + i dE/dIm C.
"""
from __future__ import annotations

import numpy as np
import torch

from .integrand import step_estimate


def step_value_and_grad(inp, walkers, taus, lam: float, Ng: float, interaction: str = "coulomb"):
    """Returns (parts[n_tau, 3] ndarray, value float, grad_eps [n_sp], grad_C [2, n_b, n_sp] complex).
    interaction: "coulomb" (the paper's), "gaunt" or "breit" (the interaction of Sec. II)."""
    C = torch.tensor(inp.coeffs, dtype=torch.complex128, requires_grad=True)
    e = torch.tensor(inp.eps, dtype=torch.float64, requires_grad=True)
    parts = step_estimate(inp, walkers, taus, lam, Ng, coeffs=C, eps=e, interaction=interaction)
    value = parts[:, 2].mean()
    value.backward()
    return (parts.detach().numpy(), float(value.detach()), e.grad.numpy().copy(),
            C.grad.numpy().copy())


def step_value(inp, walkers, taus, lam: float, Ng: float, coeffs=None, eps=None, interaction: str = "coulomb") -> float:
    """Per-step value (mean over tau of the total) for given C and eps arrays."""
    C = torch.as_tensor(inp.coeffs if coeffs is None else np.asarray(coeffs))
    e = torch.as_tensor(inp.eps if eps is None else np.asarray(eps))
    with torch.no_grad():
        return float(step_estimate(inp, walkers, taus, lam, Ng, coeffs=C, eps=e, interaction=interaction)[:, 2].mean())
