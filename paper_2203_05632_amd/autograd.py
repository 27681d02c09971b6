"""torch.autograd.Function over the HIP step: the value of one MC step and
its gradients with respect to spinor coefficients and energies, from the
library's hand-written adjoint (no autograd graph through the kernels).

The value is V = (1/n_tau) sum_t I'_t (Eq. redundant, direct + exchange),
at fixed walkers and tau samples and with lambda frozen when the context was
created.  The backward pass runs the step again with the adjoint enabled, so
spinor values and Green's functions are recomputed rather than stored.
"""
from __future__ import annotations

import torch

from .context import Context


class MCMP2Step(torch.autograd.Function):
    @staticmethod
    def forward(fctx, coeffs: torch.Tensor, eps: torch.Tensor, walkers: torch.Tensor, tau: torch.Tensor,
                context: Context) -> torch.Tensor:
        context.set_coefficients(coeffs.detach().contiguous(), eps.detach().contiguous())
        e2 = torch.empty((tau.shape[0], 3), dtype=torch.float64, device=walkers.device)
        context.step(walkers, tau, e2)
        fctx.save_for_backward(coeffs, eps, walkers, tau)
        fctx.context = context
        return e2[:, 2].mean()

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        coeffs, eps, walkers, tau = fctx.saved_tensors
        context: Context = fctx.context
        context.set_coefficients(coeffs.detach().contiguous(), eps.detach().contiguous())
        e2 = torch.empty((tau.shape[0], 3), dtype=torch.float64, device=walkers.device)
        g_eps = torch.empty_like(eps, dtype=torch.float64)
        g_c = torch.empty(coeffs.shape, dtype=torch.complex128, device=coeffs.device)
        context.step(walkers, tau, e2, grad_eps=g_eps, grad_coeffs=g_c)
        g = grad_out.to(torch.float64)
        return (g_c * g if fctx.needs_input_grad[0] else None,
                g_eps * g if fctx.needs_input_grad[1] else None, None, None, None)


def mcmp2_value(coeffs: torch.Tensor, eps: torch.Tensor, walkers: torch.Tensor, tau: torch.Tensor,
                context: Context) -> torch.Tensor:
    """Differentiable per-step value (0-d float64 tensor)."""
    return MCMP2Step.apply(coeffs, eps, walkers, tau, context)
