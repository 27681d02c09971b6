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
    """The library works on the context's stream, the caller on torch's
    current stream: the context's stream first waits for the current one (the
    inputs' producers), and the current stream waits for the context's
    before the outputs are used, so contexts on side streams are ordered too.
    Outputs are allocated on the current stream, which their writes are
    ordered before."""

    @staticmethod
    def forward(fctx, coeffs: torch.Tensor, eps: torch.Tensor, walkers: torch.Tensor, tau: torch.Tensor,
                context: Context) -> torch.Tensor:
        cur = torch.cuda.current_stream(walkers.device)
        value = torch.empty(1, dtype=torch.float64, device=walkers.device)
        e2 = torch.empty((tau.shape[0], 3), dtype=torch.float64, device=walkers.device)
        c_in, e_in = coeffs.detach().contiguous(), eps.detach().contiguous()
        context.stream.wait_stream(cur)
        context.set_coefficients(c_in, e_in)
        context.step(walkers, tau, e2, value=value)
        cur.wait_stream(context.stream)
        fctx.save_for_backward(coeffs, eps, walkers, tau)
        fctx.context = context
        return value[0]

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        coeffs, eps, walkers, tau = fctx.saved_tensors
        context: Context = fctx.context
        cur = torch.cuda.current_stream(walkers.device)
        e2 = torch.empty((tau.shape[0], 3), dtype=torch.float64, device=walkers.device)
        g_eps = torch.empty_like(eps, dtype=torch.float64)
        g_c = torch.empty(coeffs.shape, dtype=torch.complex128, device=coeffs.device)
        c_in, e_in = coeffs.detach().contiguous(), eps.detach().contiguous()
        context.stream.wait_stream(cur)
        context.set_coefficients(c_in, e_in)
        context.step(walkers, tau, e2, grad_eps=g_eps, grad_coeffs=g_c)
        cur.wait_stream(context.stream)
        g = grad_out.to(torch.float64)
        return (g_c * g if fctx.needs_input_grad[0] else None,
                g_eps * g if fctx.needs_input_grad[1] else None, None, None, None)


def mcmp2_value(coeffs: torch.Tensor, eps: torch.Tensor, walkers: torch.Tensor, tau: torch.Tensor,
                context: Context) -> torch.Tensor:
    """Differentiable per-step value (0-d float64 tensor)."""
    return MCMP2Step.apply(coeffs, eps, walkers, tau, context)
