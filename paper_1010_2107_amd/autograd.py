"""dI/dtheta through torch.autograd: the forward pass is one VEGAS iteration
(vmc_iterate) on a frozen grid, the backward pass regenerates the same
samples from the counter-based stream and runs the adjoint kernel
(vmc_iterate_adjoint), returning grad_output * (1/N) sum_s J_s df/dtheta(x_s).

Nothing is stored between the passes except (grid, seed, iteration): the
Philox counters make every sample recomputable.  With `fused=True` the
forward pass runs the combined forward+adjoint kernel once and the backward
pass only scales the stored gradient.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .grid import Grid


class VegasIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, grid: Grid, integrand: int, ncall: int, seed: int, it: int,
                fused: bool = False):
        th = theta.detach().to(device=grid.device, dtype=torch.float64).contiguous()
        ngrad = th.numel() if integrand != L.WJETS else 3
        if fused and ctx.needs_input_grad[0]:
            grid.fused(integrand, th, ncall, seed, it)
            g = grid.scal[L.S_GRAD:L.S_GRAD + 5 * ngrad].view(ngrad, 5)[:, 3].clone()
        else:
            grid.iterate(integrand, th, ncall, seed, it)
            g = None
        I = grid.scal[L.S_I].clone()
        ctx.grid, ctx.integrand, ctx.ncall, ctx.seed, ctx.it, ctx.ngrad = grid, integrand, ncall, seed, it, ngrad
        ctx.theta_shape, ctx.theta_dtype = theta.shape, theta.dtype
        ctx.save_for_backward(th)
        ctx.fused_grad = g
        return I.to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (th,) = ctx.saved_tensors
        g = ctx.fused_grad
        if g is None:
            grid = ctx.grid
            grid.adjoint(ctx.integrand, th, ctx.ncall, ctx.seed, ctx.it)
            g = grid.scal[L.S_GRAD:L.S_GRAD + 5 * ctx.ngrad].view(ctx.ngrad, 5)[:, 3].clone()
        full = torch.zeros(ctx.theta_shape, dtype=torch.float64, device=g.device).reshape(-1)
        full[: ctx.ngrad] = g
        grad_theta = (grad_out.to(torch.float64) * full).reshape(ctx.theta_shape).to(ctx.theta_dtype)
        return grad_theta, None, None, None, None, None, None


def vegas_integral(theta, grid, integrand, ncall, seed, it, fused=False):
    """Differentiable single-iteration estimate I(theta) on the grid's current
    (frozen) bins; call grid.refine() yourself between iterations."""
    return VegasIntegral.apply(theta, grid, integrand, ncall, seed, it, fused)
