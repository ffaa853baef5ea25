"""dI/dtheta through torch.autograd: the forward pass is one VEGAS iteration
(vmc_iterate) on a frozen grid, the backward pass regenerates the same
samples from the counter-based stream and runs the adjoint kernel
(vmc_iterate_adjoint), returning grad_output * (1/N) sum_s J_s df/dtheta(x_s).

The differentiable input holds exactly the parameters the adjoint pass
differentiates (the first ngrad of the integrand's parameter list, e.g.
(M, Gamma, g) of the W + partons toy); the rest of the list (collider
energy, cut values) is passed as `fixed` and is not part of the graph, so
no gradient is ever reported for a parameter the adjoint does not
differentiate.

By default (`fused=True`) a forward pass whose input requires a gradient
runs the combined forward+adjoint kernel once (a few per cent more than the
forward kernel alone) and the backward pass only scales the stored
gradient.  With `fused=False` the forward pass runs alone and the backward
pass runs the adjoint kernel; nothing is stored between the passes except
(grid, seed, iteration) and the grid-state version of the forward pass: the
Philox counters make every sample recomputable, and a backward pass after
the grid has moved (refine, set_edges, reset, stratify) raises VmcError
VMC_E_GRID instead of differentiating a different estimator.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .grid import Grid


class VegasIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, grid: Grid, integrand: int, ncall: int, seed: int, it: int,
                fused: bool = True, fixed: tuple = (), fp64: bool = False):
        ntheta, ngrad = L.integrand_info(integrand, grid.dim, fp64)
        if ngrad == 0:
            raise ValueError(f"integrand {integrand} has no differentiable parameters")
        if theta.numel() != ngrad or ngrad + len(fixed) != ntheta:
            raise ValueError(f"integrand {integrand} in dim {grid.dim}: theta takes the {ngrad} differentiable "
                             f"parameters and `fixed` the other {ntheta - ngrad}; got {theta.numel()} and "
                             f"{len(fixed)}")
        th = theta.detach().to(device=grid.device, dtype=torch.float64).reshape(-1)
        if fixed:
            th = torch.cat([th, torch.as_tensor(fixed, dtype=torch.float64, device=grid.device)])
        th = th.contiguous()
        if fused and ctx.needs_input_grad[0]:
            grid.fused(integrand, th, ncall, seed, it, fp64=fp64)
            g = grid.scal[L.S_GRAD:L.S_GRAD + 5 * ngrad].view(ngrad, 5)[:, 3].clone()
        else:
            grid.iterate(integrand, th, ncall, seed, it, fp64=fp64)
            g = None
        I = grid.scal[L.S_I].clone()
        ctx.grid, ctx.integrand, ctx.ncall, ctx.seed, ctx.it, ctx.ngrad = grid, integrand, ncall, seed, it, ngrad
        ctx.version, ctx.fp64 = grid.version(), fp64
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
            if grid.version() != ctx.version:
                raise L.VmcError(-8, "the grid moved (refine, set_edges, reset or stratify) between the forward "
                                     "pass and its backward pass")
            grid.adjoint(ctx.integrand, th, ctx.ncall, ctx.seed, ctx.it, fp64=ctx.fp64)
            g = grid.scal[L.S_GRAD:L.S_GRAD + 5 * ctx.ngrad].view(ctx.ngrad, 5)[:, 3].clone()
        grad_theta = (grad_out.to(torch.float64) * g).reshape(ctx.theta_shape).to(ctx.theta_dtype)
        return grad_theta, None, None, None, None, None, None, None, None


def vegas_integral(theta, grid, integrand, ncall, seed, it, fused=True, fixed=(), fp64=False):
    """Differentiable single-iteration estimate I(theta, fixed) on the grid's
    current (frozen) bins.  theta: the ngrad differentiable parameters;
    fixed: the remaining ones (a tuple of floats); fused: the gradient in the
    forward pass's kernel (default) or in a separate adjoint pass at
    backward(); fp64: the double-precision instantiation of the integrand.
    Call grid.refine() yourself between iterations, after backward()."""
    return VegasIntegral.apply(theta, grid, integrand, ncall, seed, it, fused, tuple(fixed), fp64)
