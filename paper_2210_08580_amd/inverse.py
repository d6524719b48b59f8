"""Far-field objective as a differentiable PyTorch function (inverse-problem use case).

The forward value and both gradients come from one library call,
fds_farfield_objective_grad (forward solve, adjoint solve and the derivative pass,
all on the device); this module only wires them into torch.autograd so that node
positions produced by a differentiable torch parametrisation (for example the
curve Fourier coefficients below) receive gradients by the chain rule.
"""
from __future__ import annotations

import math

import torch

from . import binding as B


class FarFieldObjective(torch.autograd.Function):
    """J(nodes, amps) = sum_r sum_l |u_inf,r(theta_l) - T_lr|^2 for the TE-EFIE model.

    nodes: (n, 2) float64, amps: (nrhs,) complex128 (both CUDA). The gradient
    returned for amps follows PyTorch's convention dJ/dRe + i dJ/dIm."""

    @staticmethod
    def forward(ctx, nodes, amps, fctx, k, angles, thetas, target, n_modes, max_iters, tol):
        op = B.fds_assemble(fctx, nodes.detach(), k)
        try:
            ne = B.fds_filter(op, "efie", 1.0, n_modes)
            B.fds_compress(op, rank_cap=ne, oversample=8, power_iters=2, seed=1)
            B.fds_factor(op)
            J, gn, ga, ff, st = B.fds_farfield_objective_grad(op, angles, amps.detach(), thetas, target,
                                                             max_iters=max_iters, tol=tol)
        finally:
            op.close()
        if not st["converged"]:
            raise RuntimeError(f"forward refinement did not converge: {st}")
        ctx.save_for_backward(gn, ga)
        ctx.farfield = ff
        return torch.tensor(J, dtype=torch.float64, device=nodes.device)

    @staticmethod
    def backward(ctx, gout):
        gn, ga = ctx.saved_tensors
        return gout * gn, gout * ga, None, None, None, None, None, None, None, None


def farfield_objective(nodes, amps, fctx, k, angles, thetas, target, n_modes=63, max_iters=8, tol=1e-12):
    return FarFieldObjective.apply(nodes, amps, fctx, k, angles, thetas, target, n_modes, max_iters, tol)


def star_nodes(coeffs: torch.Tensor, n: int, amp: float = 0.3, lobes: int = 5) -> torch.Tensor:
    """Nodes at t_i = 2 pi i/n of r(t) = 1 + amp cos(lobes t) + sum_m a_m cos mt + b_m sin mt,
    coeffs: (M, 2) rows (a_m, b_m); differentiable in coeffs."""
    t = 2.0 * math.pi * torch.arange(n, dtype=torch.float64, device=coeffs.device) / n
    m = torch.arange(1, coeffs.shape[0] + 1, dtype=torch.float64, device=coeffs.device)
    r = 1.0 + amp * torch.cos(lobes * t) + (coeffs[:, 0:1] * torch.cos(m[:, None] * t)).sum(0) \
        + (coeffs[:, 1:2] * torch.sin(m[:, None] * t)).sum(0)
    return torch.stack([r * torch.cos(t), r * torch.sin(t)], dim=1)
