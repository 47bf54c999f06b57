"""Differentiable detector energy: a torch.autograd.Function over the library's
hand-written adjoint (lbem_adjoint_forward / lbem_adjoint_backward).

L(eps_r, sigma) = sum over the N collided states of sum_{x, y} |E(x, y, z_d)|^2
for an MM or HV lattice initialised to the equilibrium of (E0, B0).  The forward
pass stores a checkpoint every K steps and the E frames of the last `keep`
segments; backward recomputes the other segments and runs the adjoint steps in
reverse.  Gradients are FP64 on the device.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import lbem


@dataclass
class DetectorProblem:
    shape: tuple           # (nx, ny, nz)
    E0: torch.Tensor       # [3][N]
    B0: torch.Tensor       # [3][N]
    nsteps: int
    det_z: int
    K: int = 50
    mu_r: Optional[torch.Tensor] = None
    model: str = "mm"
    # trailing segments whose E frames the forward keeps; 0: as many as fit in
    # half of the device memory free at the call (all of them, when they fit,
    # so the backward recomputes nothing)
    keep: int = 0


class DetectorEnergy(torch.autograd.Function):
    """loss = DetectorEnergy.apply(eps_r, sigma, problem) with eps_r, sigma of shape [N]."""

    @staticmethod
    def forward(ctx, eps_r: torch.Tensor, sigma: torch.Tensor, prob: DetectorProblem):
        lat = lbem.Lattice(prob.model, prob.shape, eps_r.detach(), prob.mu_r, sigma.detach(), device=eps_r.device)
        lat.set_fields(prob.E0, prob.B0)
        keep = prob.keep
        if keep == 0:
            free, _ = torch.cuda.mem_get_info(eps_r.device)
            keep = lat.adjoint_keep(prob.nsteps, prob.K, free // 2)
        ws = lat.adjoint_workspace(prob.nsteps, prob.K, keep)
        loss = lat.adjoint_forward(prob.nsteps, prob.K, prob.det_z, ws, keep)
        ctx.lat, ctx.ws, ctx.prob = lat, ws, prob
        ctx.dtypes = (eps_r.dtype, sigma.dtype)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        scale = float(grad_out.detach().cpu())
        ge, gs = ctx.lat.adjoint_backward(ctx.ws, ctx.prob.E0, ctx.prob.B0, scale=scale)
        ctx.lat, ctx.ws = None, None
        return ge.to(ctx.dtypes[0]), gs.to(ctx.dtypes[1]), None


def detector_energy(eps_r: torch.Tensor, sigma: torch.Tensor, prob: DetectorProblem) -> torch.Tensor:
    return DetectorEnergy.apply(eps_r, sigma, prob)
