"""Differentiable Helmholtz solve behind torch.autograd.

For a(u, v) = sum_e [kappa grad u . grad v + lambda_e u v] (the bilinear form
of Eq. (1) of arXiv 1906.03489 for the Helmholtz problem), u = A(kappa,
lambda)^{-1} b with b fixed, and a scalar loss L(u):
    dL/dtheta = -z^T (dA/dtheta) u,   A z = dL/du   (A symmetric).
The forward pass keeps only kappa and lambda (and the assembled operator);
the backward pass recomputes u with a second solve, solves the adjoint
system with the same CG, and evaluates -z^T (dA/dtheta) u element by element
in the library's gradient kernel (per quadrature point for kappa, per element
for lambda).  Everything numeric runs in libnk.so.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import nk


@dataclass
class HelmholtzProblem:
    """Mesh and right-hand side of a Dirichlet Helmholtz solve whose
    coefficients kappa (per point, [E, Q^d]) and lambda (per element, [E])
    are the differentiable inputs."""
    dim: int
    P: int
    Q: int
    jac: torch.Tensor           # device [E, d, d, Q^d] FP64
    l2g: torch.Tensor           # device [E, n^d] int32
    nglobal: int
    dirichlet: torch.Tensor     # device [nglobal] uint8
    b: torch.Tensor             # device [nglobal] FP64
    rtol: float = 1e-12
    maxit: int = 100000
    mode: int = nk.SOLVE_F64

    def build(self, kappa: torch.Tensor, lam: torch.Tensor):
        space = nk.Space.create(self.dim, self.P, self.Q, self.jac,
                                kappa=kappa.detach().contiguous().reshape(-1))
        sysm = nk.System.create(space, self.nglobal, self.l2g, self.dirichlet,
                                lam=lam.detach().contiguous().reshape(-1))
        return space, sysm


class HelmholtzSolve(torch.autograd.Function):
    """u = A(kappa, lambda)^{-1} b with adjoint gradients for kappa and lambda."""

    @staticmethod
    def forward(ctx, kappa, lam, problem: HelmholtzProblem):
        space, sysm = problem.build(kappa, lam)
        u, _ = sysm.solve(problem.b, rtol=problem.rtol, maxit=problem.maxit, mode=problem.mode)
        ctx.problem = problem
        ctx.space, ctx.sysm = space, sysm          # the operator, not the solution
        ctx.save_for_backward(kappa, lam)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        kappa, lam = ctx.saved_tensors
        pb, space, sysm = ctx.problem, ctx.space, ctx.sysm
        # forward solution recomputed, not stored
        u, _ = sysm.solve(pb.b, rtol=pb.rtol, maxit=pb.maxit, mode=pb.mode)
        z, _ = sysm.solve(grad_u.contiguous(), rtol=pb.rtol, maxit=pb.maxit, mode=pb.mode)
        dk, dl = nk.param_grad(space, sysm.gather(z), sysm.gather(u))
        return dk.view_as(kappa), dl.view_as(lam), None


def helmholtz_solve(kappa, lam, problem: HelmholtzProblem):
    return HelmholtzSolve.apply(kappa, lam, problem)
