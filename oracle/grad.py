"""Gradients of a solve's loss (oracle; test infrastructure only).

For the discrete weak problem of Eqs. (1)-(2) of arXiv 1906.03489 with the
Helmholtz bilinear form  a(u, v) = sum_e [kappa grad u . grad v + lambda_e u v],
u = A(kappa, lambda)^{-1} b with b fixed (homogeneous Dirichlet data), and a
loss L(u), the adjoint identity gives
  dL/dtheta = -z^T (dA/dtheta) u,   A z = dL/du   (A symmetric).
Assembly is linear, so dA/dlambda_e and dA/dkappa_{e,q} are the assembled
single-element matrices M_e and dH_e/dkappa_{e,q}.

Reading taken: L = 0.5 ||u - u_t||_2^2 over the global coefficient vector
(Dirichlet entries are zero in both), lambda per element, kappa per
quadrature point.
"""
from __future__ import annotations

import numpy as np

from .assembly import gather, direct_solve


def loss_and_solution(mats, l2g, nglobal, dirichlet, b, u_t):
    """u = A^{-1} b by sparse direct solve and L = 0.5 ||u - u_t||^2."""
    u = direct_solve(mats, l2g, nglobal, dirichlet, b)
    return 0.5 * float(np.sum((u - u_t) ** 2)), u


def param_grad(ops, l2g, u, z):
    """dL/dlambda[e] = -z_e^T M_e u_e and dL/dkappa[e, q] = -z_e^T dH_e/dkappa_q u_e,
    each matrix built explicitly (definition, one entry at a time)."""
    ul = gather(u, l2g)
    zl = gather(z, l2g)
    E = ops.nelem
    nq = ops.Q ** ops.dim
    dlam = np.zeros(E)
    dkap = np.zeros((E, nq))
    for e in range(E):
        dlam[e] = -zl[e] @ ops.mass_matrix(e) @ ul[e]
        for q in range(nq):
            dkap[e, q] = -zl[e] @ ops.dkappa_matrix(e, q) @ ul[e]
    return dkap, dlam
