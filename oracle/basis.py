"""1-D quadrature and basis tables (oracle; test infrastructure only).

Follows section 2.1 of arXiv 1906.03489: the modified hierarchical C0 basis
phi_p (the unnumbered display) evaluated at Gauss-Lobatto-Legendre points.
The paper names GLL quadrature but prints no formula; the textbook definition
is used (interior points are the roots of the derivative of the Legendre
polynomial of degree Q-1; w_i = 2 / (Q (Q-1) L_{Q-1}(x_i)^2)).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import eval_jacobi


def gll(Q: int):
    """Q Gauss-Lobatto-Legendre points (ascending, -1 and 1 included) and
    weights, in FP64."""
    if Q < 2:
        raise ValueError("GLL needs Q >= 2")
    cQ = np.zeros(Q)
    cQ[-1] = 1.0                      # Legendre series of L_{Q-1}
    interior = np.sort(np.real(npleg.legroots(npleg.legder(cQ))))
    x = np.concatenate([[-1.0], interior, [1.0]])
    LQ = npleg.legval(x, cQ)
    w = 2.0 / (Q * (Q - 1) * LQ ** 2)
    return x, w


def jacobi_p(k: int, a: float, b: float, x):
    """Jacobi polynomial P_k^{(a,b)}(x), standard normalisation
    (P_k^{(a,b)}(1) = binom(k+a, k))."""
    return eval_jacobi(k, a, b, np.asarray(x, np.float64))


def modified_basis(P: int, x):
    """B[i, p] = phi_p(x_i) and DB[i, p] = phi_p'(x_i), 0 <= p <= P.

    Section 2.1, modified basis display:
      phi_0 = (1-x)/2,  phi_P = (1+x)/2,
      phi_p = (1-x)/2 (1+x)/2 P^{1,1}_{p-1}(x),  0 < p < P.
    P is the polynomial order (n = P+1 modes).  Derivative of the bubble:
      d/dx[(1-x^2)/4 J_{k}] = -x/2 J_k + (1-x^2)/4 J_k',
      J_k' = (k+3)/2 P^{2,2}_{k-1}  (derivative rule for Jacobi polynomials).
    """
    x = np.asarray(x, np.float64)
    n = P + 1
    B = np.zeros((x.size, n))
    DB = np.zeros((x.size, n))
    B[:, 0] = (1.0 - x) / 2.0
    DB[:, 0] = -0.5
    B[:, P] = (1.0 + x) / 2.0
    DB[:, P] = 0.5
    for p in range(1, P):
        k = p - 1
        Jk = jacobi_p(k, 1.0, 1.0, x)
        dJk = (k + 3) / 2.0 * jacobi_p(k - 1, 2.0, 2.0, x) if k >= 1 else np.zeros_like(x)
        B[:, p] = (1.0 - x) / 2.0 * (1.0 + x) / 2.0 * Jk
        DB[:, p] = -x / 2.0 * Jk + (1.0 - x * x) / 4.0 * dJk
    return B, DB


def lagrange_derivative(x):
    """Collocation derivative matrix D[i, j] = l_j'(x_i) of the Lagrange
    polynomials through the nodes x (barycentric form; any distinct nodes)."""
    x = np.asarray(x, np.float64)
    n = x.size
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1.0)
    wb = 1.0 / np.prod(diff, axis=1)
    D = (wb[None, :] / wb[:, None]) / diff
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D
