"""Dense elemental operators (oracle; test infrastructure only).

Each operator of the matrix-free path is written here as its plain
definition: the tensor-product basis is formed explicitly with Kronecker
products, every elemental matrix is built, and the operator is a dense
matrix-vector product per element (the "StdMat" strategy named in section 3.3
of arXiv 1906.03489).  Sum-factorisation (section 3.3) is an exact reordering
of these products, so the GPU path must reproduce them up to rounding.

Index conventions: tensor point q = i + Q*(j + Q*l) and tensor mode
m = p + n*(q + n*r), direction 1 fastest; in a Kronecker product the
rightmost factor carries direction 1.

Geometry (section 2.1, the map chi_e): J = dx/dxi at every quadrature point,
G = J^{-1} J^{-T} so that grad_x u . grad_x v = (grad_xi u)^T G grad_xi v.

Helmholtz operator (the weak form a(u, v) of Eq. (1) for -div(kappa grad u)
+ lambda u; the paper does not write it out): H_e = L_e + lambda_e M_e with
  M_e = B^T diag(w detJ) B,
  L_e = sum_{a,b} (D_a B)^T diag(w detJ kappa G_ab) (D_b B).
Reading taken: the sign convention that makes H_e symmetric positive
definite for lambda >= 0 (the filter equation (3) has this form).
"""
from __future__ import annotations

import numpy as np

from .basis import gll, lagrange_derivative, modified_basis


def tensor_bases(B, DB, w, dim):
    """Tensor-product basis on the reference square/cube.

    Returns (Bt, [D_1 Bt, ..., D_d Bt], Wt): Bt[q, m] = prod_a B[i_a, p_a],
    D_a Bt has DB in direction a, Wt[q] = prod_a w[i_a]."""
    if dim == 2:
        Bt = np.kron(B, B)
        Dt = [np.kron(B, DB), np.kron(DB, B)]
        Wt = np.kron(w, w)
    elif dim == 3:
        Bt = np.kron(B, np.kron(B, B))
        Dt = [np.kron(B, np.kron(B, DB)),
              np.kron(B, np.kron(DB, B)),
              np.kron(DB, np.kron(B, B))]
        Wt = np.kron(w, np.kron(w, w))
    else:
        raise ValueError("dim must be 2 or 3")
    return Bt, Dt, Wt


def collocation_derivatives(x, dim):
    """Tensor collocation derivatives on the GLL grid x (per direction):
    (D_a u)[q] is the xi_a-derivative at point q of the interpolant of the
    point values u, built from the 1-D Lagrange derivative matrix; direction 1
    is the rightmost Kronecker factor."""
    D = lagrange_derivative(x)
    I = np.eye(len(x))
    if dim == 2:
        return [np.kron(I, D), np.kron(D, I)]
    if dim == 3:
        return [np.kron(I, np.kron(I, D)), np.kron(I, np.kron(D, I)), np.kron(D, np.kron(I, I))]
    raise ValueError("dim must be 2 or 3")


def inverse_jacobian(J):
    """Jinv[e, q, a, c] = d xi_a / d x_c, the matrix inverse of
    J[e, :, :, q] = d x_c / d xi_a."""
    Jm = np.moveaxis(np.asarray(J, np.float64), -1, 1)     # (E, nq, c, a)
    return np.linalg.inv(Jm)                               # (E, nq, a, c)


def geometry(J):
    """detJ[e, q] and G[e, q, a, b] = (J^{-1} J^{-T})_{ab} from
    J[e, c, a, q] = d x_c / d xi_a."""
    Jm = np.moveaxis(np.asarray(J, np.float64), -1, 1)     # (E, nq, c, a)
    detJ = np.linalg.det(Jm)
    Jinv = np.linalg.inv(Jm)                               # (E, nq, a, c)
    G = np.einsum("eqac,eqbc->eqab", Jinv, Jinv)
    return detJ, G


class ElementOps:
    """All elements of one same-shape, same-basis group (section 3.3's
    collection) at order P with Q GLL points per direction."""

    def __init__(self, dim, P, Q, J, kappa=None, lam=1.0):
        self.dim, self.P, self.Q = int(dim), int(P), int(Q)
        self.n = self.P + 1
        self.x, self.w = gll(self.Q)
        self.B, self.DB = modified_basis(self.P, self.x)
        self.Bt, self.Dt, self.Wt = tensor_bases(self.B, self.DB, self.w, self.dim)
        self.detJ, self.G = geometry(J)
        E = self.detJ.shape[0]
        self.nelem = E
        nq = self.Q ** self.dim
        self.kappa = np.ones((E, nq)) if kappa is None else np.asarray(kappa, np.float64).reshape(E, nq)
        lam = np.asarray(lam, np.float64)
        self.lam = np.broadcast_to(lam, (E,)).copy() if lam.ndim == 0 else lam.reshape(E).copy()
        self.wJ = self.Wt[None, :] * self.detJ                 # (E, nq)
        self.Jinv = inverse_jacobian(J)                        # (E, nq, a, c)
        self.Dcol = collocation_derivatives(self.x, self.dim)

    # -- elemental matrices ------------------------------------------------
    def mass_matrix(self, e):
        return self.Bt.T @ (self.wJ[e][:, None] * self.Bt)

    def laplacian_matrix(self, e):
        c = self.wJ[e] * self.kappa[e]
        L = np.zeros((self.n ** self.dim,) * 2)
        for a in range(self.dim):
            for b in range(self.dim):
                L += self.Dt[a].T @ ((c * self.G[e, :, a, b])[:, None] * self.Dt[b])
        return L

    def helmholtz_matrix(self, e):
        return self.laplacian_matrix(e) + self.lam[e] * self.mass_matrix(e)

    def iprod_matrix(self, e):
        return self.Bt.T * self.wJ[e][None, :]

    def dkappa_matrix(self, e, q):
        """d H_e / d kappa_{e,q}: the Laplacian's single-point contribution
        w_q detJ_q sum_ab (D_a B)[q,:]^T G_ab (D_b B)[q,:]."""
        rows = np.stack([self.Dt[a][q] for a in range(self.dim)])   # (d, nm)
        return self.wJ[e, q] * rows.T @ self.G[e, q] @ rows

    # -- dense applies -----------------------------------------------------
    def bwd(self, coeffs):
        """BwdTrans: u_e = Bt u^_e (elemental expansion, section 2.1)."""
        return np.asarray(coeffs, np.float64) @ self.Bt.T

    def iprod(self, f):
        """IProductWRTBase: I_e = Bt^T diag(w detJ) f_e."""
        f = np.asarray(f, np.float64)
        return np.stack([self.iprod_matrix(e) @ f[e] for e in range(self.nelem)])

    def helmholtz(self, x, elems=None):
        """y_e = H_e x_e for the listed elements (default all)."""
        x = np.asarray(x, np.float64)
        elems = range(self.nelem) if elems is None else elems
        return np.stack([self.helmholtz_matrix(e) @ x[e] for e in elems])

    def helmholtz_action(self, x, elems=None):
        """y_e = H_e x_e for the listed elements (x holds one row per listed
        element, or per element when none are listed), evaluated as the same
        quadrature sums without forming H_e: the reference gradient D_b B x_e
        and value B x_e at every point, weighted by w detJ (kappa G_ab, and
        lambda for the mass term), tested against D_a B and B.  Equal to
        `helmholtz` up to rounding; it costs O(Q^d n^d) per element instead
        of O(Q^d n^2d), so full-size meshes can be sampled at high order."""
        x = np.asarray(x, np.float64)
        elems = list(range(self.nelem)) if elems is None else list(elems)
        out = []
        for k, e in enumerate(elems):
            xe = x[k]
            grad = np.stack([self.Dt[b] @ xe for b in range(self.dim)])          # (d, nq)
            c = self.wJ[e] * self.kappa[e]
            flux = np.einsum("qab,bq->aq", self.G[e], grad) * c[None, :]
            y = sum(self.Dt[a].T @ flux[a] for a in range(self.dim))
            out.append(y + self.lam[e] * (self.Bt.T @ (self.wJ[e] * (self.Bt @ xe))))
        return np.stack(out)

    def weak_rhs(self, U, dU):
        """l_e[m] = a_e(U, phi_m) for a field given by its values U[e, q] and
        reference gradient dU[e, a, q] at the quadrature points:
        sum_a (D_a B)^T (w detJ kappa sum_b G_ab dU_b) + lambda_e Bt^T (w detJ U)."""
        U = np.asarray(U, np.float64)
        dU = np.asarray(dU, np.float64)
        out = np.zeros((self.nelem, self.n ** self.dim))
        for e in range(self.nelem):
            c = self.wJ[e] * self.kappa[e]
            acc = self.lam[e] * (self.Bt.T @ (self.wJ[e] * U[e]))
            for a in range(self.dim):
                ga = np.zeros(self.Q ** self.dim)
                for b in range(self.dim):
                    ga += self.G[e, :, a, b] * dU[e, b]
                acc += self.Dt[a].T @ (c * ga)
            out[e] = acc
        return out

    def phys_deriv(self, u):
        """PhysDeriv (differentiation, one of the core elemental operations
        listed in section 2.3): du[e, c, q] = d u / d x_c at the quadrature
        points, for u given by its values there.  Reference derivatives come
        from the collocation derivative of the interpolant; the chain rule
        gives d u / d x_c = sum_a (d xi_a / d x_c) d u / d xi_a."""
        u = np.asarray(u, np.float64)
        dref = np.stack([u @ Da.T for Da in self.Dcol], axis=1)      # (E, a, nq)
        return np.einsum("eqac,eaq->ecq", self.Jinv, dref)

    def iprod_deriv(self, f):
        """IProductWRTDerivBase (the volume term of the weak form in section
        2.2): I_e[m] = sum_q w_q detJ_q sum_c (d phi_m / d x_c)(x_q) f_c(x_q)
        = sum_a (D_a B)^T [w detJ sum_c (d xi_a / d x_c) f_c], for a vector
        field f[e, c, q] given at the quadrature points."""
        f = np.asarray(f, np.float64)
        g = np.einsum("eqac,ecq->eaq", self.Jinv, f) * self.wJ[:, None, :]
        return sum(g[:, a, :] @ self.Dt[a] for a in range(self.dim))

    def fwd(self, f):
        """FwdTrans (the projection called in the listing of section 3.5):
        the coefficients of the elemental L2 projection of the point values
        f, u^_e = M_e^{-1} I_e(f), solved densely per element."""
        rhs = self.iprod(f)
        return np.stack([np.linalg.solve(self.mass_matrix(e), rhs[e]) for e in range(self.nelem)])

    def integral(self, f):
        """Integral of a field given at the quadrature points over each
        element: sum_q w_q detJ_q f_q."""
        return (self.wJ * np.asarray(f, np.float64)).sum(axis=1)


# Convenience functional forms --------------------------------------------

def bwd_trans(ops: ElementOps, coeffs):
    return ops.bwd(coeffs)


def iprod_wrt_base(ops: ElementOps, f):
    return ops.iprod(f)


def phys_deriv(ops: ElementOps, u):
    return ops.phys_deriv(u)


def iprod_deriv(ops: ElementOps, f):
    return ops.iprod_deriv(f)


def fwd_trans(ops: ElementOps, f):
    return ops.fwd(f)


def helmholtz_apply(ops: ElementOps, x, elems=None):
    return ops.helmholtz(x, elems)


def helmholtz_matrices(ops: ElementOps):
    return [ops.helmholtz_matrix(e) for e in range(ops.nelem)]


def mass_matrices(ops: ElementOps):
    return [ops.mass_matrix(e) for e in range(ops.nelem)]


def weak_rhs(ops: ElementOps, U, dU):
    return ops.weak_rhs(U, dU)
