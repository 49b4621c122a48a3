"""Collapsed-coordinate triangles (oracle; test infrastructure only).

Section 2.1 of arXiv 1906.03489: triangles (and the other unstructured
shapes) are quadrilaterals with one coordinate direction collapsed, reached
through the Duffy map omega_T, and they carry expansions that factor in the
collapsed coordinates, which keeps sum-factorisation available (section 3.3).
The paper defers the basis and quadrature to the textbook it cites, so the
following readings are taken (each is pinned by tests/test_oracle.py):

* reference triangle T = {xi_1, xi_2 >= -1, xi_1 + xi_2 <= 0}; collapsed
  coordinates eta_1 = 2 (1 + xi_1) / (1 - xi_2) - 1, eta_2 = xi_2, so
  xi_1 = (1 + eta_1)(1 - eta_2)/2 - 1;
* modes, grouped by the eta_1 index p (the order used for the coefficients):
    p = 0:      q = 0: vertex A = a_0(eta_1) (1-eta_2)/2;  1 <= q < P: edge
                a_0(eta_1) b_q(eta_2);  q = P: vertex C = (1+eta_2)/2 (not
                multiplied by a_0: the collapsed vertex);
    0 < p < P:  q = 0: a_p(eta_1) ((1-eta_2)/2)^(p+1) (bottom edge);
                1 <= q <= P-1-p: a_p(eta_1) ((1-eta_2)/2)^(p+1) (1+eta_2)/2
                P^{2p+1,1}_{q-1}(eta_2) (interior);
    p = P:      q = 0: vertex B = a_P(eta_1) (1-eta_2)/2;  1 <= q < P: edge
                a_P(eta_1) b_q(eta_2),
  with a_p the 1-D modified basis of section 2.1 and b_q(z) = (1-z)/2 (1+z)/2
  P^{1,1}_{q-1}(z) its bubbles; (P+1)(P+2)/2 modes spanning the polynomials
  of total degree <= P;
* quadrature: Q Gauss-Lobatto-Legendre points in eta_1, Q-1 Gauss-Radau
  points of the weight (1 - eta_2) in eta_2 (eta_2 = -1 included, the
  collapsed vertex eta_2 = 1 excluded); dxi = (1 - eta_2)/2 deta, the factor
  (1 - eta_2) being the Radau weight.  Point q = i + Q j (eta_1 fastest).

Tetrahedra (the 3-D collapsed shape of section 2.1) are read the same way:
reference tetrahedron {xi_a >= -1, xi_1 + xi_2 + xi_3 <= -1}; collapsed
coordinates eta_1 = 2 (1 + xi_1)/(-xi_2 - xi_3) - 1, eta_2 = 2 (1 + xi_2)/
(1 - xi_3) - 1, eta_3 = xi_3.  Every mode is a triangle mode T_t(eta_1, eta_2)
of the order-P triangle above, of total degree s_t, times an eta_3 factor:
((1-eta_3)/2)^s_t for r = 0 (the modes of face ABC) and ((1-eta_3)/2)^s_t
(1+eta_3)/2 P^{2 s_t - 1, 1}_{r-1}(eta_3) for 1 <= r <= P - s_t (rising edge,
face and interior modes), plus the top vertex D = (1+eta_3)/2.  Coefficients
are grouped by triangle mode (in triangle order, r fastest), D last:
(P+1)(P+2)(P+3)/6 modes spanning total degree <= P.  Quadrature: Q GLL
points in eta_1, Q-1 Gauss-Radau points of the weight (1-eta_2) in eta_2 and
Q-1 of the weight (1-eta_3)^2 in eta_3; point q = i + Q (j + (Q-1) k).

Prisms: the triangle above in (xi_1, xi_2), extruded along xi_3 in [-1, 1]
(eta_1 = 2 (1 + xi_1)/(1 - xi_2) - 1, eta_2 = xi_2, xi_3 uncollapsed).  Every
mode is a triangle mode times the 1-D modified basis phi_r(xi_3), r = 0..P,
grouped by triangle mode with r fastest: (P+1)^2 (P+2)/2 modes spanning
P_P(triangle) x P_P(line).  Quadrature: GLL (Q) x Radau of (1-eta_2) (Q-1) x
GLL (Q); point q = i + Q (j + (Q-1) k).

Pyramids: base [-1, 1]^2 at xi_3 = -1, apex (-1, -1, 1) (xi_1 + xi_3 <= 0,
xi_2 + xi_3 <= 0); eta_1 = 2 (1 + xi_1)/(1 - xi_3) - 1, eta_2 = 2 (1 + xi_2)/
(1 - xi_3) - 1, eta_3 = xi_3.  Every mode is a base mode phi_p(eta_1)
phi_q(eta_2) (1-D modified bases) with s = max(deg phi_p, deg phi_q), times
((1-eta_3)/2)^s for r = 0 and ((1-eta_3)/2)^s (1+eta_3)/2
P^{2s-1,1}_{r-1}(eta_3) for 1 <= r <= P - s, grouped by base mode (p slow, q
fast, r fastest), plus the apex (1+eta_3)/2 last: (P+1)(P+2)(2P+3)/6 modes.
The base face carries the tensor-product quadrilateral basis and each
triangular face the triangle space above; the space contains every
polynomial of total degree <= P (with rational functions beyond, as the
collapsed construction gives).  Quadrature: GLL (Q) x GLL (Q) x Radau of
(1-eta_3)^2 (Q-1); point q = i + Q (j + Q k).
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi

from .basis import gll, jacobi_p, modified_basis


def gauss_radau_jacobi(n: int, alpha: float, beta: float):
    """n Gauss-Radau points (x = -1 included) and weights of the weight
    (1-x)^alpha (1+x)^beta on [-1, 1]: the interior points are the roots of
    P^{alpha, beta+1}_{n-1}; the weights are fixed by exactness on the
    monomials 1, x, ..., x^(n-1), whose moments come from a Gauss-Jacobi rule
    of the same weight (exact far beyond that degree)."""
    if n < 1:
        raise ValueError("n >= 1")
    inner = np.sort(roots_jacobi(n - 1, alpha, beta + 1)[0]) if n > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], inner])
    xg, wg = roots_jacobi(n + 8, alpha, beta)
    k = np.arange(n)
    moments = (wg[None, :] * xg[None, :] ** k[:, None]).sum(axis=1)
    V = x[None, :] ** k[:, None]
    w = np.linalg.solve(V, moments)
    return x, w


def tri_modes(P: int):
    """List of (p, q) in coefficient order (see the module docstring)."""
    modes = [(0, q) for q in range(P + 1)]
    for p in range(1, P):
        modes += [(p, q) for q in range(P - p)]
    modes += [(P, q) for q in range(P)]
    return modes


def _b_funcs(P: int, p: int, q: int, z):
    """(value, derivative) of the eta_2 factor of mode (p, q)."""
    z = np.asarray(z, np.float64)
    if p == 0 or p == P:
        if q == 0:
            return (1 - z) / 2, np.full_like(z, -0.5)
        if p == 0 and q == P:
            return (1 + z) / 2, np.full_like(z, 0.5)
        B, D = modified_basis(P, z)       # bubble q of the 1-D basis (q < P)
        return B[:, q], D[:, q]
    a = (1 - z) / 2
    if q == 0:
        return a ** (p + 1), -(p + 1) / 2 * a ** p
    J = jacobi_p(q - 1, 2 * p + 1, 1, z)
    dJ = ((q - 1 + 2 * p + 3) / 2 * jacobi_p(q - 2, 2 * p + 2, 2, z)) if q >= 2 else np.zeros_like(z)
    f = a ** (p + 1) * (1 + z) / 2
    df = -(p + 1) / 2 * a ** p * (1 + z) / 2 + a ** (p + 1) / 2
    return f * J, df * J + f * dJ


def tri_basis(P: int, e1, e2):
    """Basis values and collapsed-coordinate derivatives at points (e1, e2):
    (Phi, dPhi/deta_1, dPhi/deta_2), each (npts, nmodes)."""
    e1 = np.asarray(e1, np.float64)
    e2 = np.asarray(e2, np.float64)
    A, DA = modified_basis(P, e1)
    modes = tri_modes(P)
    Phi = np.zeros((e1.size, len(modes)))
    D1 = np.zeros_like(Phi)
    D2 = np.zeros_like(Phi)
    for m, (p, q) in enumerate(modes):
        b, db = _b_funcs(P, p, q, e2)
        if p == 0 and q == P:           # the collapsed vertex C: no eta_1 factor
            Phi[:, m], D1[:, m], D2[:, m] = b, 0.0, db
        else:
            Phi[:, m] = A[:, p] * b
            D1[:, m] = DA[:, p] * b
            D2[:, m] = A[:, p] * db
    return Phi, D1, D2


def tri_points(Q: int):
    """Collapsed quadrature: eta_1 (GLL, Q), eta_2 (Radau, Q-1) and the
    weights of dxi at every point q = i + Q j."""
    x1, w1 = gll(Q)
    x2, w2 = gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    E1 = np.tile(x1, Q - 1)
    E2 = np.repeat(x2, Q)
    W = np.outer(w2 / 2, w1).ravel()          # (1 - eta_2)/2 deta = (w2 / 2) w1
    return E1, E2, W


def xi_of_eta(e1, e2):
    return (1 + e1) * (1 - e2) / 2 - 1, e2


class TriOps:
    """Dense elemental operators of straight- or curved-sided triangles of
    order P with the collapsed quadrature of Q points.  J[e, c, a, q] =
    d x_c / d xi_a at the quadrature points."""

    def __init__(self, P, Q, J, kappa=None, lam=1.0):
        self.P, self.Q = int(P), int(Q)
        self.e1, self.e2, self.W = tri_points(self.Q)
        self.Bt, D1, D2 = tri_basis(self.P, self.e1, self.e2)
        # xi-derivatives by the chain rule through the Duffy map
        d1 = 2.0 / (1 - self.e2)
        d2 = (1 + self.e1) / (1 - self.e2)
        self.Dt = [d1[:, None] * D1, d2[:, None] * D1 + D2]
        Jm = np.moveaxis(np.asarray(J, np.float64), -1, 1)          # (E, nq, c, a)
        self.detJ = np.linalg.det(Jm)
        Ji = np.linalg.inv(Jm)
        self.G = np.einsum("eqac,eqbc->eqab", Ji, Ji)
        E = self.detJ.shape[0]
        self.nelem = E
        nq = self.W.size
        self.kappa = np.ones((E, nq)) if kappa is None else np.asarray(kappa, np.float64).reshape(E, nq)
        lam = np.asarray(lam, np.float64)
        self.lam = np.broadcast_to(lam, (E,)).copy() if lam.ndim == 0 else lam.reshape(E).copy()
        self.wJ = self.W[None, :] * self.detJ

    def mass_matrix(self, e):
        return self.Bt.T @ (self.wJ[e][:, None] * self.Bt)

    def laplacian_matrix(self, e):
        c = self.wJ[e] * self.kappa[e]
        L = np.zeros((self.Bt.shape[1],) * 2)
        for a in range(2):
            for b in range(2):
                L += self.Dt[a].T @ ((c * self.G[e, :, a, b])[:, None] * self.Dt[b])
        return L

    def helmholtz_matrix(self, e):
        return self.laplacian_matrix(e) + self.lam[e] * self.mass_matrix(e)

    def bwd(self, coeffs):
        return np.asarray(coeffs, np.float64) @ self.Bt.T

    def iprod(self, f):
        return (self.wJ * np.asarray(f, np.float64)) @ self.Bt

    def helmholtz(self, x):
        x = np.asarray(x, np.float64)
        return np.stack([self.helmholtz_matrix(e) @ x[e] for e in range(self.nelem)])

    def fwd(self, f):
        rhs = self.iprod(f)
        return np.stack([np.linalg.solve(self.mass_matrix(e), rhs[e]) for e in range(self.nelem)])


# ------------------------------------------------------------- tetrahedra

def tri_degree(P: int, p: int, q: int) -> int:
    """Total polynomial degree of triangle mode (p, q)."""
    if (p == 0 or p == P) and q == 0:
        return 1                  # vertices A, B
    if p == 0 and q == P:
        return 1                  # vertex C
    if p == 0 or p == P:
        return q + 1              # edges AC, BC: 1-D bubble q
    if q == 0:
        return p + 1              # edge AB
    return p + q + 1              # interior


def tet_modes(P: int):
    """List of (t, s, r) in coefficient order: t the index of the triangle
    mode in tri_modes(P), s its degree, r = 0..P-s; the top vertex D last as
    (-1, 0, 1)."""
    out = []
    for t, (p, q) in enumerate(tri_modes(P)):
        s = tri_degree(P, p, q)
        out += [(t, s, r) for r in range(P - s + 1)]
    return out + [(-1, 0, 1)]


def _c_funcs(s: int, r: int, z):
    """(value, derivative) of the eta_3 factor of a tet mode built on a
    triangle mode of degree s."""
    z = np.asarray(z, np.float64)
    a = (1 - z) / 2
    f = a ** s
    df = -s / 2 * a ** (s - 1) if s > 0 else np.zeros_like(z)
    if r == 0:
        return f, df
    g = (1 + z) / 2
    J = jacobi_p(r - 1, 2 * s - 1, 1, z)
    dJ = ((r - 1 + 2 * s + 1) / 2 * jacobi_p(r - 2, 2 * s, 2, z)) if r >= 2 else np.zeros_like(z)
    return f * g * J, df * g * J + f * 0.5 * J + f * g * dJ


def tet_basis(P: int, e1, e2, e3):
    """Basis values and collapsed-coordinate derivatives at points (e1, e2,
    e3): (Phi, dPhi/deta_1, dPhi/deta_2, dPhi/deta_3), each (npts, nmodes)."""
    e3 = np.asarray(e3, np.float64)
    T, T1, T2 = tri_basis(P, e1, e2)
    modes = tet_modes(P)
    Phi = np.zeros((e3.size, len(modes)))
    D1, D2, D3 = np.zeros_like(Phi), np.zeros_like(Phi), np.zeros_like(Phi)
    for m, (t, s, r) in enumerate(modes):
        if t < 0:                       # top vertex D: no eta_1, eta_2 factor
            Phi[:, m], D3[:, m] = (1 + e3) / 2, 0.5
            continue
        c, dc = _c_funcs(s, r, e3)
        Phi[:, m] = T[:, t] * c
        D1[:, m] = T1[:, t] * c
        D2[:, m] = T2[:, t] * c
        D3[:, m] = T[:, t] * dc
    return Phi, D1, D2, D3


def tet_points(Q: int):
    """Collapsed quadrature: eta_1 (GLL, Q), eta_2 (Radau of (1-x), Q-1),
    eta_3 (Radau of (1-x)^2, Q-1) and the weights of dxi at every point
    q = i + Q (j + (Q-1) k)."""
    x1, w1 = gll(Q)
    x2, w2 = gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    x3, w3 = gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    n2 = Q - 1
    E1 = np.tile(x1, n2 * n2)
    E2 = np.tile(np.repeat(x2, Q), n2)
    E3 = np.repeat(x3, Q * n2)
    # dxi = (1-eta_2)/2 ((1-eta_3)/2)^2 deta: the Radau weights carry (1-eta_2), (1-eta_3)^2
    W = (np.outer(w3 / 4, np.outer(w2 / 2, w1).ravel())).ravel()
    return E1, E2, E3, W


def xi_of_eta3(e1, e2, e3):
    e1, e2, e3 = (np.asarray(v, np.float64) for v in (e1, e2, e3))
    return (1 + e1) * (1 - e2) * (1 - e3) / 4 - 1, (1 + e2) * (1 - e3) / 2 - 1, e3


class TetOps:
    """Dense elemental operators of straight- or curved-sided tetrahedra of
    order P with the collapsed quadrature of Q points.  J[e, c, a, q] =
    d x_c / d xi_a at the quadrature points."""

    def __init__(self, P, Q, J, kappa=None, lam=1.0):
        self.P, self.Q = int(P), int(Q)
        self.e1, self.e2, self.e3, self.W = tet_points(self.Q)
        self.Bt, D1, D2, D3 = tet_basis(self.P, self.e1, self.e2, self.e3)
        e1, e2, e3 = self.e1, self.e2, self.e3
        # d eta_b / d xi_a of the collapsed map, then the chain rule
        g = (2.0 / ((1 - e2) * (1 - e3)))[:, None]
        c1 = (1 + e1)[:, None]
        dxi1 = 2 * g * D1
        dxi2 = c1 * g * D1 + (2.0 / (1 - e3))[:, None] * D2
        dxi3 = c1 * g * D1 + ((1 + e2) / (1 - e3))[:, None] * D2 + D3
        self.Dt = [dxi1, dxi2, dxi3]
        self._geometry(J, kappa, lam)

    def _geometry(self, J, kappa, lam):
        Jm = np.moveaxis(np.asarray(J, np.float64), -1, 1)          # (E, nq, c, a)
        self.detJ = np.linalg.det(Jm)
        Ji = np.linalg.inv(Jm)
        self.G = np.einsum("eqac,eqbc->eqab", Ji, Ji)
        E = self.detJ.shape[0]
        self.nelem = E
        nq = self.W.size
        self.kappa = np.ones((E, nq)) if kappa is None else np.asarray(kappa, np.float64).reshape(E, nq)
        lam = np.asarray(lam, np.float64)
        self.lam = np.broadcast_to(lam, (E,)).copy() if lam.ndim == 0 else lam.reshape(E).copy()
        # the integrals take |det J|: an element given with left-handed vertex
        # order (as sorting its vertices by global id can produce) has det J < 0
        self.wJ = self.W[None, :] * np.abs(self.detJ)

    def mass_matrix(self, e):
        return self.Bt.T @ (self.wJ[e][:, None] * self.Bt)

    def laplacian_matrix(self, e):
        c = self.wJ[e] * self.kappa[e]
        L = np.zeros((self.Bt.shape[1],) * 2)
        for a in range(3):
            for b in range(3):
                L += self.Dt[a].T @ ((c * self.G[e, :, a, b])[:, None] * self.Dt[b])
        return L

    def helmholtz_matrix(self, e):
        return self.laplacian_matrix(e) + self.lam[e] * self.mass_matrix(e)

    def bwd(self, coeffs):
        return np.asarray(coeffs, np.float64) @ self.Bt.T

    def iprod(self, f):
        return (self.wJ * np.asarray(f, np.float64)) @ self.Bt

    def helmholtz(self, x):
        x = np.asarray(x, np.float64)
        return np.stack([self.helmholtz_matrix(e) @ x[e] for e in range(self.nelem)])

    def fwd(self, f):
        rhs = self.iprod(f)
        return np.stack([np.linalg.solve(self.mass_matrix(e), rhs[e]) for e in range(self.nelem)])


# ----------------------------------------------------------------- prisms

def prism_modes(P: int):
    """List of (t, r) in coefficient order: triangle mode t, r = 0..P."""
    return [(t, r) for t in range(len(tri_modes(P))) for r in range(P + 1)]


def prism_basis(P: int, e1, e2, x3):
    """Basis values and derivatives at points (eta_1, eta_2, xi_3):
    (Phi, dPhi/deta_1, dPhi/deta_2, dPhi/dxi_3), each (npts, nmodes)."""
    T, T1, T2 = tri_basis(P, e1, e2)
    B, DB = modified_basis(P, np.asarray(x3, np.float64))
    modes = prism_modes(P)
    Phi = np.stack([T[:, t] * B[:, r] for t, r in modes], axis=1)
    D1 = np.stack([T1[:, t] * B[:, r] for t, r in modes], axis=1)
    D2 = np.stack([T2[:, t] * B[:, r] for t, r in modes], axis=1)
    D3 = np.stack([T[:, t] * DB[:, r] for t, r in modes], axis=1)
    return Phi, D1, D2, D3


def prism_points(Q: int):
    """eta_1 (GLL, Q), eta_2 (Radau of (1-x), Q-1), xi_3 (GLL, Q) and the
    weights of dxi at every point q = i + Q (j + (Q-1) k)."""
    x1, w1 = gll(Q)
    x2, w2 = gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    n2 = Q - 1
    E1 = np.tile(x1, n2 * Q)
    E2 = np.tile(np.repeat(x2, Q), Q)
    X3 = np.repeat(x1, Q * n2)
    W = (np.outer(w1, np.outer(w2 / 2, w1).ravel())).ravel()
    return E1, E2, X3, W


class PrismOps(TetOps):
    """Dense elemental operators of straight- or curved-sided prisms of order
    P with the quadrature of prism_points(Q).  J[e, c, a, q] = d x_c / d xi_a."""

    def __init__(self, P, Q, J, kappa=None, lam=1.0):
        self.P, self.Q = int(P), int(Q)
        self.e1, self.e2, self.e3, self.W = prism_points(self.Q)
        self.Bt, D1, D2, D3 = prism_basis(self.P, self.e1, self.e2, self.e3)
        e1, e2 = self.e1, self.e2
        # d eta / d xi of the collapsed triangle; xi_3 is not collapsed
        self.Dt = [(2.0 / (1 - e2))[:, None] * D1,
                   ((1 + e1) / (1 - e2))[:, None] * D1 + D2,
                   D3]
        self._geometry(J, kappa, lam)


# --------------------------------------------------------------- pyramids

def _deg1(P: int, p: int) -> int:
    """Polynomial degree of the 1-D modified basis function p."""
    return 1 if p in (0, P) else p + 1


def pyr_modes(P: int):
    """List of (p, q, s, r) in coefficient order; the apex last as
    (-1, -1, 0, 1)."""
    out = []
    for p in range(P + 1):
        for q in range(P + 1):
            s = max(_deg1(P, p), _deg1(P, q))
            out += [(p, q, s, r) for r in range(P - s + 1)]
    return out + [(-1, -1, 0, 1)]


def pyr_basis(P: int, e1, e2, e3):
    """Basis values and collapsed derivatives at points (eta_1, eta_2,
    eta_3): (Phi, d/deta_1, d/deta_2, d/deta_3), each (npts, nmodes)."""
    e3 = np.asarray(e3, np.float64)
    A1, D1a = modified_basis(P, np.asarray(e1, np.float64))
    A2, D2a = modified_basis(P, np.asarray(e2, np.float64))
    modes = pyr_modes(P)
    Phi = np.zeros((e3.size, len(modes)))
    D1, D2, D3 = np.zeros_like(Phi), np.zeros_like(Phi), np.zeros_like(Phi)
    for m, (p, q, s, r) in enumerate(modes):
        if p < 0:
            Phi[:, m], D3[:, m] = (1 + e3) / 2, 0.5
            continue
        c, dc = _c_funcs(s, r, e3)
        Phi[:, m] = A1[:, p] * A2[:, q] * c
        D1[:, m] = D1a[:, p] * A2[:, q] * c
        D2[:, m] = A1[:, p] * D2a[:, q] * c
        D3[:, m] = A1[:, p] * A2[:, q] * dc
    return Phi, D1, D2, D3


def pyr_points(Q: int):
    """GLL (Q) x GLL (Q) x Radau of (1-x)^2 (Q-1) and the weights of dxi,
    q = i + Q (j + Q k)."""
    x1, w1 = gll(Q)
    x3, w3 = gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    E1 = np.tile(x1, Q * (Q - 1))
    E2 = np.tile(np.repeat(x1, Q), Q - 1)
    E3 = np.repeat(x3, Q * Q)
    W = np.outer(w3 / 4, np.outer(w1, w1).ravel()).ravel()
    return E1, E2, E3, W


def xi_of_eta_pyr(e1, e2, e3):
    e1, e2, e3 = (np.asarray(v, np.float64) for v in (e1, e2, e3))
    return (1 + e1) * (1 - e3) / 2 - 1, (1 + e2) * (1 - e3) / 2 - 1, e3


class PyrOps(TetOps):
    """Dense elemental operators of pyramids of order P with the quadrature
    of pyr_points(Q).  J[e, c, a, q] = d x_c / d xi_a."""

    def __init__(self, P, Q, J, kappa=None, lam=1.0):
        self.P, self.Q = int(P), int(Q)
        self.e1, self.e2, self.e3, self.W = pyr_points(self.Q)
        self.Bt, D1, D2, D3 = pyr_basis(self.P, self.e1, self.e2, self.e3)
        e1, e2, e3 = self.e1, self.e2, self.e3
        g = (2.0 / (1 - e3))[:, None]
        self.Dt = [g * D1, g * D2,
                   ((1 + e1) / (1 - e3))[:, None] * D1 + ((1 + e2) / (1 - e3))[:, None] * D2 + D3]
        self._geometry(J, kappa, lam)
