"""C0 assembly and linear solves (oracle; test infrastructure only).

Section 2.1 of arXiv 1906.03489: the global C0 expansion is built from the
elemental ones by an assembly operator that sums neighbouring elements'
contributions; the weak problem of Eqs. (1)-(2) becomes a linear system for
the global coefficients.  Homogeneous Dirichlet data: the Dirichlet global
coefficients are fixed at zero and their rows/columns removed (the lifting of
section 2.1 with g_D = 0).

Readings taken where the paper is silent: the assembly map is the given
local-to-global index array, optionally with a sign +-1 per local mode (an
unstructured mesh whose elements traverse a shared edge or face in opposite
directions see its odd-parity bubbles negated): the local coefficient is
sign * x[l2g].  CG is Jacobi-preconditioned, starts from x0 = 0 and stops on
the true relative residual ||b - A x||_2 / ||b||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _ragged(l2g):
    """True for a list of per-element maps of different lengths (elements of
    different orders); such maps and their local vectors stay lists."""
    return isinstance(l2g, (list, tuple)) and len({len(g) for g in l2g}) > 1


def _signs(l2g, sign):
    """Per-element sign arrays (all +1 when sign is None)."""
    if sign is None:
        return [np.ones(len(g)) for g in l2g]
    return [np.asarray(s, np.float64) for s in sign]


def gather(x, l2g, sign=None):
    """Local copies x_loc[e, m] = sign[e, m] * x[l2g[e, m]]."""
    x = np.asarray(x, np.float64)
    if _ragged(l2g):
        return [s * x[np.asarray(g)] for g, s in zip(l2g, _signs(l2g, sign))]
    out = x[np.asarray(l2g)]
    return out if sign is None else out * np.asarray(sign, np.float64)


def assemble_vector(yloc, l2g, nglobal, sign=None):
    """Scatter-add y[l2g[e, m]] += sign[e, m] * yloc[e, m] (the transpose of
    `gather`)."""
    y = np.zeros(nglobal)
    if _ragged(l2g):
        for g, v, s in zip(l2g, yloc, _signs(l2g, sign)):
            np.add.at(y, np.asarray(g), s * np.asarray(v, np.float64))
        return y
    v = np.asarray(yloc, np.float64)
    if sign is not None:
        v = v * np.asarray(sign, np.float64)
    np.add.at(y, np.asarray(l2g).ravel(), v.ravel())
    return y


def assembled_matrix(mats, l2g, nglobal, sign=None):
    """Global sparse matrix sum_e A_e^T H_e A_e from elemental matrices, A_e
    the signed Boolean gather of element e."""
    rows, cols, vals = [], [], []
    for e, (H, s) in enumerate(zip(mats, _signs(l2g, sign))):
        g = np.asarray(l2g[e])
        rows.append(np.repeat(g, g.size))
        cols.append(np.tile(g, g.size))
        vals.append((s[:, None] * np.asarray(H) * s[None, :]).ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nglobal, nglobal))
    return A.tocsr()


def jacobi_diagonal(mats, l2g, nglobal, dirichlet, sign=None):
    """diag(A) assembled from the elemental diagonals (signs square away);
    Dirichlet rows set to one (they are not unknowns)."""
    dloc = [np.diag(H) for H in mats]
    d = assemble_vector(dloc if _ragged(l2g) else np.stack(dloc), l2g, nglobal)
    d[np.asarray(dirichlet, bool)] = 1.0
    return d


class MaskedOperator:
    """x -> mask(assemble(H_e gather(mask x))) with prebuilt H_e."""

    def __init__(self, mats, l2g, nglobal, dirichlet, sign=None):
        self.mats = mats
        self.l2g = l2g if _ragged(l2g) else np.asarray(l2g)
        self.sign = sign
        self.nglobal = int(nglobal)
        self.free = ~np.asarray(dirichlet, bool)

    def __call__(self, x):
        xm = np.where(self.free, x, 0.0)
        xl = gather(xm, self.l2g, self.sign)
        yl = [H @ xl[e] for e, H in enumerate(self.mats)]
        if not _ragged(self.l2g):
            yl = np.stack(yl)
        y = assemble_vector(yl, self.l2g, self.nglobal, self.sign)
        return np.where(self.free, y, 0.0)


def pcg(apply_A, b, diag, rtol=1e-13, maxit=100000, x0=None):
    """Jacobi-preconditioned conjugate gradients (textbook form).

    Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    r = b - apply_A(x)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    z = r / diag
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * bn and it < maxit:
        Ap = apply_A(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    res = np.linalg.norm(b - apply_A(x)) / bn
    return x, it, res


def direct_solve(mats, l2g, nglobal, dirichlet, b, sign=None):
    """Sparse direct solve of the Dirichlet-restricted system A_II x_I = b_I."""
    A = assembled_matrix(mats, l2g, nglobal, sign)
    free = np.flatnonzero(~np.asarray(dirichlet, bool))
    AII = A[free][:, free].tocsc()
    x = np.zeros(nglobal)
    x[free] = spla.spsolve(AII, np.asarray(b, np.float64)[free])
    return x
