"""Static condensation of the assembled system (oracle; test infrastructure only).

Section 2.1 of arXiv 1906.03489: with the modified basis, each tensor-product
element's modes split into boundary modes (a vertex mode 0 or P in at least
one direction) and interior modes (a bubble in every direction); the interior
modes of an element belong to that element alone, so the assembled system can
be condensed onto the elemental boundary degrees of freedom and the interior
unknowns recovered element by element afterwards.  With spatially variable
order (section 4.2) each element has its own (P_e - 1)^dim interior modes.

With the elemental matrix partitioned into boundary (b) and interior (i)
blocks,

    S_e = H_bb - H_bi H_ii^{-1} H_ib            (elemental Schur complement)
    S   = sum_e R_e^T S_e R_e                  (assembled over boundary DOFs)
    g   = b_B - sum_e R_e^T H_bi H_ii^{-1} b_i(e)
    S x_B = g,   x_i(e) = H_ii^{-1} (b_i(e) - H_ib R_e x_B)

where R_e gathers element e's boundary modes from the global boundary vector
(with the local sign of each mode) and b_i(e) are the assembled right-hand
side entries of element e's interior DOFs.  Dense FP64 linear algebra per
element (numpy solves); the global solve is the sparse direct one.

Readings taken where the paper is silent: homogeneous Dirichlet data as in
the full system (Dirichlet DOFs are boundary DOFs; their rows and columns are
removed from S); an interior mode's DOF must be referenced by that one mode
only (otherwise the map is not condensable); interior modes are numbered in
increasing local mode index (first tensor index fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import assembled_matrix


def interior_modes(dim: int, P: int) -> np.ndarray:
    """Mask over the n^dim tensor modes (first index fastest): True where every
    1-D index is a bubble (0 < p < P)."""
    n = P + 1
    idx = np.indices((n,) * dim).reshape(dim, -1)[::-1]
    return np.all((idx > 0) & (idx < P), axis=0)


def element_blocks(H, interior):
    """(H_bb, H_bi, H_ib, H_ii) of one elemental matrix."""
    H = np.asarray(H, np.float64)
    b = ~interior
    return H[b][:, b], H[b][:, interior], H[interior][:, b], H[interior][:, interior]


def schur_complement(H, interior):
    """S_e = H_bb - H_bi H_ii^{-1} H_ib."""
    Hbb, Hbi, Hib, Hii = element_blocks(H, interior)
    if Hii.shape[0] == 0:
        return Hbb.copy()
    return Hbb - Hbi @ np.linalg.solve(Hii, Hib)


class Condensed:
    """The condensed boundary system of an assembled hexahedral (dim = 3) or
    quadrilateral (dim = 2) C0 system, at one order P or with per-element
    orders (l2g a list of per-element maps of lengths (P_e + 1)^dim; P is
    then ignored and each element's order follows from its map).

    bdofs: sorted global DOFs referenced by boundary modes; S (sparse, over
    bdofs, Dirichlet rows and columns kept); the per-element blocks and maps."""

    def __init__(self, mats, l2g, nglobal, dirichlet, dim, P, sign=None):
        E = len(l2g)
        maps = [np.asarray(l2g[e], np.int64).ravel() for e in range(E)]
        signs = [np.ones(m.size) if sign is None else np.asarray(sign[e], np.float64).ravel()
                 for e, m in enumerate(maps)]
        self.dim, self.nglobal = dim, int(nglobal)
        orders = [int(round(m.size ** (1.0 / dim))) - 1 for m in maps]
        self.P = P if len(set(orders)) > 1 else orders[0]
        masks = {q: interior_modes(dim, q) for q in set(orders)}
        self.inner = [masks[q] for q in orders]
        self.dirichlet = np.asarray(dirichlet, bool)
        allg = np.concatenate(maps)
        counts = np.bincount(allg, minlength=self.nglobal)
        ig = np.concatenate([m[k] for m, k in zip(maps, self.inner)])
        if ig.size and (np.any(counts[ig] != 1) or np.any(self.dirichlet[ig])):
            raise ValueError("an interior mode's DOF is shared or Dirichlet: not condensable")
        self.bdofs = np.unique(np.concatenate([m[~k] for m, k in zip(maps, self.inner)]))
        pos = -np.ones(self.nglobal, np.int64)
        pos[self.bdofs] = np.arange(self.bdofs.size)
        self.bpos = [pos[m[~k]] for m, k in zip(maps, self.inner)]
        self.bsign = [sg[~k] for sg, k in zip(signs, self.inner)]
        self.isign = [sg[k] for sg, k in zip(signs, self.inner)]
        self.idofs = [m[k] for m, k in zip(maps, self.inner)]
        self.blocks = [element_blocks(H, k) for H, k in zip(mats, self.inner)]
        nb = self.bdofs.size
        rows, cols, vals = [], [], []
        for e in range(E):
            Se = schur_complement(mats[e], self.inner[e])
            sg = self.bsign[e]
            rows.append(np.repeat(self.bpos[e], sg.size))
            cols.append(np.tile(self.bpos[e], sg.size))
            vals.append((sg[:, None] * Se * sg[None, :]).ravel())
        self.S = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(nb, nb))
        self.bfree = ~self.dirichlet[self.bdofs]

    def apply(self, xb):
        """S x_B with Dirichlet entries of x_B taken as zero and the Dirichlet
        rows of the result zero (the boundary restriction of the system)."""
        x = np.where(self.bfree, np.asarray(xb, np.float64), 0.0)
        return np.where(self.bfree, self.S @ x, 0.0)

    def rhs(self, b):
        """g = b_B - sum_e R_e^T H_bi H_ii^{-1} b_i(e), zero on Dirichlet DOFs."""
        b = np.asarray(b, np.float64)
        g = b[self.bdofs].copy()
        for e, (Hbb, Hbi, Hib, Hii) in enumerate(self.blocks):
            if Hii.shape[0] == 0:
                continue
            bi = self.isign[e] * b[self.idofs[e]]
            np.add.at(g, self.bpos[e], -self.bsign[e] * (Hbi @ np.linalg.solve(Hii, bi)))
        return np.where(self.bfree, g, 0.0)

    def interior_solution(self, xb, b):
        """Full solution vector from the boundary one: x_i(e) =
        H_ii^{-1}(b_i(e) - H_ib R_e x_B); Dirichlet DOFs zero."""
        b = np.asarray(b, np.float64)
        xb = np.where(self.bfree, np.asarray(xb, np.float64), 0.0)
        x = np.zeros(self.nglobal)
        x[self.bdofs] = xb
        x[self.dirichlet] = 0.0
        for e, (Hbb, Hbi, Hib, Hii) in enumerate(self.blocks):
            if Hii.shape[0] == 0:
                continue
            xl = self.bsign[e] * xb[self.bpos[e]]
            bi = self.isign[e] * b[self.idofs[e]]
            x[self.idofs[e]] = self.isign[e] * np.linalg.solve(Hii, bi - Hib @ xl)
        return x

    def solve(self, b):
        """Sparse direct solve of the condensed system, then the interior
        recovery: the full solution x."""
        g = self.rhs(b)
        f = np.flatnonzero(self.bfree)
        xb = np.zeros(self.bdofs.size)
        if f.size:
            xb[f] = spla.spsolve(self.S[f][:, f].tocsc(), g[f])
        return self.interior_solution(xb, b)


def condensed_solve(mats, l2g, nglobal, dirichlet, b, dim, P, sign=None):
    """Solution of the Dirichlet-restricted assembled system by static
    condensation (boundary solve, then interior recovery)."""
    return Condensed(mats, l2g, nglobal, dirichlet, dim, P, sign).solve(b)


def global_schur(mats, l2g, nglobal, interior_dofs, sign=None):
    """Schur complement of the assembled matrix onto the complement of the
    given global DOF set, formed from the assembled matrix by block
    elimination (no elemental structure used): A_BB - A_BI A_II^{-1} A_IB,
    rows and columns in increasing global DOF order."""
    A = assembled_matrix(mats, l2g, nglobal, sign).tocsc()
    Iset = np.zeros(nglobal, bool)
    Iset[np.asarray(interior_dofs, np.int64)] = True
    I, B = np.flatnonzero(Iset), np.flatnonzero(~Iset)
    Abb = A[B][:, B].toarray()
    if I.size == 0:
        return B, Abb
    Aii = A[I][:, I].tocsc()
    Aib = A[I][:, B].toarray()
    return B, Abb - A[B][:, I].toarray() @ spla.spsolve(Aii, Aib)
