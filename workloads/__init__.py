"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds input generation only: structured element lattices, the
analytic curving map and its derivative, a manufactured field, the lattice
local-to-global numbering, and seeded random draws.  It contains no
quadrature, basis or operator arithmetic: every caller passes in the 1-D
reference points at which the map is to be evaluated, so the oracle and the
GPU path each use their own quadrature tables.

Conventions (shared data formats, not method arithmetic):
  * element index e = ex + Nx*(ey + Ny*ez)  (x fastest);
  * 1-D reference points xi in [-1, 1]; tensor point index
    q = i + Q*(j + Q*l)  (direction 1 fastest);
  * local mode index m = p + n*(q + n*r), n = P + 1 (direction 1 fastest),
    with mode 0 the left vertex mode and mode P the right vertex mode of the
    1-D modified basis (the order in which the paper's modified basis
    display in section 2.1 lists them);
  * Jacobian array J[e, c, a, q] = d x_c / d xi_a at point q.

Seeds follow seed = 1000 * config_index + k with k = 0 coefficients,
1 point values, 2 lambda, 3 kappa, 4 polynomial-order draws, 5 solve sizes,
6 finite-difference directions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

WARP_AMPLITUDE = 0.05

# The five workloads: sizes and shapes of the paper's tensor-product element
# groupings (section 3.3) at the scales this library is measured on.
CONFIGS = {
    0: dict(name="quad2d_8x8_P4", dim=2, shape=(8, 8), P=4, Q=6, warp=0.0, lam=1.0),
    1: dict(name="hex3d_32c_P6_curved", dim=3, shape=(32, 32, 32), P=6, Q=8,
            warp=WARP_AMPLITUDE, lam=1.0),
    2: dict(name="hex3d_24c_cg", dim=3, shape=(24, 24, 24), P=(4, 6, 8),
            warp=WARP_AMPLITUDE, lam=1.0),
    3: dict(name="batch_varp20000_and_256solves", dim=3, varp_shape=(20, 20, 50),
            varp_P=(2, 10), nsolves=256, solve_P=5, solve_sizes=(64, 4096),
            warp=WARP_AMPLITUDE, lam=1.0),
    4: dict(name="grad_16c_P6", dim=3, shape=(16, 16, 16), P=6, Q=8,
            warp=WARP_AMPLITUDE, coef_range=(0.5, 2.0)),
}


def seed(config_index: int, k: int) -> int:
    return 1000 * int(config_index) + int(k)


def uniform(seed_: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. U[lo, hi] FP64 draws from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed_).uniform(lo, hi, size=shape)


# ---------------------------------------------------------------- lattices

@dataclass(frozen=True)
class Lattice:
    shape: tuple          # elements per direction (Nx, Ny[, Nz])
    h: np.ndarray         # element edge lengths per direction
    origins: np.ndarray   # (E, d) lower corner of each element

    @property
    def dim(self) -> int:
        return len(self.shape)

    @property
    def nelem(self) -> int:
        return int(np.prod(self.shape))


def lattice(shape, lengths=None) -> Lattice:
    """Structured lattice of shape[0] x shape[1] (x shape[2]) boxes on
    [0, L_0] x [0, L_1] (x [0, L_2]), element index x-fastest."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    lengths = np.ones(d) if lengths is None else np.asarray(lengths, float)
    h = lengths / np.asarray(shape, float)
    idx = np.indices(shape[::-1]).reshape(d, -1)[::-1]   # idx[0] fastest
    origins = (idx.T * h).astype(np.float64)
    return Lattice(shape, h, origins)


def lattice_points(xi: np.ndarray, lat: Lattice) -> np.ndarray:
    """Undeformed lattice coordinates X[e, c, q] of the tensor points built
    from the 1-D reference points xi (affine map X = X_e0 + (xi+1)/2 * h)."""
    xi = np.asarray(xi, np.float64)
    Q = xi.size
    d = lat.dim
    t = (xi + 1.0) / 2.0
    grids = np.meshgrid(*([t] * d), indexing="ij")        # grids[a][i0, i1, ...]
    # point index q = i + Q*(j + Q*l): direction 1 fastest -> reverse axes
    local = np.stack([g.transpose(tuple(range(d))[::-1]).reshape(-1) for g in grids])
    X = lat.origins[:, :, None] + lat.h[None, :, None] * local[None, :, :]
    return X


# ---------------------------------------------------------- curving map

def _s(t):
    return np.sin(2.0 * math.pi * t)


def _ds(t):
    return 2.0 * math.pi * np.cos(2.0 * math.pi * t)


def warp(X: np.ndarray, amp: float = WARP_AMPLITUDE) -> np.ndarray:
    """Cyclic curving map of the unit cube (3-D) or square (2-D):
    x = X + a s(Y) s(Z), y = Y + a s(Z) s(X), z = Z + a s(X) s(Y),
    s(t) = sin(2 pi t).  X has the coordinate on axis -2: (..., d, npts)."""
    X = np.asarray(X, np.float64)
    d = X.shape[-2]
    if d == 2:
        x, y = X[..., 0, :], X[..., 1, :]
        return np.stack([x + amp * _s(y), y + amp * _s(x)], axis=-2)
    x, y, z = X[..., 0, :], X[..., 1, :], X[..., 2, :]
    return np.stack([x + amp * _s(y) * _s(z),
                     y + amp * _s(z) * _s(x),
                     z + amp * _s(x) * _s(y)], axis=-2)


def warp_jacobian(X: np.ndarray, amp: float = WARP_AMPLITUDE) -> np.ndarray:
    """d x_c / d X_a of `warp`, shape (..., d, d, npts) indexed [c, a]."""
    X = np.asarray(X, np.float64)
    d = X.shape[-2]
    one = np.ones_like(X[..., 0, :])
    if d == 2:
        x, y = X[..., 0, :], X[..., 1, :]
        rows = [[one, amp * _ds(y)], [amp * _ds(x), one]]
    else:
        x, y, z = X[..., 0, :], X[..., 1, :], X[..., 2, :]
        rows = [[one, amp * _ds(y) * _s(z), amp * _s(y) * _ds(z)],
                [amp * _s(z) * _ds(x), one, amp * _ds(z) * _s(x)],
                [amp * _ds(x) * _s(y), amp * _s(x) * _ds(y), one]]
    return np.stack([np.stack(r, axis=-2) for r in rows], axis=-3)


def element_jacobians(xi: np.ndarray, lat: Lattice, amp: float) -> np.ndarray:
    """J[e, c, a, q] = d x_c / d xi_a at the tensor points of xi for the
    composition (reference -> lattice box -> curving map).  The lattice step
    is affine, d X_a / d xi_a = h_a / 2, so J = (d x / d X) diag(h / 2)."""
    X = lattice_points(xi, lat)
    if amp == 0.0:
        d = lat.dim
        J = np.zeros((X.shape[0], d, d, X.shape[-1]))
        for a in range(d):
            J[:, a, a, :] = lat.h[a] / 2.0
        return J
    dxdX = warp_jacobian(X, amp)
    return dxdX * (lat.h[None, None, :, None] / 2.0)


# ---------------------------------------------------- manufactured field

def manufactured_sine(X: np.ndarray):
    """U = prod_c sin(pi X_c) on the undeformed lattice coordinates and its
    gradient dU/dX_c; X is (..., d, npts).  U vanishes on the boundary of the
    unit box."""
    X = np.asarray(X, np.float64)
    d = X.shape[-2]
    s = np.sin(math.pi * X)
    c = math.pi * np.cos(math.pi * X)
    U = np.prod(s, axis=-2)
    grads = []
    for a in range(d):
        g = c[..., a, :].copy()
        for b in range(d):
            if b != a:
                g = g * s[..., b, :]
        grads.append(g)
    return U, np.stack(grads, axis=-2)


def manufactured_ref_gradient(xi: np.ndarray, lat: Lattice):
    """U and its reference-coordinate gradient dU/dxi_a = (h_a/2) dU/dX_a at
    the tensor points of xi in every element: (E, Q^d) and (E, d, Q^d)."""
    X = lattice_points(xi, lat)
    U, dU = manufactured_sine(X)
    return U, dU * (lat.h[None, :, None] / 2.0)


# ------------------------------------------------ lattice C0 numbering

def lattice_l2g(shape, P: int, interior_last: bool = False):
    """Local-to-global map of a conforming structured lattice at uniform
    order P with the modified-basis mode order (vertex modes at 0 and P).

    Global index of local mode (p, q, r) of element (ex, ey, ez):
      gx = ex*P + p, gy = ey*P + q, gz = ez*P + r,
      g = gx + Gx*(gy + Gy*gz),  G_c = N_c*P + 1.
    Right vertex mode P of element e coincides with left vertex mode 0 of
    element e+1; bubble modes interior to an element edge are shared along
    that edge in the other directions.  With interior_last, the same global
    functions are renumbered: DOFs on element boundaries first (in the order
    above), then each element's interior modes as one contiguous block, in
    element order (the boundary-interior ordering).  Returns (l2g[E, n^d]
    int32, nglobal, dirichlet[nglobal] uint8) with Dirichlet DOFs on the
    lattice boundary.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    n = P + 1
    G = [s * P + 1 for s in shape]
    eidx = np.indices(shape[::-1]).reshape(d, -1)[::-1]           # (d, E)
    midx = np.indices((n,) * d).reshape(d, -1)[::-1]             # (d, n^d)
    gc = eidx[:, :, None] * P + midx[:, None, :]                 # (d, E, n^d)
    g = gc[d - 1]
    for c in range(d - 2, -1, -1):
        g = gc[c] + G[c] * g
    nglobal = int(np.prod(G))
    gall = np.indices(G[::-1]).reshape(d, -1)[::-1]
    dir_mask = np.zeros(nglobal, np.uint8)
    for c in range(d):
        dir_mask |= ((gall[c] == 0) | (gall[c] == G[c] - 1)).astype(np.uint8)
    if interior_last:
        inner = np.all((midx > 0) & (midx < P), axis=0)             # (n^d,)
        is_int = np.zeros(nglobal, bool)
        is_int[g[:, inner].ravel()] = True
        bnd = np.flatnonzero(~is_int)
        new = np.empty(nglobal, np.int64)
        new[bnd] = np.arange(bnd.size)
        new[g[:, inner].ravel()] = bnd.size + np.arange(int(inner.sum()) * g.shape[0])
        dm = np.empty_like(dir_mask)
        dm[new] = dir_mask
        return new[g].astype(np.int32), nglobal, dm
    return g.astype(np.int32), nglobal, dir_mask


def varp_lattice_l2g(shape, orders):
    """Conforming C0 map of a structured lattice whose elements carry their
    own order P_e (per-element isotropic), by the minimum rule: a bubble mode
    on a face or edge is a global DOF only up to the lowest order among the
    elements sharing that face or edge; higher modes there are constrained
    to zero.  The modified basis is hierarchical (bubble p is the same
    function whatever P), so the kept face/edge modes coincide between
    neighbours.

    Elements are returned grouped by ascending order (the element order of a
    mixed-order space): `perm[k]` is the lattice index of space element k.
    Local modes are numbered p fastest as for uniform order.  Constrained
    modes map to one extra global DOF (the last) that is flagged Dirichlet,
    so they read as zero and receive nothing.  Global DOFs are numbered in
    lattice order of their position on the P_max grid; Dirichlet = lattice
    boundary.  Returns (perm, [l2g of each space element], nglobal,
    dirichlet uint8)."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    E = int(np.prod(shape))
    orders = np.asarray(orders, np.int64).reshape(E)
    Pm = int(orders.max())
    G = [s * Pm + 1 for s in shape]
    eidx = np.indices(shape[::-1]).reshape(d, -1)[::-1].T          # (E, d)
    strides = np.cumprod([1] + list(shape[:-1]))
    keys, sharedmin = [], {}
    for e in range(E):
        P = int(orders[e])
        m = np.indices((P + 1,) * d).reshape(d, -1)[::-1]            # (d, n^d)
        side = np.where(m == 0, 0, np.where(m == P, 2, 1))           # L, B, R
        pat = (side * (3 ** np.arange(d))[:, None]).sum(axis=0)
        ok = np.ones(m.shape[1], bool)
        g = np.zeros(m.shape[1], np.int64)
        for c in range(d - 1, -1, -1):
            gc = eidx[e, c] * Pm + np.where(side[c] == 0, 0, np.where(side[c] == 2, Pm, m[c]))
            g = gc + G[c] * g
        for s in np.unique(pat):
            sd = [(s // 3 ** c) % 3 for c in range(d)]
            if all(x == 1 for x in sd) or all(x != 1 for x in sd):
                continue                     # interior modes, or a vertex: nothing to limit
            pmin = P
            offs = [[0] if x == 1 else ([0, -1] if x == 0 else [0, 1]) for x in sd]
            for dl in np.array(np.meshgrid(*offs, indexing="ij")).reshape(d, -1).T:
                nb = eidx[e] + dl
                if np.all(nb >= 0) and np.all(nb < np.asarray(shape)):
                    pmin = min(pmin, int(orders[int(nb @ strides)]))
            sel = pat == s
            for c in range(d):
                if sd[c] == 1:
                    ok[sel] &= m[c][sel] <= pmin - 1
        g[~ok] = -1
        keys.append(g)
    used = np.unique(np.concatenate([k[k >= 0] for k in keys]))
    nglobal = used.size + 1                                        # + the zero DOF
    rank = {int(v): i for i, v in enumerate(used)}
    zero = nglobal - 1
    perm = np.argsort(orders, kind="stable")
    l2g = []
    for e in perm:
        k = keys[e]
        l2g.append(np.array([rank[int(v)] if v >= 0 else zero for v in k], np.int32))
    gl = used.copy()
    dirichlet = np.zeros(nglobal, np.uint8)
    for c in range(d):
        gc = gl % G[c]
        gl = gl // G[c]
        dirichlet[:-1] |= ((gc == 0) | (gc == G[c] - 1)).astype(np.uint8)
    dirichlet[zero] = 1
    return perm, l2g, nglobal, dirichlet


def tri_lattice_vertices(n: int):
    """Vertex ids (lattice point i + (n+1) j) of the triangle mesh of the unit
    square: square k = i + n j gives element 2k = (v00, v10, v11) and element
    2k+1 = (v00, v11, v01), both counter-clockwise.  Returns (E, 3) int64."""
    k = np.arange(n * n)
    i, j = k % n, k // n
    v00, v10 = i + (n + 1) * j, i + 1 + (n + 1) * j
    v11, v01 = i + 1 + (n + 1) * (j + 1), i + (n + 1) * (j + 1)
    out = np.empty((2 * n * n, 3), np.int64)
    out[0::2] = np.stack([v00, v10, v11], axis=1)
    out[1::2] = np.stack([v00, v11, v01], axis=1)
    return out


def tri_rotations(seed_: int, nelem: int) -> np.ndarray:
    """Seeded cyclic rotation r in {0, 1, 2} of each triangle's local vertex
    order: local (A, B, C) = (v_r, v_{r+1}, v_{r+2}) (orientation kept)."""
    return np.random.default_rng(seed_).integers(0, 3, size=nelem)


def tri_lattice_jacobians(n: int, e1, e2, amp: float = 0.05, rot=None):
    """Jacobians of the triangle mesh of the unit square (tri_lattice_vertices),
    composed with the curving map x' = x + a s(x) s(y), y' = y + a/2 s(x) s(y),
    s(t) = sin(2 pi t).  With local vertices (A, B, C) (rotated by rot, if
    given), the affine reference map is x = A (-(xi_1 + xi_2)/2)
    + B (1 + xi_1)/2 + C (1 + xi_2)/2 evaluated at the collapsed points
    (eta_1, eta_2) (xi_1 = (1 + eta_1)(1 - eta_2)/2 - 1, xi_2 = eta_2).
    Returns J[E, c, a, q] = d x'_c / d xi_a with q = i + Q j over (e1, e2)."""
    e1 = np.asarray(e1, np.float64)
    e2 = np.asarray(e2, np.float64)
    E1 = np.tile(e1, e2.size)
    E2 = np.repeat(e2, e1.size)
    x1 = (1 + E1) * (1 - E2) / 2 - 1
    x2 = E2
    h = 1.0 / n
    k = np.arange(n * n)
    V0s = np.stack([(k % n) * h, (k // n) * h], axis=1)                    # (n^2, 2)
    out = np.empty((2 * n * n, 2, 2, x1.size))
    for t, (d1, d2) in enumerate((([h, 0], [h, h]), ([h, h], [0, h]))):
        corners = np.stack([V0s, V0s + d1, V0s + d2], axis=1)               # (n^2, 3, 2)
        if rot is not None:
            r = np.asarray(rot)[t::2]
            idx = (r[:, None] + np.arange(3)[None, :]) % 3
            corners = np.take_along_axis(corners, idx[:, :, None], axis=1)
        V0, V1, V2 = corners[:, 0], corners[:, 1], corners[:, 2]
        A = np.stack([(V1 - V0) / 2, (V2 - V0) / 2], axis=2)                # (n^2, c, a)
        X = (V0[:, :, None] * (-(x1 + x2) / 2) + V1[:, :, None] * (1 + x1) / 2
             + V2[:, :, None] * (1 + x2) / 2)                               # (n^2, 2, nq)
        sx, sy = np.sin(2 * np.pi * X[:, 0]), np.sin(2 * np.pi * X[:, 1])
        cx, cy = 2 * np.pi * np.cos(2 * np.pi * X[:, 0]), 2 * np.pi * np.cos(2 * np.pi * X[:, 1])
        Wm = np.empty((n * n, 2, 2, x1.size))                              # d x' / d x
        Wm[:, 0, 0] = 1 + amp * cx * sy
        Wm[:, 0, 1] = amp * sx * cy
        Wm[:, 1, 0] = amp / 2 * cx * sy
        Wm[:, 1, 1] = 1 + amp / 2 * sx * cy
        out[t::2] = np.einsum("ecbq,eba->ecaq", Wm, A)
    return out


def tri_lattice_l2g(n: int, P: int, rot=None):
    """C0 numbering of the triangle mesh (tri_lattice_vertices) for the
    collapsed modal basis in its mode order (p = 0: q = 0 vertex A, q = 1..P-1
    edge AC, q = P vertex C; 0 < p < P: q = 0 edge AB, q >= 1 interior; p = P:
    q = 0 vertex B, q >= 1 edge BC), with orientation signs.  Global DOFs:
    mesh vertices, then P-1 per mesh edge, then the interior modes of each
    triangle.  A mesh edge runs from its lower to its higher vertex id; a
    triangle traversing it the other way sees its k-th edge bubble (k =
    1..P-1) as (-1)^(k-1) times the global one, the parity of the 1-D
    bubbles (1-x)(1+x)/4 P^{1,1}_{k-1}(x).  Dirichlet: vertices and edges on
    the boundary of the unit square.
    Returns (l2g (E, nm) int32, sign (E, nm) int8, nglobal, dirichlet uint8)."""
    V = tri_lattice_vertices(n)
    E = V.shape[0]
    if rot is not None:
        r = np.asarray(rot)
        V = np.take_along_axis(V, (r[:, None] + np.arange(3)[None, :]) % 3, axis=1)
    nv = (n + 1) ** 2
    nb = max(P - 1, 0)
    nint = max((P - 1) * (P - 2) // 2, 0)
    edges = {}
    for a_, b_ in np.concatenate([V[:, [0, 1]], V[:, [0, 2]], V[:, [1, 2]]]):
        key = (min(a_, b_), max(a_, b_))
        if key not in edges:
            edges[key] = len(edges)
    ne = len(edges)
    nglobal = nv + ne * nb + E * nint
    modes = [(0, q) for q in range(P + 1)] + [(p, q) for p in range(1, P) for q in range(P - p)] \
        + [(P, q) for q in range(P)]
    l2g = np.empty((E, len(modes)), np.int64)
    sign = np.ones((E, len(modes)), np.int8)
    for e in range(E):
        A_, B_, C_ = V[e]
        def edge(a_, b_, k):
            g = nv + edges[(min(a_, b_), max(a_, b_))] * nb + (k - 1)
            return g, (1 if a_ < b_ or k % 2 == 1 else -1)
        it = 0
        for m, (p, q) in enumerate(modes):
            if p == 0 and q == 0:
                g, s = A_, 1
            elif p == 0 and q == P:
                g, s = C_, 1
            elif p == 0:
                g, s = edge(A_, C_, q)
            elif p == P and q == 0:
                g, s = B_, 1
            elif p == P:
                g, s = edge(B_, C_, q)
            elif q == 0:
                g, s = edge(A_, B_, p)
            else:
                g, s = nv + ne * nb + e * nint + it, 1
                it += 1
            l2g[e, m], sign[e, m] = g, s
    on_bd = lambda v: (v % (n + 1) == 0) | (v % (n + 1) == n) | (v // (n + 1) == 0) | (v // (n + 1) == n)
    dirichlet = np.zeros(nglobal, np.uint8)
    dirichlet[:nv][on_bd(np.arange(nv))] = 1
    for (a_, b_), k in edges.items():
        ia, ja, ib, jb = a_ % (n + 1), a_ // (n + 1), b_ % (n + 1), b_ // (n + 1)
        if (ia == ib and ia in (0, n)) or (ja == jb and ja in (0, n)):
            dirichlet[nv + k * nb: nv + (k + 1) * nb] = 1
    return l2g.astype(np.int32), sign, nglobal, dirichlet


def tet_lattice_vertices(n: int, sorted_ids: bool = False) -> np.ndarray:
    """Vertex coordinates of the tetrahedral mesh of the unit cube: an n^3
    lattice of cubes (cube index i + n (j + n k)), each split into the six
    tetrahedra of the path decomposition, v0 = corner, v1 = v0 + h e_a,
    v2 = v1 + h e_b, v3 = v0 + h (1, 1, 1) for the permutations (a, b, c)
    of the axes.  By default v1 and v2 are swapped for odd permutations so
    that every tetrahedron (A, B, C, D) = (v0, v1, v2, v3) is positively
    oriented; with sorted_ids the path order is kept, which is the order of
    the lattice vertex ids i + (n+1)(j + (n+1) k) (half the tetrahedra are
    then left-handed).  Returns (E, 4, 3), E = 6 n^3, element 6 cube +
    permutation index."""
    h = 1.0 / n
    c = np.arange(n ** 3)
    corner = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1) * h      # (n^3, 3)
    perms = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]   # 3 even, 3 odd
    eye = np.eye(3) * h
    out = np.empty((n ** 3, 6, 4, 3))
    for t, (a, b, _) in enumerate(perms):
        v0 = corner
        v1 = v0 + eye[a]
        v2 = v1 + eye[b]
        v3 = v0 + h
        if t >= 3 and not sorted_ids:
            v1, v2 = v2, v1
        out[:, t] = np.stack([v0, v1, v2, v3], axis=1)
    return out.reshape(-1, 4, 3)


def tet_lattice_jacobians(n: int, e1, e2, e3, amp: float = WARP_AMPLITUDE, elems=None,
                          sorted_ids: bool = False):
    """Jacobians of the tetrahedral mesh of the unit cube
    (tet_lattice_vertices), composed with the cyclic curving map `warp`.  With
    vertices (A, B, C, D), the affine reference map is x = A (-(1 + xi_1 +
    xi_2 + xi_3)/2) + B (1 + xi_1)/2 + C (1 + xi_2)/2 + D (1 + xi_3)/2, taken at
    the collapsed points (xi_3 = eta_3, xi_2 = (1 + eta_2)(1 - eta_3)/2 - 1,
    xi_1 = (1 + eta_1)(1 - eta_2)(1 - eta_3)/4 - 1) of the 1-D point sets
    (e1, e2, e3), q = i + len(e1) (j + len(e2) k).  elems: optional subset of
    element indices.  Returns J[E, c, a, q] = d x'_c / d xi_a."""
    e1, e2, e3 = (np.asarray(v, np.float64) for v in (e1, e2, e3))
    n1, n2 = e1.size, e2.size
    E1 = np.tile(e1, n2 * e3.size)
    E2 = np.tile(np.repeat(e2, n1), e3.size)
    E3 = np.repeat(e3, n1 * n2)
    x3 = E3
    x2 = (1 + E2) * (1 - E3) / 2 - 1
    x1 = (1 + E1) * (1 - E2) * (1 - E3) / 4 - 1
    V = tet_lattice_vertices(n, sorted_ids)
    if elems is not None:
        V = V[np.asarray(elems)]
    A = np.stack([(V[:, 1] - V[:, 0]) / 2, (V[:, 2] - V[:, 0]) / 2, (V[:, 3] - V[:, 0]) / 2], axis=2)
    if amp == 0.0:
        return np.broadcast_to(A[:, :, :, None], A.shape + (x1.size,)).copy()
    X = (V[:, 0, :, None] * (-(1 + x1 + x2 + x3) / 2) + V[:, 1, :, None] * ((1 + x1) / 2)
         + V[:, 2, :, None] * ((1 + x2) / 2) + V[:, 3, :, None] * ((1 + x3) / 2))     # (E, 3, nq)
    Wm = warp_jacobian(X, amp)                                                        # (E, c, b, nq)
    return np.einsum("ecbq,eba->ecaq", Wm, A)


def tet_lattice_l2g(n: int, P: int):
    """C0 numbering of the tetrahedral mesh with sorted vertex orders
    (tet_lattice_vertices(n, sorted_ids=True)), for the tetrahedron modes
    (triangle mode t = (p, q) of the order-P triangle in its mode order, r
    fastest, the top vertex last).  With every element's vertices in
    increasing global id, each edge is traversed from its lower to its
    higher vertex and each face has its highest vertex as the collapsed one,
    in every element that shares it, so no signs are needed.  Global DOFs:
    lattice vertices; P-1 bubbles per mesh edge (k = 1..P-1); the interior
    modes (i, j), i, j >= 1, i + j <= P-1, of each mesh face; then the
    interior modes of each element.  Local modes by the tetrahedron's
    entities: vertices A = ((0,0), 0), B = ((P,0), 0), C = ((0,P), 0), D (top);
    edges AB ((p,0), 0), AC ((0,q), 0), BC ((P,q), 0) with bubble p or q, AD
    ((0,0), r), BD ((P,0), r), CD ((0,P), r) with bubble r; faces ABC
    ((p,q), 0) -> (p, q), ABD ((p,0), r) -> (p, r), ACD ((0,q), r) -> (q, r),
    BCD ((P,q), r) -> (q, r); interior ((p,q), r >= 1) with p, q >= 1.
    Dirichlet: vertices, edges and faces on the boundary of the unit cube.
    Returns (l2g (E, nm) int32, nglobal, dirichlet uint8)."""
    V = tet_lattice_vertices(n, sorted_ids=True)
    E = V.shape[0]
    ids = np.rint(V[..., 0] * n).astype(np.int64) + (n + 1) * (
        np.rint(V[..., 1] * n).astype(np.int64) + (n + 1) * np.rint(V[..., 2] * n).astype(np.int64))
    assert np.all(np.diff(ids, axis=1) > 0)
    nv = (n + 1) ** 3
    nb = max(P - 1, 0)
    fmodes = [(i, j) for i in range(1, P) for j in range(1, P - i)]
    nf = len(fmodes)
    fidx = {ij: k for k, ij in enumerate(fmodes)}
    tri = [(0, q) for q in range(P + 1)] + [(p, q) for p in range(1, P) for q in range(P - p)] \
        + [(P, q) for q in range(P)]

    def deg(p, q):
        if (p in (0, P) and q == 0) or (p == 0 and q == P):
            return 1
        if p in (0, P):
            return q + 1
        return p + 1 if q == 0 else p + q + 1
    modes = [((p, q), r) for (p, q) in tri for r in range(P - deg(p, q) + 1)] + [None]
    ninner = sum(1 for mm in modes if mm and mm[0][0] not in (0, P) and mm[0][1] >= 1 and mm[1] >= 1)
    edges, faces = {}, {}
    for e in range(E):
        a, b, c, d = ids[e]
        for pair in ((a, b), (a, c), (b, c), (a, d), (b, d), (c, d)):
            edges.setdefault(pair, len(edges))
        for tri3 in ((a, b, c), (a, b, d), (a, c, d), (b, c, d)):
            faces.setdefault(tri3, len(faces))
    ne, nfc = len(edges), len(faces)
    e0, f0 = nv, nv + ne * nb
    i0 = f0 + nfc * nf
    nglobal = i0 + E * ninner
    l2g = np.empty((E, len(modes)), np.int64)
    for e in range(E):
        A_, B_, C_, D_ = ids[e]
        it = 0
        for mi, mm in enumerate(modes):
            if mm is None:
                g = D_
            else:
                (p, q), r = mm
                vert = {(0, 0): A_, (P, 0): B_, (0, P): C_}
                if (p, q) in vert and r == 0:
                    g = vert[(p, q)]
                elif (p, q) in vert:                       # rising edges AD, BD, CD
                    g = e0 + edges[(vert[(p, q)], D_)] * nb + r - 1
                elif r == 0 and q == 0:                     # edge AB
                    g = e0 + edges[(A_, B_)] * nb + p - 1
                elif r == 0 and p == 0:                     # edge AC
                    g = e0 + edges[(A_, C_)] * nb + q - 1
                elif r == 0 and p == P:                     # edge BC
                    g = e0 + edges[(B_, C_)] * nb + q - 1
                elif r == 0:                                # face ABC
                    g = f0 + faces[(A_, B_, C_)] * nf + fidx[(p, q)]
                elif q == 0:                                # face ABD
                    g = f0 + faces[(A_, B_, D_)] * nf + fidx[(p, r)]
                elif p == 0:                                # face ACD
                    g = f0 + faces[(A_, C_, D_)] * nf + fidx[(q, r)]
                elif p == P:                                # face BCD
                    g = f0 + faces[(B_, C_, D_)] * nf + fidx[(q, r)]
                else:                                       # interior
                    g = i0 + e * ninner + it
                    it += 1
            l2g[e, mi] = g
    coord = lambda v: np.stack([v % (n + 1), (v // (n + 1)) % (n + 1), v // (n + 1) ** 2], axis=-1)
    on = lambda v: (coord(v) == 0) | (coord(v) == n)                  # (…, 3) per axis
    dm = np.zeros(nglobal, np.uint8)
    dm[:nv][np.any(on(np.arange(nv)), axis=1)] = 1
    for (a, b), k in edges.items():
        if np.any(on(a) & on(b) & (coord(a) == coord(b))):
            dm[e0 + k * nb: e0 + (k + 1) * nb] = 1
    for (a, b, c), k in faces.items():
        if np.any(on(a) & on(b) & on(c) & (coord(a) == coord(b)) & (coord(b) == coord(c))):
            dm[f0 + k * nf: f0 + (k + 1) * nf] = 1
    return l2g.astype(np.int32), nglobal, dm


def prism_lattice_vertices(n: int, rot=None) -> np.ndarray:
    """(x, y) of the local triangle vertices (A, B, C) of the prismatic mesh's
    2 n^2 columns: the triangles of tri_lattice_vertices, each rotated by
    rot (one cyclic rotation per column, shared by its n layers), if given.
    Returns (2 n^2, 3, 2)."""
    V = tri_lattice_vertices(n)
    if rot is not None:
        r = np.asarray(rot)
        V = np.take_along_axis(V, (r[:, None] + np.arange(3)[None, :]) % 3, axis=1)
    return np.stack([V % (n + 1), V // (n + 1)], axis=-1) / n


def prism_lattice_jacobians(n: int, e1, e2, x3, amp: float = WARP_AMPLITUDE, elems=None, rot=None):
    """Jacobians of the prismatic mesh of the unit cube: the triangle mesh of
    the unit square (tri_lattice_vertices) extruded into n layers, prism
    e = layer * 2 n^2 + triangle, curved by the cyclic warp.  With the
    triangle's vertices (A, B, C) (rotated by rot per column, if given) and
    the layer [z0, z0 + h], the affine
    reference map is (x, y) = A (-(xi_1 + xi_2)/2) + B (1 + xi_1)/2
    + C (1 + xi_2)/2, z = z0 + h (1 + xi_3)/2, taken at the points of the 1-D
    sets (e1 = eta_1, e2 = eta_2 = xi_2, x3 = xi_3), q = i + len(e1) (j +
    len(e2) k), xi_1 = (1 + eta_1)(1 - eta_2)/2 - 1.  Returns J[E, c, a, q]."""
    e1, e2, x3 = (np.asarray(v, np.float64) for v in (e1, e2, x3))
    n1, n2 = e1.size, e2.size
    E1 = np.tile(e1, n2 * x3.size)
    E2 = np.tile(np.repeat(e2, n1), x3.size)
    X3 = np.repeat(x3, n1 * n2)
    xi1 = (1 + E1) * (1 - E2) / 2 - 1
    xi2 = E2
    h = 1.0 / n
    xy = prism_lattice_vertices(n, rot)                                # (2 n^2, 3, 2)
    nt = xy.shape[0]
    e = np.arange(n * nt) if elems is None else np.asarray(elems)
    tri, layer = e % nt, e // nt
    T = xy[tri]
    A = np.zeros((e.size, 3, 3))
    A[:, :2, 0] = (T[:, 1] - T[:, 0]) / 2
    A[:, :2, 1] = (T[:, 2] - T[:, 0]) / 2
    A[:, 2, 2] = h / 2
    if amp == 0.0:
        return np.broadcast_to(A[:, :, :, None], A.shape + (xi1.size,)).copy()
    XY = (T[:, 0, :, None] * (-(xi1 + xi2) / 2) + T[:, 1, :, None] * ((1 + xi1) / 2)
          + T[:, 2, :, None] * ((1 + xi2) / 2))                          # (E, 2, nq)
    Z = layer[:, None] * h + h * (1 + X3[None, :]) / 2
    X = np.concatenate([XY, Z[:, None, :]], axis=1)
    Wm = warp_jacobian(X, amp)
    return np.einsum("ecbq,eba->ecaq", Wm, A)


def prism_lattice_l2g(n: int, P: int, rot=None):
    """C0 numbering of the prismatic mesh (prism_lattice_jacobians, the same
    rot), for the prism modes (triangle mode t in its mode order, r fastest):
    the signed triangle numbering of tri_lattice_l2g(n, P, rot) times the
    1-D numbering of each column, layer * P + r (r = 0 bottom vertex, P top
    vertex, bubbles between), so global = g_t + ng_t (layer P + r) with the
    triangle mode's sign.  Vertical faces are a triangle edge times the
    column, so their orientation is the edge's; horizontal faces are whole
    triangles of one column and match exactly.  Dirichlet: the triangle
    numbering's boundary DOFs in every layer, and the bottom and top planes.
    Returns (l2g (E, nm) int32, sign (E, nm) int8, nglobal, dirichlet uint8)."""
    l2, s2, ng2, dm2 = tri_lattice_l2g(n, P, rot)
    nt = l2.shape[0]
    nz = n * P + 1
    layer = np.repeat(np.arange(n), nt)
    tri = np.tile(np.arange(nt), n)
    r = np.arange(P + 1)
    g = l2[tri][:, :, None].astype(np.int64) + ng2 * (layer[:, None, None] * P + r[None, None, :])
    l2g = g.reshape(n * nt, -1)
    sign = np.repeat(s2[tri], P + 1, axis=1)
    zbd = np.zeros(nz, bool)
    zbd[[0, nz - 1]] = True
    dm = (dm2[None, :].astype(bool) | zbd[:, None]).astype(np.uint8).ravel()
    return l2g.astype(np.int32), sign, ng2 * nz, dm


def pyr_lattice_jacobians(n: int, e1, e2, e3, amp: float = WARP_AMPLITUDE, elems=None):
    """Jacobians of the pyramidal mesh of the unit cube: an n^3 lattice of
    cubes, each split into six pyramids with the cube's centre as apex and
    one face as base (element 6 cube + face, faces -x, +x, -y, +y, -z, +z),
    curved by the cyclic warp.  With base corner a, its neighbours b and d
    (ordered so the map is positively oriented) and apex e, the reference
    map is x = a + (b - a)(1 + xi_1)/2 + (d - a)(1 + xi_2)/2 + (e - a)(1 + xi_3)/2,
    taken at the collapsed points (xi_1 = (1 + eta_1)(1 - eta_3)/2 - 1, xi_2
    likewise with eta_2, xi_3 = eta_3) of the 1-D sets (e1, e2, e3),
    q = i + len(e1) (j + len(e2) k).  Returns J[E, c, a, q]."""
    e1, e2, e3 = (np.asarray(v, np.float64) for v in (e1, e2, e3))
    n1, n2 = e1.size, e2.size
    E1 = np.tile(e1, n2 * e3.size)
    E2 = np.tile(np.repeat(e2, n1), e3.size)
    E3 = np.repeat(e3, n1 * n2)
    x1 = (1 + E1) * (1 - E3) / 2 - 1
    x2 = (1 + E2) * (1 - E3) / 2 - 1
    x3 = E3
    V = pyr_lattice_vertices(n)
    if elems is not None:
        V = V[np.asarray(elems)]
    A = np.stack([(V[:, 1] - V[:, 0]) / 2, (V[:, 2] - V[:, 0]) / 2, (V[:, 3] - V[:, 0]) / 2], axis=2)
    if amp == 0.0:
        return np.broadcast_to(A[:, :, :, None], A.shape + (x1.size,)).copy()
    X = (V[:, 0, :, None] + A[:, :, 0, None] * (1 + x1) + A[:, :, 1, None] * (1 + x2)
         + A[:, :, 2, None] * (1 + x3))
    Wm = warp_jacobian(X, amp)
    return np.einsum("ecbq,eba->ecaq", Wm, A)


def pyr_lattice_vertices(n: int) -> np.ndarray:
    """Vertices (a, b, d, e) of the pyramidal mesh's elements (6 per cube,
    element 6 cube + face, faces -x, +x, -y, +y, -z, +z): a the face's lowest
    corner, b and d its neighbours along the face's two axes (swapped where
    needed so the map is positively oriented), e the cube's centre; the base's
    fourth corner is c = b + d - a.  Returns (E, 4, 3)."""
    h = 1.0 / n
    c = np.arange(n ** 3)
    corner = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1) * h
    faces = []
    for ax in range(3):
        u, v = [d for d in range(3) if d != ax]
        for side in (0, 1):
            a = np.zeros(3)
            a[ax] = side * h
            b, d = a.copy(), a.copy()
            b[u] += h
            d[v] += h
            eap = np.full(3, h / 2)
            if np.linalg.det(np.stack([b - a, d - a, eap - a], axis=1)) < 0:
                b, d = d, b
            faces.append((a, b, d, eap))
    V = np.stack([np.stack([corner + f[k] for k in range(4)], axis=1) for f in faces], axis=1)
    return V.reshape(-1, 4, 3)


def pyr_lattice_l2g(n: int, P: int):
    """C0 numbering of the pyramidal mesh (pyr_lattice_vertices) for the
    pyramid modes (base mode (p, q), p slow, r fastest, the apex last).  Every
    base edge runs along + x, + y or + z from the base's lowest corner a, and
    every rising edge from a cube corner to the cube's centre, in each element
    that holds it, so no signs are needed: a shared triangular face (centre
    and a cube edge) has the same edge direction and collapsed apex in both
    pyramids, and a shared base (a cube face between two cubes) is the same
    tensor face, seen with its two axes swapped where b and d were swapped.
    Global DOFs: lattice corners, cube centres; P-1 bubbles per edge (cube
    edges, corner-centre edges); (P-1)^2 per cube face, indexed (i, j) along
    its lower and higher axis; (P-1)(P-2)/2 per triangular face, (k, r) with
    k the edge bubble; then each element's interior modes ((p, q) bubbles,
    r >= 1).  Dirichlet: corners, cube edges and cube faces on the boundary
    of the unit cube.  Returns (l2g (E, nm) int32, nglobal, dirichlet
    uint8)."""
    V = pyr_lattice_vertices(n)
    E = V.shape[0]
    K = np.rint(V * 2 * n).astype(np.int64)                            # corners even, centres odd
    nc = (n + 1) ** 3

    def vid(k):
        if k[0] % 2 == 0:
            i, j, l = k // 2
            return int(i + (n + 1) * (j + (n + 1) * l))
        i, j, l = (k - 1) // 2
        return int(nc + i + n * (j + n * l))
    deg = lambda p: 1 if p in (0, P) else p + 1
    modes = [(p, q, r) for p in range(P + 1) for q in range(P + 1)
             for r in range(P - max(deg(p), deg(q)) + 1)] + [None]
    nb = max(P - 1, 0)
    nq = nb * nb
    tmodes = [(k, r) for k in range(1, P) for r in range(1, P - k)]
    tidx = {kr: i for i, kr in enumerate(tmodes)}
    nt = len(tmodes)
    ninner = sum(1 for mm in modes if mm and 0 < mm[0] < P and 0 < mm[1] < P and mm[2] >= 1)
    edges, qfaces, tfaces = {}, {}, {}
    ent = []
    for e in range(E):
        a, b, d, ap = (vid(K[e, k]) for k in range(4))
        c = vid(K[e, 1] + K[e, 2] - K[e, 0])
        ax_b = int(np.flatnonzero(K[e, 1] != K[e, 0])[0])
        ax_d = int(np.flatnonzero(K[e, 2] != K[e, 0])[0])
        for pr in ((a, b), (a, d), (b, c), (d, c), (a, ap), (b, ap), (d, ap), (c, ap)):
            edges.setdefault(pr, len(edges))
        qk = tuple(sorted((a, b, c, d)))
        qfaces.setdefault(qk, len(qfaces))
        for pr in ((a, b), (a, d), (b, c), (d, c)):
            tfaces.setdefault(pr + (ap,), len(tfaces))
        ent.append((a, b, c, d, ap, ax_b < ax_d, qk))
    ne, nqf, ntf = len(edges), len(qfaces), len(tfaces)
    nv = nc + n ** 3
    e0 = nv
    q0 = e0 + ne * nb
    t0 = q0 + nqf * nq
    i0 = t0 + ntf * nt
    nglobal = i0 + E * ninner
    l2g = np.empty((E, len(modes)), np.int64)
    for e in range(E):
        a, b, c, d, ap, straight, qk = ent[e]
        vert = {(0, 0): a, (P, 0): b, (0, P): d, (P, P): c}
        it = 0
        for m, mm in enumerate(modes):
            if mm is None:
                g = ap
            else:
                p, q, r = mm
                pv, qv = p in (0, P), q in (0, P)
                if pv and qv:                                   # corner, or rising edge
                    g = vert[(p, q)] if r == 0 else e0 + edges[(vert[(p, q)], ap)] * nb + r - 1
                elif r == 0 and qv:                             # edge a-b (q = 0) or d-c
                    g = e0 + edges[(vert[(0, q)], vert[(P, q)])] * nb + p - 1
                elif r == 0 and pv:                             # edge a-d (p = 0) or b-c
                    g = e0 + edges[(vert[(p, 0)], vert[(p, P)])] * nb + q - 1
                elif r == 0:                                    # base face, axes (u, v)
                    i, j = (p, q) if straight else (q, p)
                    g = q0 + qfaces[qk] * nq + (i - 1) + nb * (j - 1)
                elif qv:                                        # triangle on edge a-b / d-c
                    g = t0 + tfaces[(vert[(0, q)], vert[(P, q)], ap)] * nt + tidx[(p, r)]
                elif pv:                                        # triangle on edge a-d / b-c
                    g = t0 + tfaces[(vert[(p, 0)], vert[(p, P)], ap)] * nt + tidx[(q, r)]
                else:
                    g = i0 + e * ninner + it
                    it += 1
            l2g[e, m] = g
    coord = lambda v: np.array([v % (n + 1), (v // (n + 1)) % (n + 1), v // (n + 1) ** 2])
    on_bd = lambda v: v < nc and bool(np.any((coord(v) == 0) | (coord(v) == n)))
    dm = np.zeros(nglobal, np.uint8)
    for v in range(nc):
        dm[v] = on_bd(v)
    same_plane = lambda vs: vs[0] < nc and all(v < nc for v in vs) and bool(np.any(
        np.all([(coord(v) == coord(vs[0])) & ((coord(v) == 0) | (coord(v) == n)) for v in vs], axis=0)))
    for (u, w), k in edges.items():
        if same_plane((u, w)):
            dm[e0 + k * nb: e0 + (k + 1) * nb] = 1
    for qk, k in qfaces.items():
        if same_plane(qk):
            dm[q0 + k * nq: q0 + (k + 1) * nq] = 1
    return l2g.astype(np.int32), nglobal, dm


# ----------------------------------------------------------- draws

def varp_orders(seed_: int, nelem: int, lo: int = 2, hi: int = 10) -> np.ndarray:
    """Per-element polynomial order drawn uniformly from {lo..hi}."""
    return np.random.default_rng(seed_).integers(lo, hi + 1, size=nelem)


def solve_boxes(seed_: int, nsolves: int, smin: int = 64, smax: int = 4096):
    """Independent solve sizes s ~ log-uniform[smin, smax] mapped to box
    lattices a x b x c with a = round(s^(1/3)), b = round(sqrt(s/a)),
    c = ceil(s/(a b)).  Returns a list of (a, b, c)."""
    rng = np.random.default_rng(seed_)
    s = np.exp(rng.uniform(math.log(smin), math.log(smax), size=nsolves))
    boxes = []
    for si in s:
        a = max(1, int(round(si ** (1.0 / 3.0))))
        b = max(1, int(round(math.sqrt(si / a))))
        c = max(1, int(math.ceil(si / (a * b))))
        boxes.append((a, b, c))
    return boxes


def dof_signs(seed_: int, l2g: np.ndarray, nglobal: int) -> np.ndarray:
    """A consistent orientation-sign array for a map: each global DOF draws
    sigma_g = +-1 with equal odds and every local mode referencing it gets
    sign sigma_g (the same global functions, some negated).  int8, shape of
    l2g."""
    sig = np.where(np.random.default_rng(seed_).random(int(nglobal)) < 0.5, -1, 1).astype(np.int8)
    return sig[np.asarray(l2g, np.int64)]
