"""Pins for the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, an
exact integral, an invariant, a textbook special case, a value printed in the
paper (Listing 1, section 3.5) or a brute-force/independent computation, chosen
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import MaskedOperator, pcg, jacobi_diagonal, direct_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ GLL

@pytest.mark.parametrize("Q", [3, 4, 6, 8, 10, 12])
def test_gll_exactness_degree(Q):
    """GLL with Q points integrates x^k exactly for k <= 2Q-3 and not 2Q-2."""
    x, w = oracle.gll(Q)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * Q - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13, k
    k = 2 * Q - 2
    assert abs(w @ x ** k - 2.0 / (k + 1)) > 1e-7


def test_gll_textbook_small_cases():
    """Closed forms: Q=3 -> (-1,0,1), (1/3,4/3,1/3); Q=4 -> +-1, +-1/sqrt(5),
    weights 1/6, 5/6."""
    x, w = oracle.gll(3)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = oracle.gll(4)
    s = 1 / math.sqrt(5)
    np.testing.assert_allclose(x, [-1, -s, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("Q", [5, 8, 11])
def test_gll_symmetry(Q):
    x, w = oracle.gll(Q)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    np.testing.assert_allclose(w, w[::-1], atol=1e-15)
    assert np.all(np.diff(x) > 0)


# ---------------------------------------------------------- modified basis

@pytest.mark.parametrize("P", [1, 2, 4, 6, 8, 10])
def test_basis_partition_and_bubbles(P):
    """phi_0 + phi_P = 1; bubbles vanish at both ends (section 2.1 display)."""
    x = np.linspace(-1, 1, 37)
    B, _ = oracle.modified_basis(P, x)
    np.testing.assert_allclose(B[:, 0] + B[:, P], 1.0, atol=1e-15)
    Bend, _ = oracle.modified_basis(P, np.array([-1.0, 1.0]))
    np.testing.assert_allclose(Bend[:, 1:P], 0.0, atol=1e-15)
    np.testing.assert_allclose(Bend[0, [0, P]], [1, 0], atol=1e-15)
    np.testing.assert_allclose(Bend[1, [0, P]], [0, 1], atol=1e-15)


def test_basis_low_bubbles_closed_form():
    """P^{1,1}_0 = 1 and P^{1,1}_1(x) = 2x give phi_1 = (1-x^2)/4 and
    phi_2 = (1-x^2) x / 2 at P >= 3."""
    x = np.linspace(-1, 1, 11)
    B, DB = oracle.modified_basis(4, x)
    np.testing.assert_allclose(B[:, 1], (1 - x * x) / 4, atol=1e-15)
    np.testing.assert_allclose(B[:, 2], (1 - x * x) * x / 2, atol=1e-15)
    np.testing.assert_allclose(DB[:, 1], -x / 2, atol=1e-15)
    np.testing.assert_allclose(DB[:, 2], (1 - 3 * x * x) / 2, atol=1e-14)


@pytest.mark.parametrize("P", [2, 4, 6, 8, 10])
def test_basis_derivative_against_finite_differences(P):
    x = np.linspace(-0.97, 0.97, 23)
    h = 1e-6
    _, DB = oracle.modified_basis(P, x)
    Bp, _ = oracle.modified_basis(P, x + h)
    Bm, _ = oracle.modified_basis(P, x - h)
    np.testing.assert_allclose(DB, (Bp - Bm) / (2 * h), atol=1e-7)


@pytest.mark.parametrize("P", [2, 4, 6, 8, 10])
def test_basis_derivative_equals_collocation(P):
    """phi_p has degree <= P <= Q-1, so the GLL collocation derivative of its
    point values equals its analytic derivative."""
    x, _ = oracle.gll(P + 2)
    B, DB = oracle.modified_basis(P, x)
    D = oracle.lagrange_derivative(x)
    np.testing.assert_allclose(D @ B, DB, atol=1e-12)


@pytest.mark.parametrize("P", [2, 4, 6, 8, 10])
def test_1d_stiffness_closed_form(P):
    """phi_p' = -(p/2) L_p for bubbles (L_p Legendre), which fixes the Jacobi
    normalisation: S1 = [[1/2, ..., -1/2], diag(p^2/(2(2p+1))), ...]."""
    x, w = oracle.gll(P + 2)
    _, DB = oracle.modified_basis(P, x)
    S1 = DB.T @ (w[:, None] * DB)
    ref = np.zeros((P + 1, P + 1))
    ref[0, 0] = ref[P, P] = 0.5
    ref[0, P] = ref[P, 0] = -0.5
    for p in range(1, P):
        ref[p, p] = p * p / (2.0 * (2 * p + 1))
    np.testing.assert_allclose(S1, ref, atol=5e-14)


@pytest.mark.parametrize("P", [4, 6, 8])
def test_1d_mass_sparsity_and_spd(P):
    """Bubble-bubble entries vanish unless |p-q| in {0,2}; vertex-bubble
    entries vanish unless the bubble is p in {1, 2}; M1 is SPD."""
    x, w = oracle.gll(P + 2)
    B, _ = oracle.modified_basis(P, x)
    M1 = B.T @ (w[:, None] * B)
    for p in range(1, P):
        for q in range(1, P):
            if abs(p - q) not in (0, 2):
                assert abs(M1[p, q]) < 1e-15
        for v in (0, P):
            if p not in (1, 2):
                assert abs(M1[v, p]) < 1e-15
    assert np.linalg.eigvalsh(M1).min() > 1e-4


# ------------------------------------------------- tensor-product elements

def _affine_box_J(h, Q, dim):
    nq = Q ** dim
    J = np.zeros((1, dim, dim, nq))
    for a in range(dim):
        J[0, a, a, :] = h[a] / 2
    return J


@pytest.mark.parametrize("P", [2, 4, 6])
def test_kronecker_identities_affine_box(P):
    """Box of sides (hx, hy, hz) all distinct: M_e = (hx hy hz / 8) Mz(x)My(x)Mx and
    L_e = detJ (4/hx^2 M(x)M(x)S1 + 4/hy^2 M(x)S1(x)M + 4/hz^2 S1(x)M(x)M),
    direction 1 in the rightmost factor.  Catches swapped directions."""
    Q = P + 2
    h = np.array([0.3, 0.7, 1.9])
    ops = oracle.ElementOps(3, P, Q, _affine_box_J(h, Q, 3), lam=0.0)
    x, w = oracle.gll(Q)
    B, DB = oracle.modified_basis(P, x)
    M1 = B.T @ (w[:, None] * B)
    S1 = DB.T @ (w[:, None] * DB)
    det = h.prod() / 8
    Mref = det * np.kron(M1, np.kron(M1, M1))
    Lref = det * (4 / h[0] ** 2 * np.kron(M1, np.kron(M1, S1))
                  + 4 / h[1] ** 2 * np.kron(M1, np.kron(S1, M1))
                  + 4 / h[2] ** 2 * np.kron(S1, np.kron(M1, M1)))
    np.testing.assert_allclose(ops.mass_matrix(0), Mref, atol=1e-15)
    np.testing.assert_allclose(ops.laplacian_matrix(0), Lref, atol=1e-13)


def test_2d_laplacian_independent_of_h():
    """On an affine square the 2-D Laplacian S1(x)M1 + M1(x)S1 does not depend on h."""
    P, Q = 4, 6
    L = [oracle.ElementOps(2, P, Q, _affine_box_J([hh, hh], Q, 2), lam=0.0).laplacian_matrix(0)
         for hh in (0.125, 1.0, 3.0)]
    x, w = oracle.gll(Q)
    B, DB = oracle.modified_basis(P, x)
    M1 = B.T @ (w[:, None] * B)
    S1 = DB.T @ (w[:, None] * DB)
    for Li in L:
        np.testing.assert_allclose(Li, np.kron(M1, S1) + np.kron(S1, M1), atol=1e-14)


def _warped_ops(shape, P, lam=1.0, kappa=None, amp=0.05):
    Q = P + 2
    lat = W.lattice(shape)
    x, _ = oracle.gll(Q)
    J = W.element_jacobians(x, lat, amp)
    return oracle.ElementOps(len(shape), P, Q, J, kappa=kappa, lam=lam), lat


def _vertex_constant(P, dim):
    c1 = np.zeros(P + 1)
    c1[0] = c1[P] = 1.0
    c = c1
    for _ in range(dim - 1):
        c = np.kron(c1, c)
    return c


@pytest.mark.parametrize("P", [2, 5])
def test_constants_volume_symmetry_spd_curved(P):
    """On curved elements: L_e 1 = 0, 1^T M_e 1 = element volume (sum w detJ),
    H_e symmetric, M_e Cholesky succeeds."""
    ops, _ = _warped_ops((2, 2, 2), P)
    c = _vertex_constant(P, 3)
    for e in range(ops.nelem):
        L = ops.laplacian_matrix(e)
        M = ops.mass_matrix(e)
        np.testing.assert_allclose(L @ c, 0.0, atol=1e-12)
        assert abs(c @ M @ c - ops.wJ[e].sum()) < 1e-14
        H = ops.helmholtz_matrix(e)
        np.testing.assert_allclose(H, H.T, atol=1e-13)
        np.linalg.cholesky(M)


def test_warped_unit_cube_volume_is_one():
    """Every off-diagonal product of the cyclic warp integrates to zero over a
    period, so the warped unit cube keeps volume 1."""
    for shape, P in (((8, 8, 8), 6), ((3, 5, 4), 4)):
        ops, lat = _warped_ops(shape, P)
        assert abs(ops.wJ.sum() - 1.0) < 1e-13
        dwarp = ops.detJ / np.prod(lat.h / 2)          # det of the curving map alone
        assert dwarp.min() > 0.89 and dwarp.max() < 1.11


@pytest.mark.parametrize("P", [3, 6])
def test_fwd_bwd_roundtrip_curved(P):
    """FwdTrans o BwdTrans = I on curved elements: M_e^{-1} I_e (B u^) = u^."""
    ops, _ = _warped_ops((2, 1, 2), P)
    rng = np.random.default_rng(5)
    c = rng.uniform(-1, 1, (ops.nelem, (P + 1) ** 3))
    u = ops.bwd(c)
    f = ops.iprod(u)
    for e in range(ops.nelem):
        # M_e has condition number ~1e7 at P=6, so the round trip holds to ~1e-9
        np.testing.assert_allclose(np.linalg.solve(ops.mass_matrix(e), f[e]), c[e], atol=1e-8)


def test_projection_reproduces_polynomials():
    """A polynomial of degree <= P per reference direction lies in the space:
    BwdTrans(FwdTrans f) = f at the quadrature points, on a curved element."""
    P = 4
    ops, _ = _warped_ops((1, 1, 1), P)
    x = ops.x
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    f = (X ** 4 - 2 * X * Y ** 3 + Z ** 2 * Y * X + 0.5).transpose(2, 1, 0).reshape(1, -1)
    c = np.linalg.solve(ops.mass_matrix(0), ops.iprod(f)[0])
    np.testing.assert_allclose(ops.bwd(c[None]), f, atol=1e-12)


def test_listing1_integral_and_projection():
    """Listing 1 (section 3.5): 8 modes (P=7), nModes+1 = 9 GLL points; the
    integral of cos(x)cos(y) over [-1,1]^2 is 4 sin^2(1) (value in the text)."""
    with open(os.path.join(GOLDEN, "listing1_integral.txt")) as fh:
        nm, npts, exact = [l for l in fh if not l.startswith("#")][0].split()
    P, Q, exact = int(nm) - 1, int(npts), float(exact)
    assert abs(exact - 4 * math.sin(1.0) ** 2) < 1e-15
    ops = oracle.ElementOps(2, P, Q, _affine_box_J([2.0, 2.0], Q, 2), lam=0.0)
    x = ops.x
    Xg, Yg = np.meshgrid(x, x, indexing="ij")
    f = (np.cos(Xg) * np.cos(Yg)).T.reshape(1, -1)
    assert abs(ops.integral(f)[0] - exact) < 1e-14
    # Galerkin orthogonality of the projection (FwdTrans): I(f - B u^) = 0
    c = np.linalg.solve(ops.mass_matrix(0), ops.iprod(f)[0])
    np.testing.assert_allclose(ops.iprod(f - ops.bwd(c[None]))[0], 0.0, atol=1e-15)


def test_listing1_point_count_reading():
    """Reading of Listing 1: nine points (Q = P+2) integrate the P=7 mass matrix
    exactly; eight (P+1) do not, so the text's 'P+1 points' is read as the
    code's nModes+1."""
    P = 7
    xg, wg = np.polynomial.legendre.leggauss(20)
    Bg, _ = oracle.modified_basis(P, xg)
    M_exact = Bg.T @ (wg[:, None] * Bg)
    for Q, ok in ((9, True), (8, False)):
        x, w = oracle.gll(Q)
        B, _ = oracle.modified_basis(P, x)
        err = np.abs(B.T @ (w[:, None] * B) - M_exact).max()
        assert (err < 1e-14) == ok, (Q, err)


def test_sheared_affine_energy_of_physical_polynomials():
    """On an affine element x = A xi + x0 with non-normal A, the stiffness
    quadratic form of u = x1*x2 + 3 x3 equals int |grad_x u|^2 dx computed
    in physical terms (gradient (x2, x1, 3)) by tensor Gauss quadrature.
    Catches G = J^{-T} J^{-1} instead of J^{-1} J^{-T}."""
    P, Q = 3, 5
    A = np.array([[0.7, 0.4, -0.1], [0.05, 0.9, 0.3], [0.2, -0.25, 1.1]])
    x0 = np.array([0.1, -0.2, 0.3])
    J = np.broadcast_to(A[None, :, :, None], (1, 3, 3, Q ** 3)).copy()
    ops = oracle.ElementOps(3, P, Q, J, lam=0.0)
    xq = ops.x
    XI = np.stack([g.transpose(2, 1, 0).reshape(-1) for g in np.meshgrid(xq, xq, xq, indexing="ij")])
    Xp = A @ XI + x0[:, None]
    u = Xp[0] * Xp[1] + 3 * Xp[2]
    c = np.linalg.solve(ops.mass_matrix(0), ops.iprod(u[None])[0])
    np.testing.assert_allclose(ops.bwd(c[None])[0], u, atol=1e-12)    # u in the space
    xg, wg = np.polynomial.legendre.leggauss(6)
    XG = np.stack([g.transpose(2, 1, 0).reshape(-1) for g in np.meshgrid(xg, xg, xg, indexing="ij")])
    WG = np.kron(wg, np.kron(wg, wg))
    Xg = A @ XG + x0[:, None]
    grad2 = Xg[1] ** 2 + Xg[0] ** 2 + 9.0
    exact = abs(np.linalg.det(A)) * WG @ grad2
    assert abs(c @ ops.laplacian_matrix(0) @ c - exact) < 1e-12 * exact
    # mass quadratic form: int u^2 dx
    ug = Xg[0] * Xg[1] + 3 * Xg[2]
    assert abs(c @ ops.mass_matrix(0) @ c - abs(np.linalg.det(A)) * WG @ ug ** 2) < 1e-12


def test_variable_kappa_laplacian_single_point():
    """dH_e/dkappa_q summed over all points with weights kappa_q rebuilds L_e."""
    P = 2
    rng = np.random.default_rng(3)
    ops, _ = _warped_ops((1, 1, 1), P, kappa=rng.uniform(0.5, 2, (1, 64)))
    L = sum(ops.kappa[0, q] * ops.dkappa_matrix(0, q) for q in range(64))
    np.testing.assert_allclose(L, ops.laplacian_matrix(0), atol=1e-13)


# ----------------------------------------------------------- assembly/solve

def test_lattice_assembly_volume_and_constants():
    """Assembled with the lattice map: the global constant (ones on global
    vertex DOFs) has 1^T M 1 = 1 on the warped unit cube and L 1 = 0."""
    P, shape = 3, (3, 2, 2)
    ops, _ = _warped_ops(shape, P, lam=0.0)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    G = [s * P + 1 for s in shape]
    gidx = np.indices(G[::-1]).reshape(3, -1)[::-1]
    one = np.all(gidx % P == 0, axis=0).astype(float)
    Mg = oracle.assembled_matrix(oracle.mass_matrices(ops), l2g, ng)
    Lg = oracle.assembled_matrix([ops.laplacian_matrix(e) for e in range(ops.nelem)], l2g, ng)
    assert abs(one @ (Mg @ one) - 1.0) < 1e-13
    np.testing.assert_allclose(Lg @ one, 0.0, atol=1e-12)
    np.testing.assert_allclose((Lg - Lg.T).toarray(), 0.0, atol=1e-13)
    # gathered constant is the local vertex-constant on every element
    np.testing.assert_array_equal(oracle.gather(one, l2g), np.tile(_vertex_constant(P, 3), (ops.nelem, 1)))


def test_polynomial_manufactured_solution_is_exact():
    """U = X(1-X) Y(1-Y) Z(1-Z) lies in the C0 space at P >= 2 on the affine
    lattice and vanishes on the boundary: the discrete solution of the weak
    problem with l(v) = a(U, v) reproduces U exactly.  Pins the weak RHS, the
    assembly, the Dirichlet restriction and the solve together."""
    P, shape = 2, (2, 3, 2)
    ops, lat = _warped_ops(shape, P, lam=1.5, amp=0.0)
    Xp = W.lattice_points(ops.x, lat)
    f = Xp * (1 - Xp)
    U = f.prod(axis=1)
    dfX = 1 - 2 * Xp
    dU = np.stack([dfX[:, 0] * f[:, 1] * f[:, 2], f[:, 0] * dfX[:, 1] * f[:, 2],
                   f[:, 0] * f[:, 1] * dfX[:, 2]], axis=1) * (lat.h[None, :, None] / 2)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    b = oracle.assemble_vector(ops.weak_rhs(U, dU), l2g, ng)
    b[dm.astype(bool)] = 0
    u = direct_solve(oracle.helmholtz_matrices(ops), l2g, ng, dm, b)
    np.testing.assert_allclose(ops.bwd(oracle.gather(u, l2g)), U, atol=1e-14)


def test_manufactured_sine_converges_exponentially():
    """Curved 3^3 lattice, U = sin(pi X) sin(pi Y) sin(pi Z): the max error at
    the quadrature points falls by > 5x per two orders (exponential
    convergence of the spectral/hp discretisation)."""
    errs = []
    for P in (2, 4, 6):
        ops, lat = _warped_ops((3, 3, 3), P)
        l2g, ng, dm = W.lattice_l2g((3, 3, 3), P)
        U, dU = W.manufactured_ref_gradient(ops.x, lat)
        b = oracle.assemble_vector(ops.weak_rhs(U, dU), l2g, ng)
        b[dm.astype(bool)] = 0
        u = direct_solve(oracle.helmholtz_matrices(ops), l2g, ng, dm, b)
        errs.append(np.abs(ops.bwd(oracle.gather(u, l2g)) - U).max())
    assert errs[0] < 2e-2 and errs[1] < errs[0] / 100 and errs[2] < errs[1] / 100, errs


def test_pcg_matches_direct_solve():
    P, shape = 3, (3, 3, 2)
    ops, lat = _warped_ops(shape, P)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    mats = oracle.helmholtz_matrices(ops)
    b = oracle.assemble_vector(ops.iprod(np.ones((ops.nelem, ops.Q ** 3))), l2g, ng)
    b[dm.astype(bool)] = 0
    xd = direct_solve(mats, l2g, ng, dm, b)
    A = MaskedOperator(mats, l2g, ng, dm)
    xc, it, res = pcg(A, b, jacobi_diagonal(mats, l2g, ng, dm), rtol=1e-13)
    assert res < 1e-13 and it > 5
    np.testing.assert_allclose(xc, xd, atol=1e-12 * np.abs(xd).max())


# ----------------------------------------------------------------- gradient

def _grad_problem(shape, P, seed):
    Q = P + 2
    lat = W.lattice(shape)
    x, _ = oracle.gll(Q)
    J = W.element_jacobians(x, lat, 0.05)
    E, nq = lat.nelem, Q ** 3
    kap = W.uniform(seed, (E, nq), 0.5, 2.0)
    lam = W.uniform(seed + 1, (E,), 0.5, 2.0)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    ref = oracle.ElementOps(3, P, Q, J, lam=1.0)
    U, dU = W.manufactured_ref_gradient(x, lat)
    b = oracle.assemble_vector(ref.weak_rhs(U, dU), l2g, ng)
    b[dm.astype(bool)] = 0
    _, u_t = oracle.loss_and_solution(oracle.helmholtz_matrices(ref), l2g, ng, dm, b, np.zeros(ng))
    return J, kap, lam, l2g, ng, dm, b, u_t


def test_adjoint_gradient_matches_finite_differences():
    """Central differences of the loss along random directions agree with
    -z^T dA u for both lambda (per element) and kappa (per point)."""
    P, shape = 2, (2, 2, 1)
    J, kap, lam, l2g, ng, dm, b, u_t = _grad_problem(shape, P, 77)

    def loss(k, l):
        ops = oracle.ElementOps(3, P, P + 2, J, kappa=k, lam=l)
        return oracle.loss_and_solution(oracle.helmholtz_matrices(ops), l2g, ng, dm, b, u_t)

    ops = oracle.ElementOps(3, P, P + 2, J, kappa=kap, lam=lam)
    mats = oracle.helmholtz_matrices(ops)
    L0, u = loss(kap, lam)
    assert L0 > 1e-8
    z = direct_solve(mats, l2g, ng, dm, u - u_t)
    dkap, dlam = oracle.param_grad(ops, l2g, u, z)
    rng = np.random.default_rng(6)
    for _ in range(2):
        vk = rng.standard_normal(kap.shape)
        vl = rng.standard_normal(lam.shape)
        eps = 1e-5
        fd = (loss(kap + eps * vk, lam + eps * vl)[0] - loss(kap - eps * vk, lam - eps * vl)[0]) / (2 * eps)
        an = np.sum(dkap * vk) + np.sum(dlam * vl)
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-12), (fd, an)


# ---------------------------------------------------------------- PhysDeriv,
# IProductWRTDerivBase and FwdTrans (the explicit-type building blocks of
# section 2.2 and the projection of the listing in section 3.5)

def _points(x, dim):
    """Reference coordinates of the tensor points, q = i + Q(j + Q l)."""
    g = np.meshgrid(*([x] * dim), indexing="ij")
    return np.stack([gg.transpose(*range(dim)[::-1]).reshape(-1) for gg in g])


def test_phys_deriv_exact_on_sheared_affine_element():
    """u = x1^2 + x1 x2 + 3 x3 (degree <= 2 per reference direction, so its
    interpolant is exact) on x = A xi + x0 with a non-normal A: the physical
    gradient (2 x1 + x2, x1, 3) is reproduced at every point.  A transposed
    inverse Jacobian or a swapped direction fails."""
    P, Q = 3, 5
    A = np.array([[0.7, 0.4, -0.1], [0.05, 0.9, 0.3], [0.2, -0.25, 1.1]])
    x0 = np.array([0.1, -0.2, 0.3])
    J = np.broadcast_to(A[None, :, :, None], (1, 3, 3, Q ** 3)).copy()
    ops = oracle.ElementOps(3, P, Q, J)
    X = A @ _points(ops.x, 3) + x0[:, None]
    u = X[0] ** 2 + X[0] * X[1] + 3 * X[2]
    du = ops.phys_deriv(u[None])[0]
    np.testing.assert_allclose(du[0], 2 * X[0] + X[1], atol=1e-12)
    np.testing.assert_allclose(du[1], X[0], atol=1e-12)
    np.testing.assert_allclose(du[2], 3.0, atol=1e-12)


def test_phys_deriv_2d_affine_exact():
    """2-D: u = x^3 - 2 x y on a sheared parallelogram, gradient (3x^2 - 2y, -2x)."""
    P, Q = 4, 6
    A = np.array([[0.8, 0.3], [-0.2, 1.1]])
    J = np.broadcast_to(A[None, :, :, None], (1, 2, 2, Q ** 2)).copy()
    ops = oracle.ElementOps(2, P, Q, J)
    X = A @ _points(ops.x, 2)
    du = ops.phys_deriv((X[0] ** 3 - 2 * X[0] * X[1])[None])[0]
    np.testing.assert_allclose(du[0], 3 * X[0] ** 2 - 2 * X[1], atol=1e-12)
    np.testing.assert_allclose(du[1], -2 * X[0], atol=1e-12)


def test_phys_deriv_chain_rule_on_curved_elements():
    """On warped elements, for u a polynomial of the reference coordinates of
    degree <= Q-1 per direction, J^T grad_x u equals the analytic reference
    gradient: checks the inverse Jacobian against J itself."""
    P = 4
    ops, _ = _warped_ops((2, 2, 1), P)
    xi = _points(ops.x, 3)
    u = xi[0] ** 5 - xi[0] * xi[1] ** 2 * xi[2] + 2 * xi[2] ** 3
    dref = np.stack([5 * xi[0] ** 4 - xi[1] ** 2 * xi[2],
                     -2 * xi[0] * xi[1] * xi[2],
                     -xi[0] * xi[1] ** 2 + 6 * xi[2] ** 2])
    lat = W.lattice((2, 2, 1))
    J = W.element_jacobians(ops.x, lat, 0.05)                   # (E, c, a, q)
    du = ops.phys_deriv(np.broadcast_to(u, (ops.nelem, u.size)))
    back = np.einsum("ecaq,ecq->eaq", J, du)
    np.testing.assert_allclose(back, np.broadcast_to(dref, back.shape), atol=1e-11)


@pytest.mark.parametrize("dim,P", [(3, 3), (3, 5), (2, 4)])
def test_iprod_deriv_of_gradient_is_the_laplacian(dim, P):
    """IProductWRTDerivBase of the physical gradient of a discrete field is its
    Laplacian matrix-vector product (kappa = 1) on curved elements: the
    gradient of B u^ is exact at the points, so sum_q w detJ grad phi_m . grad u
    = (L_e u^)_m.  Three independent constructions meet: G (Laplacian), the
    collocation derivative with J^{-1} (PhysDeriv) and D_a B with J^{-1}."""
    shape = (2, 1, 2) if dim == 3 else (2, 3)
    ops, _ = _warped_ops(shape, P, lam=0.0, amp=0.05 if dim == 3 else 0.0)
    rng = np.random.default_rng(31 + P)
    c = rng.uniform(-1, 1, (ops.nelem, (P + 1) ** dim))
    got = ops.iprod_deriv(ops.phys_deriv(ops.bwd(c)))
    want = np.stack([ops.laplacian_matrix(e) @ c[e] for e in range(ops.nelem)])
    np.testing.assert_allclose(got, want, atol=1e-11 * np.abs(want).max())


def test_iprod_deriv_divergence_theorem_affine():
    """For the constant field f = e_1 on an affine box [0,hx]x[0,hy]x[0,hz],
    sum_m I[m] c_m = int d(u)/dx1 dx = int over the two x1-faces of u, with u
    the vertex-constant 1 of the box (all derivatives vanish): 0; and for u = x1
    (coefficients of the linear vertex modes) the result is the volume."""
    P, Q = 3, 5
    h = np.array([0.5, 0.25, 0.75])
    ops = oracle.ElementOps(3, P, Q, _affine_box_J(h, Q, 3))
    f = np.zeros((1, 3, Q ** 3))
    f[0, 0] = 1.0
    I = ops.iprod_deriv(f)[0]
    one = _vertex_constant(P, 3)
    assert abs(I @ one) < 1e-14
    # x1 on [0, hx]: vertex modes p=0 -> 0, p=P -> hx in direction 1
    c1 = np.zeros(P + 1)
    c1[P] = h[0]
    e1 = np.zeros(P + 1)
    e1[0] = e1[P] = 1.0
    cx = np.kron(e1, np.kron(e1, c1))
    assert abs(I @ cx - h.prod()) < 1e-14


@pytest.mark.parametrize("P", [3, 5])
def test_fwd_trans_inverts_bwd_and_is_galerkin(P):
    """FwdTrans o BwdTrans = I on curved elements, and the projection of an
    arbitrary point field is Galerkin-orthogonal: I_e(f - B FwdTrans(f)) = 0."""
    ops, _ = _warped_ops((2, 1, 1), P)
    rng = np.random.default_rng(41 + P)
    c = rng.uniform(-1, 1, (ops.nelem, (P + 1) ** 3))
    np.testing.assert_allclose(ops.fwd(ops.bwd(c)), c, atol=1e-9)
    f = rng.uniform(-1, 1, (ops.nelem, (P + 2) ** 3))
    r = ops.iprod(f - ops.bwd(ops.fwd(f)))
    assert np.abs(r).max() < 1e-13 * np.abs(ops.iprod(f)).max()


# ------------------------------------------- conforming variable-order assembly
# (section 4.2: the order varies per element and the variation is built into
# the assembly between neighbours; the modified basis' boundary-interior
# decomposition makes the minimum rule on shared faces and edges conforming)

def _varp_problem(shape, orders, amp=0.05, lam=1.0, mass_only=False):
    perm, l2g, ng, dm = W.varp_lattice_l2g(shape, orders)
    lat = W.lattice(shape)
    ords = np.asarray(orders)[perm]
    groups, mats = [], []
    for P in sorted(set(ords.tolist())):
        idx = perm[ords == P]
        Q = P + 2
        sub = W.Lattice(lat.shape, lat.h, lat.origins[idx])
        ops = oracle.ElementOps(3, P, Q, W.element_jacobians(oracle.gll(Q)[0], sub, amp), lam=lam)
        groups.append((P, idx, ops))
        mats += oracle.mass_matrices(ops) if mass_only else oracle.helmholtz_matrices(ops)
    return perm, l2g, ng, dm, groups, mats


def _eval_expansion(P, c, pts):
    """u(xi) = sum_m c_m phi_p(xi_1) phi_q(xi_2) phi_r(xi_3), m = p + n(q + n r)."""
    n = P + 1
    B = [oracle.modified_basis(P, pts[:, a])[0] for a in range(3)]     # (npts, n) each
    C = c.reshape(n, n, n)                                             # [r][q][p]
    return np.einsum("rqp,kp,kq,kr->k", C, B[0], B[1], B[2])


def test_varp_uniform_orders_reduce_to_the_lattice_map():
    perm, l2g, ng, dm = W.varp_lattice_l2g((2, 3, 2), [4] * 12)
    g0, ng0, dm0 = W.lattice_l2g((2, 3, 2), 4)
    assert ng == ng0 + 1 and dm[-1] == 1
    np.testing.assert_array_equal(np.stack(l2g), g0)
    np.testing.assert_array_equal(dm[:-1], dm0)


def test_varp_assembly_is_continuous_across_faces():
    """Any global coefficient vector gives element expansions whose traces
    agree on every shared face (checked at random face points, both
    elements' own bases): the minimum rule makes the space conforming."""
    shape = (3, 2, 2)
    orders = [2, 5, 3, 4, 2, 6, 3, 3, 5, 2, 4, 6]
    perm, l2g, ng, dm, _, _ = _varp_problem(shape, orders)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, ng)
    x[-1] = 0.0                              # the constrained-mode DOF is zero
    pos = {int(e): k for k, e in enumerate(perm)}
    st = (1, shape[0], shape[0] * shape[1])
    st_ = np.asarray(st)
    ords = np.asarray(orders)
    checked = 0
    for e in range(int(np.prod(shape))):
        ce = np.indices(shape[::-1]).reshape(3, -1)[::-1][:, e]
        for a in range(3):
            if ce[a] + 1 >= shape[a]:
                continue
            nb = e + st[a]
            pts = rng.uniform(-1, 1, (9, 3))
            pe, pn = pts.copy(), pts.copy()
            pe[:, a], pn[:, a] = 1.0, -1.0
            ue = _eval_expansion(ords[e], x[l2g[pos[e]]], pe)
            un = _eval_expansion(ords[nb], x[l2g[pos[nb]]], pn)
            np.testing.assert_allclose(ue, un, atol=1e-13)
            checked += 1
    assert checked == 20


def test_varp_projection_reproduces_a_conforming_polynomial():
    """X(1-X)Y(1-Y)Z(1-Z) (degree 2 per direction, zero on the boundary) lies
    in the assembled variable-order space when every order is >= 2, so its
    Galerkin projection with the assembled mass matrix returns it exactly at
    every element's points (affine lattice)."""
    shape = (2, 3, 2)
    orders = [2, 3, 4, 2, 5, 2, 3, 4, 2, 6, 3, 2]
    perm, l2g, ng, dm, groups, mats = _varp_problem(shape, orders, amp=0.0, mass_only=True)
    lat = W.lattice(shape)
    bl, fl = [None] * len(perm), {}
    for P, idx, ops in groups:
        sub = W.Lattice(lat.shape, lat.h, lat.origins[idx])
        X = W.lattice_points(ops.x, sub)                           # (E_g, 3, nq)
        f = np.prod(X * (1 - X), axis=1)
        rhs = ops.iprod(f)
        for k, e in enumerate(idx):
            k_space = int(np.flatnonzero(perm == e)[0])
            bl[k_space] = rhs[k]
            fl[k_space] = (ops, k, f[k])
    b = oracle.assemble_vector(bl, l2g, ng)
    x = direct_solve(mats, l2g, ng, dm, b)
    for k_space, (ops, k, fk) in fl.items():
        np.testing.assert_allclose(ops.bwd(x[l2g[k_space]][None])[0], fk, atol=1e-13)


# ----------------------------------------- the Neumann filter equation (3)
# u** - alpha^2 lap u** = u*, du**/dn = 0 (section 3.4, Eq. (3)): the same
# Helmholtz operator with kappa = alpha^2, lambda = 1 and no Dirichlet DOFs.

def test_neumann_filter_equation_exact_for_a_polynomial_solution():
    """U = g(X) g(Y) g(Z), g = X^2 (1-X)^2, has zero normal derivative on the
    unit cube and degree 4 per direction.  With the right-hand side taken from
    the strong form, f = U - alpha^2 lap U (integrated exactly at Q = 6), the
    Neumann Galerkin solve at P = 4 on an affine lattice returns U exactly --
    only if the operator is mass + alpha^2 times the stiffness and no boundary
    DOF is constrained (integration by parts with dU/dn = 0)."""
    shape, P, alpha = (2, 2, 2), 4, 0.3
    Q = P + 2
    lat = W.lattice(shape)
    J = W.element_jacobians(oracle.gll(Q)[0], lat, 0.0)
    kap = np.full((lat.nelem, Q ** 3), alpha ** 2)
    ops = oracle.ElementOps(3, P, Q, J, kappa=kap, lam=1.0)
    X = W.lattice_points(ops.x, lat)                       # (E, 3, nq)
    g = X ** 2 * (1 - X) ** 2
    d2g = 2 - 12 * X + 12 * X ** 2
    U = g.prod(axis=1)
    lapU = d2g[:, 0] * g[:, 1] * g[:, 2] + g[:, 0] * d2g[:, 1] * g[:, 2] + g[:, 0] * g[:, 1] * d2g[:, 2]
    l2g, ng, _ = W.lattice_l2g(shape, P)
    b = oracle.assemble_vector(ops.iprod(U - alpha ** 2 * lapU), l2g, ng)
    x = direct_solve(oracle.helmholtz_matrices(ops), l2g, ng, np.zeros(ng, np.uint8), b)
    np.testing.assert_allclose(ops.bwd(oracle.gather(x, l2g)), U, atol=1e-14)


# ------------------------------------- collapsed-coordinate triangles (2.1)
from math import comb, factorial

from oracle import collapsed as C


def _tri_integral(a, b):
    """Closed form of the integral of xi_1^a xi_2^b over the reference
    triangle (shifted to u, v >= 0, u + v <= 2: a Dirichlet integral)."""
    s = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            s += (comb(a, i) * comb(b, j) * (-1) ** (a - i + b - j)
                  * 2.0 ** (i + j + 2) * factorial(i) * factorial(j) / factorial(i + j + 2))
    return s


@pytest.mark.parametrize("n", [2, 4, 7])
def test_gauss_radau_jacobi_exactness(n):
    x, w = C.gauss_radau_jacobi(n, 1.0, 0.0)
    assert x[0] == -1.0 and np.all(np.diff(x) > 0) and x[-1] < 1.0
    for k in range(2 * n):
        # int_{-1}^{1} x^k (1-x) dx = int x^k - int x^(k+1)
        ik = (2.0 / (k + 1)) if k % 2 == 0 else 0.0
        ik1 = (2.0 / (k + 2)) if (k + 1) % 2 == 0 else 0.0
        got = w @ x ** k
        if k <= 2 * n - 2:
            assert abs(got - (ik - ik1)) < 1e-13, (n, k)
        else:
            assert abs(got - (ik - ik1)) > 1e-8, (n, k)


@pytest.mark.parametrize("P", [2, 4, 6])
def test_triangle_quadrature_integrates_degree_2P(P):
    Q = P + 2
    e1, e2, W = C.tri_points(Q)
    x1, x2 = C.xi_of_eta(e1, e2)
    assert abs(W.sum() - 2.0) < 1e-14
    for a in range(2 * P + 1):
        for b in range(2 * P + 1 - a):
            # the closed form sums alternating binomial terms: allow 1e-12
            assert abs(W @ (x1 ** a * x2 ** b) - _tri_integral(a, b)) < 1e-12, (a, b)


@pytest.mark.parametrize("P", [1, 3, 5, 8])
def test_triangle_basis_spans_total_degree_P(P):
    """Every mode is a polynomial of total degree <= P in xi, and the
    (P+1)(P+2)/2 modes are independent: they span exactly that space."""
    rng = np.random.default_rng(P)
    e1, e2 = rng.uniform(-1, 1, 200), rng.uniform(-1, 0.95, 200)
    x1, x2 = C.xi_of_eta(e1, e2)
    Phi, _, _ = C.tri_basis(P, e1, e2)
    nm = (P + 1) * (P + 2) // 2
    assert Phi.shape[1] == nm
    Mon = np.stack([x1 ** a * x2 ** b for a in range(P + 1) for b in range(P + 1 - a)], axis=1)
    coef, *_ = np.linalg.lstsq(Mon, Phi, rcond=None)
    assert np.abs(Mon @ coef - Phi).max() < 1e-11
    assert np.linalg.matrix_rank(Phi) == nm


@pytest.mark.parametrize("P", [2, 5])
def test_triangle_vertex_edge_interior_structure(P):
    """A + B + C = 1; interior modes vanish on all three edges; each edge
    carries only its two vertices and its own edge modes."""
    modes = C.tri_modes(P)
    iA, iC, iB = modes.index((0, 0)), modes.index((0, P)), modes.index((P, 0))
    t = np.linspace(-1, 1, 9)
    Phi, _, _ = C.tri_basis(P, t, np.full_like(t, 0.3))
    np.testing.assert_allclose(Phi[:, iA] + Phi[:, iB] + Phi[:, iC], 1.0, atol=1e-14)
    interior = [m for m, (p, q) in enumerate(modes) if 0 < p < P and q >= 1]
    bottom = {iA, iB} | {m for m, (p, q) in enumerate(modes) if 0 < p < P and q == 0}
    left = {iA, iC} | {m for m, (p, q) in enumerate(modes) if p == 0 and 0 < q < P}
    right = {iB, iC} | {m for m, (p, q) in enumerate(modes) if p == P and 0 < q < P}
    s = np.linspace(-0.9, 0.9, 7)
    for edge, (e1, e2) in (("bottom", (s, -np.ones_like(s))), ("left", (-np.ones_like(s), s)),
                           ("right", (np.ones_like(s), s))):
        Phi, _, _ = C.tri_basis(P, e1, e2)
        keep = {"bottom": bottom, "left": left, "right": right}[edge]
        others = [m for m in range(len(modes)) if m not in keep]
        assert np.abs(Phi[:, others]).max() < 1e-14, edge
        if interior:
            assert np.abs(Phi[:, interior]).max() < 1e-14


@pytest.mark.parametrize("P", [2, 4, 6])
def test_triangle_mass_projection_and_laplacian(P):
    """On a sheared affine triangle: M SPD, 1^T M 1 = area, FwdTrans o BwdTrans
    = I, total-degree-P polynomials reproduced, L 1 = 0, and the stiffness
    form of the physical polynomial u = x1^2 - x1 x2 + 2 x2 equals the
    integral of |grad u|^2 (gradient (2 x1 - x2, -x1 + 2))."""
    Q = P + 2
    A = np.array([[0.8, 0.35], [-0.1, 1.2]])
    nq = Q * (Q - 1)
    J = np.broadcast_to(A[None, :, :, None], (1, 2, 2, nq)).copy()
    ops = C.TriOps(P, Q, J, lam=0.0)
    M = ops.mass_matrix(0)
    np.linalg.cholesky(M)
    modes = C.tri_modes(P)
    one = np.zeros(len(modes))
    for v in ((0, 0), (0, P), (P, 0)):
        one[modes.index(v)] = 1.0
    area = 2.0 * abs(np.linalg.det(A))
    assert abs(one @ M @ one - area) < 1e-13
    rng = np.random.default_rng(9)
    c = rng.uniform(-1, 1, (1, len(modes)))
    np.testing.assert_allclose(ops.fwd(ops.bwd(c)), c, atol=1e-10)
    np.testing.assert_allclose(ops.laplacian_matrix(0) @ one, 0.0, atol=1e-12)
    x1r, x2r = C.xi_of_eta(ops.e1, ops.e2)
    X = A @ np.stack([x1r, x2r])
    u = X[0] ** 2 - X[0] * X[1] + 2 * X[1]
    cu = ops.fwd(u[None])[0]
    np.testing.assert_allclose(ops.bwd(cu[None])[0], u, atol=1e-12)
    grad2 = (2 * X[0] - X[1]) ** 2 + (-X[0] + 2) ** 2
    exact = ops.wJ[0] @ grad2          # degree 2 <= 2P: the rule is exact
    assert abs(cu @ ops.laplacian_matrix(0) @ cu - exact) < 1e-12 * exact


# ------------------------- triangle meshes: C0 assembly with orientation signs

def _tri_affine_mesh(n, P, rot):
    """Oracle operators of the affine triangle mesh of the unit square with
    rotated local vertex orders, its signed numbering and the physical
    coordinates of every quadrature point."""
    Q = P + 2
    x1r, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    J = W.tri_lattice_jacobians(n, oracle.gll(Q)[0], x1r, 0.0, rot)
    ops = C.TriOps(P, Q, J)
    V = W.tri_lattice_vertices(n)
    V = np.take_along_axis(V, (np.asarray(rot)[:, None] + np.arange(3)[None, :]) % 3, axis=1)
    xy = np.stack([V % (n + 1), V // (n + 1)], axis=-1) / n          # (E, 3, 2)
    x1, x2 = C.xi_of_eta(ops.e1, ops.e2)
    X = (xy[:, 0, None, :] * (-(x1 + x2) / 2)[None, :, None] + xy[:, 1, None, :] * ((1 + x1) / 2)[None, :, None]
         + xy[:, 2, None, :] * ((1 + x2) / 2)[None, :, None])        # (E, nq, 2)
    return ops, V, X


def _edge_traces(P, V, xloc, s):
    """Values of each element's expansion along its three edges at the global
    edge parameters s (edges run from the lower to the higher vertex id)."""
    out = {}
    for e in range(V.shape[0]):
        A_, B_, C_ = V[e]
        for a_, b_, which in ((A_, B_, "AB"), (A_, C_, "AC"), (B_, C_, "BC")):
            t = s if a_ < b_ else -s
            if which == "AB":
                e1, e2 = t, -np.ones_like(t)
            elif which == "AC":
                e1, e2 = -np.ones_like(t), t
            else:
                e1, e2 = np.ones_like(t), t
            Phi, _, _ = C.tri_basis(P, e1, e2)
            out.setdefault((min(a_, b_), max(a_, b_)), []).append(Phi @ xloc[e])
    return out


@pytest.mark.parametrize("P", [2, 4, 5])
def test_signed_triangle_numbering_is_continuous_across_edges(P):
    """A random global vector, gathered with the signs, gives element
    expansions that agree along every shared edge (the traces are continuous);
    dropping the signs breaks continuity from P = 3 on (bubble k = 2 is the
    first that changes sign when its edge is traversed the other way)."""
    n = 3
    E = 2 * n * n
    rot = W.tri_rotations(11 + P, E)
    l2g, sign, ng, _ = W.tri_lattice_l2g(n, P, rot)
    V = np.take_along_axis(W.tri_lattice_vertices(n), (rot[:, None] + np.arange(3)[None, :]) % 3, axis=1)
    x = np.random.default_rng(P).uniform(-1, 1, ng)
    s = np.linspace(-0.9, 0.8, 7)
    worst = 0.0
    for vals in _edge_traces(P, V, oracle.gather(x, l2g, sign), s).values():
        if len(vals) == 2:
            worst = max(worst, np.abs(vals[0] - vals[1]).max())
    assert worst < 1e-12
    if P < 3:
        return
    bad = 0.0
    for vals in _edge_traces(P, V, oracle.gather(x, l2g), s).values():
        if len(vals) == 2:
            bad = max(bad, np.abs(vals[0] - vals[1]).max())
    assert bad > 1e-3


@pytest.mark.parametrize("P", [4, 6])
def test_signed_triangle_projection_is_exact_for_degree_P(P):
    """Global L2 projection (assembled mass matrix with signs) reproduces a
    polynomial of total degree P on the affine mesh; without the signs it
    does not."""
    n = 3
    E = 2 * n * n
    rot = W.tri_rotations(21 + P, E)
    ops, V, X = _tri_affine_mesh(n, P, rot)
    l2g, sign, ng, _ = W.tri_lattice_l2g(n, P, rot)
    u = X[..., 0] ** 3 * X[..., 1] - 2 * X[..., 0] * X[..., 1] ** 2 + 0.5 * X[..., 0] ** 4 + X[..., 1]
    mats = [ops.mass_matrix(e) for e in range(E)]
    none = np.zeros(ng, np.uint8)
    for sg, ok in ((sign, True), (None, False)):
        b = oracle.assemble_vector(ops.iprod(u), l2g, ng, sg)
        x = oracle.direct_solve(mats, l2g, ng, none, b, sg)
        err = np.abs(ops.bwd(oracle.gather(x, l2g, sg)) - u).max()
        assert (err < 1e-11) == ok, (sg is None, err)


@pytest.mark.parametrize("P", [4, 5])
def test_signed_triangle_helmholtz_solve_is_exact(P):
    """-lap u + u = f on the unit square, u = x(1-x)y(1-y) (zero on the
    boundary), weak right-hand side integral f phi_m, Dirichlet boundary
    DOFs: the assembled solve with signs reproduces u at every point."""
    n = 3
    E = 2 * n * n
    rot = W.tri_rotations(31 + P, E)
    ops, V, X = _tri_affine_mesh(n, P, rot)
    l2g, sign, ng, dirichlet = W.tri_lattice_l2g(n, P, rot)
    x_, y_ = X[..., 0], X[..., 1]
    u = x_ * (1 - x_) * y_ * (1 - y_)
    f = 2 * y_ * (1 - y_) + 2 * x_ * (1 - x_) + u
    mats = [ops.helmholtz_matrix(e) for e in range(E)]
    b = oracle.assemble_vector(ops.iprod(f), l2g, ng, sign)
    x = oracle.direct_solve(mats, l2g, ng, dirichlet, b, sign)
    assert np.abs(ops.bwd(oracle.gather(x, l2g, sign)) - u).max() < 1e-12


# ------------------------------------------------- collapsed-coordinate tetrahedra (2.1)

def _tet_integral(a, b, c):
    """Closed form of the integral of xi_1^a xi_2^b xi_3^c over the reference
    tetrahedron (shifted to u = 1 + xi, u >= 0, u_1 + u_2 + u_3 <= 2: a
    Dirichlet integral 2^(i+j+k+3) i! j! k! / (i+j+k+3)!)."""
    s = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            for k in range(c + 1):
                s += (comb(a, i) * comb(b, j) * comb(c, k) * (-1) ** (a - i + b - j + c - k)
                      * 2.0 ** (i + j + k + 3) * factorial(i) * factorial(j) * factorial(k)
                      / factorial(i + j + k + 3))
    return s


def test_gauss_radau_jacobi_weight_two_exactness():
    for n in (2, 3, 6):
        x, w = C.gauss_radau_jacobi(n, 2.0, 0.0)
        for k in range(2 * n):
            # int_{-1}^{1} x^k (1-x)^2 dx = I_k - 2 I_{k+1} + I_{k+2}
            I = lambda j: (2.0 / (j + 1)) if j % 2 == 0 else 0.0
            exact = I(k) - 2 * I(k + 1) + I(k + 2)
            err = abs(w @ x ** k - exact)
            assert (err < 1e-13) == (k <= 2 * n - 2), (n, k, err)


@pytest.mark.parametrize("P", [1, 2, 4])
def test_tetrahedron_quadrature_integrates_degree_2P(P):
    Q = P + 2
    e1, e2, e3, W = C.tet_points(Q)
    x1, x2, x3 = C.xi_of_eta3(e1, e2, e3)
    assert abs(W.sum() - 4.0 / 3.0) < 1e-14
    for a in range(2 * P + 1):
        for b in range(2 * P + 1 - a):
            for c in range(2 * P + 1 - a - b):
                got = W @ (x1 ** a * x2 ** b * x3 ** c)
                assert abs(got - _tet_integral(a, b, c)) < 1e-12, (a, b, c)


@pytest.mark.parametrize("P", [1, 2, 3, 5])
def test_tetrahedron_basis_spans_total_degree_P(P):
    """(P+1)(P+2)(P+3)/6 independent modes that reproduce every monomial of
    total degree <= P (L2 projection exact), but not every one of degree P+1."""
    Q = P + 2
    e1, e2, e3, W = C.tet_points(Q)
    x1, x2, x3 = C.xi_of_eta3(e1, e2, e3)
    Phi, _, _, _ = C.tet_basis(P, e1, e2, e3)
    assert Phi.shape[1] == (P + 1) * (P + 2) * (P + 3) // 6
    M = Phi.T @ (W[:, None] * Phi)
    np.linalg.cholesky(M)
    for a in range(P + 1):
        for b in range(P + 1 - a):
            for c in range(P + 1 - a - b):
                f = x1 ** a * x2 ** b * x3 ** c
                cf = np.linalg.solve(M, Phi.T @ (W * f))
                assert np.abs(Phi @ cf - f).max() < 1e-11, (a, b, c)
    worst = 0.0                      # some monomial of degree P+1 is not reproduced
    for a in range(P + 2):
        for b in range(P + 2 - a):
            f = x1 ** a * x2 ** b * x3 ** (P + 1 - a - b)
            cf = np.linalg.solve(M, Phi.T @ (W * f))
            worst = max(worst, np.abs(Phi @ cf - f).max())
    assert worst > 1e-6


@pytest.mark.parametrize("P", [2, 4])
def test_tetrahedron_vertex_modes_and_bottom_face(P):
    """The four vertex modes are 1 at their vertex and 0 at the other three,
    every other mode vanishes at all four vertices, the vertex modes sum to 1,
    and on face ABC (eta_3 = -1) the r = 0 modes are the triangle basis while
    all rising modes and D vanish."""
    modes = C.tet_modes(P)
    tri = C.tri_modes(P)
    verts = {"A": (-1.0, -1.0, -1.0), "B": (1.0, -1.0, -1.0), "C": (0.3, 1.0, -1.0), "D": (0.3, -0.2, 1.0)}
    vidx = {"A": modes.index((tri.index((0, 0)), 1, 0)), "B": modes.index((tri.index((P, 0)), 1, 0)),
            "C": modes.index((tri.index((0, P)), 1, 0)), "D": len(modes) - 1}
    for name, (a, b, c) in verts.items():
        Phi, _, _, _ = C.tet_basis(P, np.array([a]), np.array([b]), np.array([c]))
        expect = np.zeros(len(modes))
        expect[vidx[name]] = 1.0
        np.testing.assert_allclose(Phi[0], expect, atol=1e-13)
    rng = np.random.default_rng(3)
    e1, e2, e3 = rng.uniform(-1, 1, (3, 20))
    Phi, _, _, _ = C.tet_basis(P, e1, e2, e3)
    np.testing.assert_allclose(Phi[:, list(vidx.values())].sum(axis=1), 1.0, atol=1e-13)
    PhiB, _, _, _ = C.tet_basis(P, e1, e2, -np.ones(20))
    T, _, _ = C.tri_basis(P, e1, e2)
    for m, (t, s, r) in enumerate(modes):
        if t >= 0 and r == 0:
            np.testing.assert_allclose(PhiB[:, m], T[:, t], atol=1e-13)
        else:
            np.testing.assert_allclose(PhiB[:, m], 0.0, atol=1e-13)


@pytest.mark.parametrize("P", [2, 4])
def test_tetrahedron_projection_gradient_and_laplacian(P):
    """On a sheared affine tetrahedron: M SPD, 1^T M 1 = volume, FwdTrans o
    BwdTrans = I, L 1 = 0, the xi-gradient of the basis (chain rule through
    the collapsed map) reproduces the gradient of a physical polynomial, and
    the stiffness form of that polynomial equals the exact integral of its
    squared gradient."""
    Q = P + 2
    A = np.array([[0.9, 0.2, -0.1], [0.1, 1.1, 0.3], [-0.2, 0.05, 0.8]])
    nq = Q * (Q - 1) ** 2
    J = np.broadcast_to(A[None, :, :, None], (1, 3, 3, nq)).copy()
    ops = C.TetOps(P, Q, J, lam=0.0)
    M = ops.mass_matrix(0)
    np.linalg.cholesky(M)
    modes = C.tet_modes(P)
    tri = C.tri_modes(P)
    one = np.zeros(len(modes))
    for v in ((0, 0), (P, 0), (0, P)):
        one[modes.index((tri.index(v), 1, 0))] = 1.0
    one[-1] = 1.0
    vol = abs(np.linalg.det(A)) * 4.0 / 3.0
    assert abs(one @ M @ one - vol) < 1e-13
    c = np.random.default_rng(5).uniform(-1, 1, (1, len(modes)))
    np.testing.assert_allclose(ops.fwd(ops.bwd(c)), c, atol=1e-9)
    np.testing.assert_allclose(ops.laplacian_matrix(0) @ one, 0.0, atol=1e-12)
    xr = np.stack(C.xi_of_eta3(ops.e1, ops.e2, ops.e3))
    X = A @ xr
    x, y, z = X
    u = x * y - 0.5 * z ** 2 + 2 * x
    grad = np.stack([y + 2, x, -z])
    cu = ops.fwd(u[None])[0]
    np.testing.assert_allclose(ops.bwd(cu[None])[0], u, atol=1e-12)
    # reference gradient of the expansion, mapped to physical: grad_x = A^{-T} grad_xi
    gxi = np.stack([ops.Dt[a] @ cu for a in range(3)])
    np.testing.assert_allclose(np.linalg.solve(A.T, gxi), grad, atol=1e-11)
    exact = ops.wJ[0] @ (grad ** 2).sum(axis=0)
    assert abs(cu @ ops.laplacian_matrix(0) @ cu - exact) < 1e-12 * exact


def test_tetrahedral_mesh_volume_and_orientation():
    """The tetrahedral mesh of the unit cube: straight-sided, the volumes sum
    to one exactly; curved by the cyclic warp (which maps the cube onto
    itself), every Jacobian determinant is positive and the quadrature
    volume converges to one spectrally (its determinant is not a
    polynomial)."""
    errs = []
    for Q, amp in ((6, 0.0), (4, W.WARP_AMPLITUDE), (8, W.WARP_AMPLITUDE), (12, W.WARP_AMPLITUDE)):
        x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
        x2, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
        J = W.tet_lattice_jacobians(2, oracle.gll(Q)[0], x1, x2, amp)
        ops = C.TetOps(Q - 2, Q, J)
        assert ops.detJ.min() > 0
        errs.append(abs(ops.wJ.sum() - 1.0))
    assert errs[0] < 1e-14
    assert errs[1] < 1e-3 and errs[2] < 2e-6 and errs[3] < 1e-10
    assert errs[3] < errs[2] < errs[1]


# -------------------------------------------------------------- prisms (2.1)

@pytest.mark.parametrize("P", [1, 3, 4])
def test_prism_quadrature_and_span(P):
    """Prism rule: exact for xi_1^a xi_2^b xi_3^c with a + b <= 2P and
    c <= 2P (triangle closed form times the 1-D integral); the basis has
    (P+1)^2 (P+2)/2 modes and reproduces P_P(triangle) x P_P(line)."""
    Q = P + 2
    e1, e2, x3, W = C.prism_points(Q)
    x1, x2 = C.xi_of_eta(e1, e2)
    assert abs(W.sum() - 4.0) < 1e-14
    for a in range(2 * P + 1):
        for b in range(2 * P + 1 - a):
            for c in range(2 * P + 1):
                line = 2.0 / (c + 1) if c % 2 == 0 else 0.0
                assert abs(W @ (x1 ** a * x2 ** b * x3 ** c) - _tri_integral(a, b) * line) < 1e-12
    Phi, _, _, _ = C.prism_basis(P, e1, e2, x3)
    assert Phi.shape[1] == (P + 1) ** 2 * (P + 2) // 2
    M = Phi.T @ (W[:, None] * Phi)
    np.linalg.cholesky(M)
    for a in range(P + 1):
        for b in range(P + 1 - a):
            for c in range(P + 1):
                f = x1 ** a * x2 ** b * x3 ** c
                cf = np.linalg.solve(M, Phi.T @ (W * f))
                assert np.abs(Phi @ cf - f).max() < 1e-11, (a, b, c)


@pytest.mark.parametrize("P", [2, 4])
def test_prism_faces_gradient_and_laplacian(P):
    """Bottom and top triangle faces (xi_3 = -1, 1) carry exactly the
    triangle basis on r = 0 and r = P; on a sheared affine prism, M SPD,
    1^T M 1 = volume, L 1 = 0, the chain-rule gradient of a physical
    polynomial and its exact stiffness form."""
    rng = np.random.default_rng(2)
    e1, e2 = rng.uniform(-1, 1, (2, 15))
    T, _, _ = C.tri_basis(P, e1, e2)
    modes = C.prism_modes(P)
    for x3v, rface in ((-1.0, 0), (1.0, P)):
        Phi, _, _, _ = C.prism_basis(P, e1, e2, np.full(15, x3v))
        for m, (t, r) in enumerate(modes):
            np.testing.assert_allclose(Phi[:, m], T[:, t] if r == rface else 0.0, atol=1e-13)
    Q = P + 2
    A = np.array([[0.9, 0.2, -0.1], [0.1, 1.1, 0.3], [-0.2, 0.05, 0.8]])
    nq = Q * Q * (Q - 1)
    J = np.broadcast_to(A[None, :, :, None], (1, 3, 3, nq)).copy()
    ops = C.PrismOps(P, Q, J, lam=0.0)
    M = ops.mass_matrix(0)
    np.linalg.cholesky(M)
    tri = C.tri_modes(P)
    one = np.zeros(len(modes))
    for v in ((0, 0), (P, 0), (0, P)):
        for r in (0, P):
            one[modes.index((tri.index(v), r))] = 1.0
    assert abs(one @ M @ one - 4.0 * abs(np.linalg.det(A))) < 1e-13
    np.testing.assert_allclose(ops.laplacian_matrix(0) @ one, 0.0, atol=1e-12)
    x1, x2 = C.xi_of_eta(ops.e1, ops.e2)
    X = A @ np.stack([x1, x2, ops.e3])
    x, y, z = X
    u = x * y - 0.5 * z ** 2 + 2 * x
    grad = np.stack([y + 2, x, -z])
    cu = ops.fwd(u[None])[0]
    np.testing.assert_allclose(ops.bwd(cu[None])[0], u, atol=1e-12)
    gxi = np.stack([ops.Dt[a] @ cu for a in range(3)])
    np.testing.assert_allclose(np.linalg.solve(A.T, gxi), grad, atol=1e-11)
    exact = ops.wJ[0] @ (grad ** 2).sum(axis=0)
    assert abs(cu @ ops.laplacian_matrix(0) @ cu - exact) < 1e-12 * exact


def test_prismatic_mesh_volume_and_orientation():
    """The prismatic mesh of the unit cube: positive determinants and volume
    one, straight-sided and curved (the layered lattice is symmetric enough
    that the warp's sine terms cancel between elements, so even the curved
    volume comes out exact at every order)."""
    errs = []
    for Q, amp in ((6, 0.0), (4, W.WARP_AMPLITUDE), (8, W.WARP_AMPLITUDE), (12, W.WARP_AMPLITUDE)):
        x, _ = oracle.gll(Q)
        xr, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
        J = W.prism_lattice_jacobians(2, x, xr, x, amp)
        ops = C.PrismOps(Q - 2, Q, J)
        assert ops.detJ.min() > 0
        errs.append(abs(ops.wJ.sum() - 1.0))
    assert max(errs) < 1e-13


# ------------------------------------------------------------- pyramids (2.1)

def _pyr_integral(a, b, c):
    """Integral of xi_1^a xi_2^b xi_3^c over the reference pyramid: for each
    xi_3 the square [-1, -xi_3]^2, integrated in closed form per direction
    and then in xi_3 by exact polynomial arithmetic."""
    from numpy.polynomial import polynomial as Pn

    def side(k):   # int_{-1}^{-z} x^k dx as a polynomial in z
        coef = np.zeros(k + 2)
        coef[k + 1] = (-1.0) ** (k + 1) / (k + 1)
        coef[0] -= (-1.0) ** (k + 1) / (k + 1)
        return coef
    poly = Pn.polymul(Pn.polymul(side(a), side(b)), np.eye(c + 1)[c])
    anti = Pn.polyint(poly)
    return Pn.polyval(1.0, anti) - Pn.polyval(-1.0, anti)


@pytest.mark.parametrize("P", [1, 2, 4])
def test_pyramid_quadrature_and_span(P):
    Q = P + 2
    e1, e2, e3, W = C.pyr_points(Q)
    x1, x2, x3 = C.xi_of_eta_pyr(e1, e2, e3)
    assert abs(W.sum() - 8.0 / 3.0) < 1e-14
    for a in range(2 * P + 1):
        for b in range(2 * P + 1 - a):
            for c in range(2 * P + 1 - a - b):
                assert abs(W @ (x1 ** a * x2 ** b * x3 ** c) - _pyr_integral(a, b, c)) < 1e-12, (a, b, c)
    Phi, _, _, _ = C.pyr_basis(P, e1, e2, e3)
    assert Phi.shape[1] == (P + 1) * (P + 2) * (2 * P + 3) // 6
    M = Phi.T @ (W[:, None] * Phi)
    np.linalg.cholesky(M)
    for a in range(P + 1):
        for b in range(P + 1 - a):
            for c in range(P + 1 - a - b):
                f = x1 ** a * x2 ** b * x3 ** c
                cf = np.linalg.solve(M, Phi.T @ (W * f))
                assert np.abs(Phi @ cf - f).max() < 1e-11, (a, b, c)


@pytest.mark.parametrize("P", [2, 4])
def test_pyramid_faces(P):
    """Base face (eta_3 = -1): the r = 0 modes are the tensor-product 1-D
    modified basis, every other mode vanishes.  Triangular face xi_1 = -1:
    the p = 0 modes and the apex are exactly the triangle basis in the face's
    collapsed coordinates (eta_2, eta_3), every other mode vanishes."""
    rng = np.random.default_rng(4)
    u, v = rng.uniform(-1, 1, (2, 20))
    modes = C.pyr_modes(P)
    Phi, _, _, _ = C.pyr_basis(P, u, v, -np.ones(20))
    A1, _ = oracle.modified_basis(P, u)
    A2, _ = oracle.modified_basis(P, v)
    for m, (p, q, s, r) in enumerate(modes):
        expect = A1[:, p] * A2[:, q] if (p >= 0 and r == 0) else 0.0
        np.testing.assert_allclose(Phi[:, m], expect, atol=1e-13)
    Phi, _, _, _ = C.pyr_basis(P, -np.ones(20), u, v)
    T, _, _ = C.tri_basis(P, u, v)
    tri = C.tri_modes(P)
    for m, (p, q, s, r) in enumerate(modes):
        if p < 0:
            t = tri.index((0, P))                       # the apex: triangle vertex C
        elif p != 0:
            np.testing.assert_allclose(Phi[:, m], 0.0, atol=1e-13)
            continue
        elif q == 0:
            t = tri.index((0, r))
        elif q == P:
            t = tri.index((P, r))
        else:
            t = tri.index((q, r))
        np.testing.assert_allclose(Phi[:, m], T[:, t], atol=1e-13)


@pytest.mark.parametrize("P", [2, 4])
def test_pyramid_projection_gradient_and_laplacian(P):
    Q = P + 2
    A = np.array([[0.9, 0.2, -0.1], [0.1, 1.1, 0.3], [-0.2, 0.05, 0.8]])
    nq = Q * Q * (Q - 1)
    J = np.broadcast_to(A[None, :, :, None], (1, 3, 3, nq)).copy()
    ops = C.PyrOps(P, Q, J, lam=0.0)
    M = ops.mass_matrix(0)
    np.linalg.cholesky(M)
    modes = C.pyr_modes(P)
    one = np.zeros(len(modes))
    for m, (p, q, s, r) in enumerate(modes):
        if p < 0 or (p in (0, P) and q in (0, P) and r == 0):
            one[m] = 1.0
    assert abs(one @ M @ one - 8.0 / 3.0 * abs(np.linalg.det(A))) < 1e-13
    np.testing.assert_allclose(ops.laplacian_matrix(0) @ one, 0.0, atol=1e-12)
    X = A @ np.stack(C.xi_of_eta_pyr(ops.e1, ops.e2, ops.e3))
    x, y, z = X
    u = x * y - 0.5 * z ** 2 + 2 * x
    grad = np.stack([y + 2, x, -z])
    cu = ops.fwd(u[None])[0]
    np.testing.assert_allclose(ops.bwd(cu[None])[0], u, atol=1e-12)
    gxi = np.stack([ops.Dt[a] @ cu for a in range(3)])
    np.testing.assert_allclose(np.linalg.solve(A.T, gxi), grad, atol=1e-11)
    exact = ops.wJ[0] @ (grad ** 2).sum(axis=0)
    assert abs(cu @ ops.laplacian_matrix(0) @ cu - exact) < 1e-12 * exact


def test_pyramidal_mesh_volume_and_orientation():
    """The pyramidal mesh of the unit cube: positive determinants and volume
    one, straight-sided and curved (the warp's sine terms cancel between the
    six pyramids of each cube, so the curved volume is exact too)."""
    errs = []
    for Q, amp in ((6, 0.0), (4, W.WARP_AMPLITUDE), (8, W.WARP_AMPLITUDE), (12, W.WARP_AMPLITUDE)):
        x, _ = oracle.gll(Q)
        x3, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
        J = W.pyr_lattice_jacobians(2, x, x, x3, amp)
        ops = C.PyrOps(Q - 2, Q, J)
        assert ops.detJ.min() > 0
        errs.append(abs(ops.wJ.sum() - 1.0))
    assert max(errs) < 1e-13


# --------------------- tetrahedral meshes: C0 assembly with sorted vertex orders

def _tet_ref_coords(V, X):
    """Reference coordinates (collapsed) of physical points X (k, 3) in the
    straight-sided tetrahedron with vertices V (4, 3)."""
    M = np.stack([V[1] - V[0], V[2] - V[0], V[3] - V[0]], axis=1)
    xi = 2 * np.linalg.solve(M, (X - V[0]).T).T - 1
    e3 = xi[:, 2]
    e2 = 2 * (1 + xi[:, 1]) / (1 - xi[:, 2]) - 1
    e1 = 2 * (1 + xi[:, 0]) / (-xi[:, 1] - xi[:, 2]) - 1
    return e1, e2, e3


@pytest.mark.parametrize("P", [2, 3, 5])
def test_sorted_tetrahedral_numbering_is_continuous_across_faces(P):
    """A random global vector gathered with the sorted-vertex numbering gives
    element expansions that agree at random points of every shared face; with
    the same numbering on the positively reordered vertices (B and C swapped
    in half the elements) they do not."""
    n = 2
    l2g, ng, _ = W.tet_lattice_l2g(n, P)
    x = np.random.default_rng(P).uniform(-1, 1, ng)
    xl = oracle.gather(x, l2g)
    rng = np.random.default_rng(10 + P)
    for sorted_ids, expect_ok in ((True, True), (False, False)):
        V = W.tet_lattice_vertices(n, sorted_ids=sorted_ids)
        faces = {}
        for e in range(V.shape[0]):
            for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
                key = tuple(sorted(tuple(np.round(V[e, k] * n).astype(int)) for k in f))
                faces.setdefault(key, []).append(e)
        worst = 0.0
        for key, els in faces.items():
            if len(els) != 2:
                continue
            w = rng.dirichlet(np.ones(3), 4)
            X = w @ (np.array(key, float) / n)
            vals = []
            for e in els:
                Phi, _, _, _ = C.tet_basis(P, *_tet_ref_coords(V[e], X))
                vals.append(Phi @ xl[e])
            worst = max(worst, np.abs(vals[0] - vals[1]).max())
        assert (worst < 1e-11) == expect_ok, (sorted_ids, worst)


@pytest.mark.parametrize("P", [2, 4])
def test_sorted_tetrahedral_projection_is_exact(P):
    """Global L2 projection with the assembled mass matrix of the sorted
    tetrahedral mesh (half the elements left-handed, |det J| in the
    integrals) reproduces a polynomial of total degree P."""
    n, Q = 2, P + 2
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    x2, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    J = W.tet_lattice_jacobians(n, oracle.gll(Q)[0], x1, x2, 0.0, sorted_ids=True)
    ops = C.TetOps(P, Q, J)
    assert (ops.detJ < 0).any() and (ops.detJ > 0).any()
    l2g, ng, _ = W.tet_lattice_l2g(n, P)
    V = W.tet_lattice_vertices(n, sorted_ids=True)
    r1, r2, r3 = C.xi_of_eta3(ops.e1, ops.e2, ops.e3)
    X = (V[:, 0, :, None] + (V[:, 1] - V[:, 0])[:, :, None] * (1 + r1) / 2
         + (V[:, 2] - V[:, 0])[:, :, None] * (1 + r2) / 2 + (V[:, 3] - V[:, 0])[:, :, None] * (1 + r3) / 2)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    u = x ** (P - 1) * y - 2 * x * y * z ** (P - 2) + z ** P + 1
    mats = [ops.mass_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(u), l2g, ng)
    sol = oracle.direct_solve(mats, l2g, ng, np.zeros(ng, np.uint8), b)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g)) - u).max() < 1e-11


def test_sorted_tetrahedral_helmholtz_solve_is_exact():
    """-lap u + u = f on the unit cube, u = x(1-x)y(1-y)z(1-z) (degree 6,
    zero on the boundary), P = 6, weak right-hand side, Dirichlet boundary:
    the assembled tetrahedral solve reproduces u at every point."""
    n, P = 1, 6
    Q = P + 2
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    x2, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    J = W.tet_lattice_jacobians(n, oracle.gll(Q)[0], x1, x2, 0.0, sorted_ids=True)
    ops = C.TetOps(P, Q, J)
    l2g, ng, dm = W.tet_lattice_l2g(n, P)
    V = W.tet_lattice_vertices(n, sorted_ids=True)
    r1, r2, r3 = C.xi_of_eta3(ops.e1, ops.e2, ops.e3)
    X = (V[:, 0, :, None] + (V[:, 1] - V[:, 0])[:, :, None] * (1 + r1) / 2
         + (V[:, 2] - V[:, 0])[:, :, None] * (1 + r2) / 2 + (V[:, 3] - V[:, 0])[:, :, None] * (1 + r3) / 2)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    s = lambda t: t * (1 - t)
    u = s(x) * s(y) * s(z)
    f = 2 * (s(y) * s(z) + s(x) * s(z) + s(x) * s(y)) + u
    mats = [ops.helmholtz_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(f), l2g, ng)
    sol = oracle.direct_solve(mats, l2g, ng, dm, b)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g)) - u).max() < 1e-12


# ------------- prismatic meshes: C0 assembly of the signed triangle numbering in layers

def _prism_ref_coords(T, z0, h, X):
    """Collapsed reference coordinates (eta_1, eta_2, xi_3) of physical points
    X (k, 3) in the straight prism over the triangle T (3, 2) and the layer
    [z0, z0 + h]."""
    M = np.stack([T[1] - T[0], T[2] - T[0]], axis=1)
    xi = 2 * np.linalg.solve(M, (X[:, :2] - T[0]).T).T - 1
    e2 = xi[:, 1]
    e1 = 2 * (1 + xi[:, 0]) / (1 - xi[:, 1]) - 1
    return e1, e2, 2 * (X[:, 2] - z0) / h - 1


@pytest.mark.parametrize("P", [2, 3, 5])
def test_prismatic_numbering_is_continuous_across_faces(P):
    """A random global vector gathered with the signed prismatic numbering
    (rotated triangle vertex orders) gives element expansions that agree at
    random points of every shared vertical (quadrilateral) and horizontal
    (triangular) face; with the signs dropped they do not (from P = 3, where
    odd edge bubbles exist; at P = 2 every sign is +1)."""
    n = 2
    nt = 2 * n * n
    rot = W.tri_rotations(60 + P, nt)
    l2g, sign, ng, _ = W.prism_lattice_l2g(n, P, rot)
    T = W.prism_lattice_vertices(n, rot)
    h = 1.0 / n
    x = np.random.default_rng(P).uniform(-1, 1, ng)
    rng = np.random.default_rng(20 + P)
    # shared vertical faces: triangle edges shared by two columns, in each layer
    edge_cols = {}
    for c in range(nt):
        for a, b in ((0, 1), (1, 2), (0, 2)):
            key = tuple(sorted((tuple(np.rint(T[c, a] * n).astype(int)), tuple(np.rint(T[c, b] * n).astype(int)))))
            edge_cols.setdefault(key, []).append(c)
    if P == 2:
        assert np.all(sign == 1)
    for signed, expect_ok in ((True, True), (False, P == 2)):
        xl = oracle.gather(x, l2g, sign if signed else None)
        worst = 0.0
        for key, cols in edge_cols.items():
            if len(cols) != 2:
                continue
            a, b = (np.array(v, float) / n for v in key)
            for layer in range(n):
                t = rng.uniform(0.05, 0.95, 4)
                X = np.concatenate([a + t[:, None] * (b - a), (layer + rng.uniform(0.05, 0.95, 4))[:, None] * h], axis=1)
                vals = [C.prism_basis(P, *_prism_ref_coords(T[c], layer * h, h, X))[0] @ xl[layer * nt + c]
                        for c in cols]
                worst = max(worst, np.abs(vals[0] - vals[1]).max())
        for c in range(nt):
            for layer in range(n - 1):
                w = rng.dirichlet(np.ones(3), 4)
                X = np.concatenate([w @ T[c], np.full((4, 1), (layer + 1) * h)], axis=1)
                lo = C.prism_basis(P, *_prism_ref_coords(T[c], layer * h, h, X))[0] @ xl[layer * nt + c]
                hi = C.prism_basis(P, *_prism_ref_coords(T[c], (layer + 1) * h, h, X))[0] @ xl[(layer + 1) * nt + c]
                worst = max(worst, np.abs(lo - hi).max())
        assert (worst < 1e-11) == expect_ok, (signed, worst)


def _prism_points_xyz(ops, T, n):
    """Physical points of every prism of the straight prismatic mesh."""
    h = 1.0 / n
    nt = T.shape[0]
    xi1 = (1 + ops.e1) * (1 - ops.e2) / 2 - 1
    E = ops.nelem
    col, layer = np.arange(E) % nt, np.arange(E) // nt
    Tc = T[col]
    XY = (Tc[:, 0, :, None] * (-(xi1 + ops.e2) / 2) + Tc[:, 1, :, None] * ((1 + xi1) / 2)
          + Tc[:, 2, :, None] * ((1 + ops.e2) / 2))
    Z = layer[:, None] * h + h * (1 + ops.e3[None, :]) / 2
    return XY[:, 0], XY[:, 1], Z


@pytest.mark.parametrize("P", [2, 4])
def test_prismatic_projection_is_exact(P):
    """Global L2 projection with the assembled mass matrix of the signed
    prismatic mesh reproduces a function of the prism space (total degree P
    in x, y times degree P in z)."""
    n, Q = 2, P + 2
    rot = W.tri_rotations(70 + P, 2 * n * n)
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    g = oracle.gll(Q)[0]
    ops = C.PrismOps(P, Q, W.prism_lattice_jacobians(n, g, x1, g, 0.0, rot=rot))
    l2g, sign, ng, _ = W.prism_lattice_l2g(n, P, rot)
    x, y, z = _prism_points_xyz(ops, W.prism_lattice_vertices(n, rot), n)
    u = x ** (P - 1) * y - 2 * x * y * z ** (P - 2) + z ** P * (1 + x) + 1
    mats = [ops.mass_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(u), l2g, ng, sign)
    sol = oracle.direct_solve(mats, l2g, ng, np.zeros(ng, np.uint8), b, sign)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g, sign)) - u).max() < 1e-11 * np.abs(u).max()


def test_prismatic_helmholtz_solve_is_exact():
    """-lap u + u = f on the unit cube, u = x(1-x)y(1-y)z(1-z) (total degree
    4 in x, y, degree 2 in z, zero on the boundary), P = 4, weak right-hand
    side, Dirichlet boundary, rotated triangle vertex orders: the assembled
    prismatic solve reproduces u at every point."""
    n, P = 2, 4
    Q = P + 2
    rot = W.tri_rotations(80, 2 * n * n)
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    g = oracle.gll(Q)[0]
    ops = C.PrismOps(P, Q, W.prism_lattice_jacobians(n, g, x1, g, 0.0, rot=rot))
    l2g, sign, ng, dm = W.prism_lattice_l2g(n, P, rot)
    x, y, z = _prism_points_xyz(ops, W.prism_lattice_vertices(n, rot), n)
    s = lambda t: t * (1 - t)
    u = s(x) * s(y) * s(z)
    f = 2 * (s(y) * s(z) + s(x) * s(z) + s(x) * s(y)) + u
    mats = [ops.helmholtz_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(f), l2g, ng, sign)
    b[dm.astype(bool)] = 0.0
    sol = oracle.direct_solve(mats, l2g, ng, dm, b, sign)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g, sign)) - u).max() < 1e-12


# -------------------- pyramidal meshes: C0 assembly without signs

def _pyr_ref_coords(Vx, X):
    """Collapsed reference coordinates of physical points X (k, 3) in the
    straight pyramid with vertices Vx = (a, b, d, e)."""
    M = np.stack([Vx[1] - Vx[0], Vx[2] - Vx[0], Vx[3] - Vx[0]], axis=1)
    xi = 2 * np.linalg.solve(M, (X - Vx[0]).T).T - 1
    e3 = xi[:, 2]
    return 2 * (1 + xi[:, 0]) / (1 - e3) - 1, 2 * (1 + xi[:, 1]) / (1 - e3) - 1, e3


def _pyr_shared_faces(V, n):
    """Shared faces of the pyramidal mesh: {key: (elements, corner points)}
    for the triangular faces inside each cube and the square bases between
    cubes."""
    faces = {}
    for e in range(V.shape[0]):
        a, b, d, ap = V[e]
        c = b + d - a
        cand = [(a, b, ap), (a, d, ap), (b, c, ap), (d, c, ap), (a, b, c, d)]
        for f in cand:
            key = tuple(sorted(tuple(np.rint(np.asarray(v) * 2 * n).astype(int)) for v in f))
            faces.setdefault(key, ([], np.array(f)))[0].append(e)
    return {k: v for k, v in faces.items() if len(v[0]) == 2}


@pytest.mark.parametrize("P", [2, 3, 5])
def test_pyramidal_numbering_is_continuous_across_faces(P):
    """A random global vector gathered with the pyramidal numbering gives
    element expansions that agree at random points of every shared
    triangular face and every shared square base; without the transposition
    of the base modes where an element's b and d are swapped, the bases do
    not."""
    n = 2
    V = W.pyr_lattice_vertices(n)
    l2g, ng, _ = W.pyr_lattice_l2g(n, P)
    modes = C.pyr_modes(P)
    swapped = [int(np.flatnonzero(V[e, 1] != V[e, 0])[0]) > int(np.flatnonzero(V[e, 2] != V[e, 0])[0])
               for e in range(V.shape[0])]
    assert any(swapped) and not all(swapped)
    # the numbering without that transposition: base-face mode (p, q) of a
    # swapped element takes the global index of its own (q, p)
    broken = l2g.copy()
    pos = {(p, q): m for m, (p, q, s, r) in enumerate(modes) if r == 0 and 0 < p < P and 0 < q < P}
    for e in np.flatnonzero(swapped):
        for (p, q), m in pos.items():
            broken[e, m] = l2g[e, pos[(q, p)]]
    x = np.random.default_rng(P).uniform(-1, 1, ng)
    rng = np.random.default_rng(30 + P)
    faces = _pyr_shared_faces(V, n)
    assert any(len(f[1]) == 4 for f in faces.values()) and any(len(f[1]) == 3 for f in faces.values())
    for numbering, expect_ok in ((l2g, True), (broken, P == 2)):
        xl = oracle.gather(x, numbering)
        worst = 0.0
        for els, corners in faces.values():
            if len(corners) == 3:
                X = rng.dirichlet(np.ones(3), 4) @ corners
            else:
                s, t = rng.uniform(0.05, 0.95, (2, 4))
                X = corners[0] + s[:, None] * (corners[1] - corners[0]) + t[:, None] * (corners[3] - corners[0])
            vals = [C.pyr_basis(P, *_pyr_ref_coords(V[e], X))[0] @ xl[e] for e in els]
            worst = max(worst, np.abs(vals[0] - vals[1]).max())
        assert (worst < 1e-11) == expect_ok, (expect_ok, worst)


def _pyr_points_xyz(ops, V):
    r1, r2, r3 = C.xi_of_eta_pyr(ops.e1, ops.e2, ops.e3)
    X = (V[:, 0, :, None] + (V[:, 1] - V[:, 0])[:, :, None] * (1 + r1) / 2
         + (V[:, 2] - V[:, 0])[:, :, None] * (1 + r2) / 2 + (V[:, 3] - V[:, 0])[:, :, None] * (1 + r3) / 2)
    return X[:, 0], X[:, 1], X[:, 2]


@pytest.mark.parametrize("P", [2, 4])
def test_pyramidal_projection_is_exact(P):
    """Global L2 projection with the assembled mass matrix of the pyramidal
    mesh reproduces a polynomial of total degree P, to the rounding the
    matrix's condition number allows (1.4e5 at P = 2, 2.9e7 at P = 4; an
    error in the numbering shows as O(1))."""
    n, Q = 2, P + 2
    x, _ = oracle.gll(Q)
    x3, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    ops = C.PyrOps(P, Q, W.pyr_lattice_jacobians(n, x, x, x3, 0.0))
    l2g, ng, _ = W.pyr_lattice_l2g(n, P)
    X, Y, Z = _pyr_points_xyz(ops, W.pyr_lattice_vertices(n))
    u = X ** (P - 1) * Y - 2 * X * Y * Z ** (P - 2) + Z ** P + 1
    mats = [ops.mass_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(u), l2g, ng)
    sol = oracle.direct_solve(mats, l2g, ng, np.zeros(ng, np.uint8), b)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g)) - u).max() < 1e-9 * np.abs(u).max()


def test_pyramidal_helmholtz_solve_is_exact():
    """-lap u + u = f on the unit cube, u = x(1-x)y(1-y)z(1-z) (total degree
    6, zero on the boundary), P = 6, weak right-hand side, Dirichlet boundary:
    the assembled pyramidal solve reproduces u at every point."""
    n, P = 1, 6
    Q = P + 2
    x, _ = oracle.gll(Q)
    x3, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    ops = C.PyrOps(P, Q, W.pyr_lattice_jacobians(n, x, x, x3, 0.0))
    l2g, ng, dm = W.pyr_lattice_l2g(n, P)
    X, Y, Z = _pyr_points_xyz(ops, W.pyr_lattice_vertices(n))
    s = lambda t: t * (1 - t)
    u = s(X) * s(Y) * s(Z)
    f = 2 * (s(Y) * s(Z) + s(X) * s(Z) + s(X) * s(Y)) + u
    mats = [ops.helmholtz_matrix(e) for e in range(ops.nelem)]
    b = oracle.assemble_vector(ops.iprod(f), l2g, ng)
    b[dm.astype(bool)] = 0.0
    sol = oracle.direct_solve(mats, l2g, ng, dm, b)
    assert np.abs(ops.bwd(oracle.gather(sol, l2g)) - u).max() < 1e-12


@pytest.mark.parametrize("dim,P", [(2, 3), (3, 2), (3, 4)])
def test_helmholtz_action_equals_the_elemental_matrices(dim, P):
    """The matrix-free form of the oracle's Helmholtz (quadrature sums
    without forming H_e) equals H_e x_e with the pinned elemental matrices,
    on curved elements with per-point kappa and per-element lambda."""
    Q = P + 2
    shape = (2,) * dim
    lat = W.lattice(shape)
    J = W.element_jacobians(oracle.gll(Q)[0], lat, 0.05)
    E = lat.nelem
    rng = np.random.default_rng(dim * 10 + P)
    kap = rng.uniform(0.5, 2.0, (E, Q ** dim))
    lam = rng.uniform(0.5, 2.0, E)
    ops = oracle.ElementOps(dim, P, Q, J, kappa=kap, lam=lam)
    x = rng.uniform(-1, 1, (E, (P + 1) ** dim))
    ref = ops.helmholtz(x)
    got = ops.helmholtz_action(x)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    sub = [E - 1, 0]
    assert np.abs(ops.helmholtz_action(x[sub], sub) - ref[sub]).max() <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------- Jacobi diagonal (a7)
# The preconditioner is diag(A) of the Dirichlet-restricted assembled
# operator, with the Dirichlet rows (not unknowns) set to one.  Two pins that
# do not go through `jacobi_diagonal`'s own route (elemental diagonals
# scatter-added): brute force -- apply the masked operator, built from the
# full elemental matrices through gather / scatter-add, to every unit vector
# e_g and read row g -- and the diagonal of the sparse assembled matrix.

def _probe_diagonal(mats, l2g, ng, dm, sign=None):
    A = MaskedOperator(mats, l2g, ng, dm, sign)
    d = np.empty(ng)
    for g in range(ng):
        e = np.zeros(ng)
        e[g] = 1.0
        d[g] = A(e)[g]
    d[np.asarray(dm, bool)] = 1.0
    return d


def _check_jacobi_diagonal(mats, l2g, ng, dm, sign=None):
    d = jacobi_diagonal(mats, l2g, ng, dm, sign)
    dmb = np.asarray(dm, bool)
    assert dmb.any() and (~dmb).any()
    np.testing.assert_allclose(d, _probe_diagonal(mats, l2g, ng, dm, sign), rtol=1e-13, atol=1e-15)
    sparse = oracle.assembled_matrix(mats, l2g, ng, sign).diagonal()
    np.testing.assert_allclose(d[~dmb], sparse[~dmb], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(d[dmb], 1.0)
    assert (d[~dmb] > 0).all()


def test_jacobi_diagonal_unsigned_hex_lattice():
    P, shape = 3, (2, 2, 2)
    ops, _ = _warped_ops(shape, P, lam=1.3)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    _check_jacobi_diagonal(oracle.helmholtz_matrices(ops), l2g, ng, dm)


@pytest.mark.parametrize("P", [3, 5])
def test_jacobi_diagonal_signed_triangle_mesh(P):
    """Signs square away on the diagonal: a negated odd-parity edge bubble
    keeps its positive diagonal entry.  The mesh has negative signs."""
    n = 2
    E = 2 * n * n
    rot = W.tri_rotations(41 + P, E)
    ops, _, _ = _tri_affine_mesh(n, P, rot)
    l2g, sign, ng, dm = W.tri_lattice_l2g(n, P, rot)
    assert (np.asarray(sign) < 0).any()
    _check_jacobi_diagonal([ops.helmholtz_matrix(e) for e in range(E)], l2g, ng, dm, sign)


def test_jacobi_diagonal_ragged_mixed_order_map():
    shape = (2, 2, 1)
    perm, l2g, ng, dm, _, mats = _varp_problem(shape, [2, 4, 3, 5])
    assert len({len(g) for g in l2g}) > 1
    _check_jacobi_diagonal(mats, l2g, ng, dm)
