"""Pins for the oracle's static condensation (section 2.1: the assembled system
condensed onto the elemental boundary DOFs, interiors recovered per element).

Each check goes through a route the condensed code does not use: the full
sparse direct solve, block elimination of the assembled matrix with no
elemental structure, the closed-form count of boundary DOFs on a lattice, the
P = 1 special case, and the energy-minimising property of the Schur
complement."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import direct_solve
from oracle.condense import Condensed, condensed_solve, global_schur, interior_modes


def _system(shape, P, lam=1.0, amp=0.05):
    Q = P + 2
    lat = W.lattice(shape)
    x, _ = oracle.gll(Q)
    ops = oracle.ElementOps(len(shape), P, Q, W.element_jacobians(x, lat, amp), lam=lam)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    return ops, oracle.helmholtz_matrices(ops), l2g, ng, dm


@pytest.mark.parametrize("dim,P", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 5)])
def test_interior_mode_count_and_position(dim, P):
    """(P-1)^dim interior modes, none with a 1-D index 0 or P."""
    m = interior_modes(dim, P)
    assert m.sum() == max(P - 1, 0) ** dim
    idx = np.indices((P + 1,) * dim).reshape(dim, -1)
    assert not np.any(m & np.any((idx == 0) | (idx == P), axis=0))


@pytest.mark.parametrize("shape,P", [((3, 2, 2), 3), ((2, 2, 1), 4), ((4, 3), 5)])
def test_boundary_count_closed_form(shape, P):
    """On a lattice the boundary DOFs are all DOFs but the E (P-1)^d element
    interiors: prod(N_c P + 1) - E (P-1)^d."""
    ops, mats, l2g, ng, dm = _system(shape, P)
    c = Condensed(mats, l2g, ng, dm, len(shape), P)
    E = int(np.prod(shape))
    assert c.bdofs.size == int(np.prod([s * P + 1 for s in shape])) - E * (P - 1) ** len(shape)


@pytest.mark.parametrize("shape,P,signed", [((3, 2, 2), 3, False), ((2, 2, 2), 4, True),
                                            ((3, 3), 5, True)])
def test_condensed_operator_is_the_global_schur_complement(shape, P, signed):
    """The sum of elemental Schur complements equals the Schur complement of
    the assembled matrix onto its boundary DOFs, eliminated globally."""
    ops, mats, l2g, ng, dm = _system(shape, P)
    sign = W.dof_signs(7, l2g, ng) if signed else None
    c = Condensed(mats, l2g, ng, dm, len(shape), P, sign)
    B, Sg = global_schur(mats, l2g, ng, l2g[:, interior_modes(len(shape), P)].ravel(), sign)
    np.testing.assert_array_equal(B, c.bdofs)
    Sc = c.S.toarray()
    assert np.abs(Sc - Sg).max() <= 1e-12 * np.abs(Sg).max()


@pytest.mark.parametrize("shape,P,signed", [((3, 2, 2), 2, False), ((2, 2, 2), 5, True),
                                            ((4, 3), 6, False)])
def test_condensed_solve_equals_direct_solve(shape, P, signed):
    """Boundary solve plus interior recovery reproduces the full direct solve."""
    ops, mats, l2g, ng, dm = _system(shape, P)
    sign = W.dof_signs(3, l2g, ng) if signed else None
    b = W.uniform(11, ng)
    b[dm.astype(bool)] = 0
    xd = direct_solve(mats, l2g, ng, dm, b, sign)
    xc = condensed_solve(mats, l2g, ng, dm, b, len(shape), P, sign)
    assert np.abs(xc - xd).max() <= 1e-11 * np.abs(xd).max()


def test_linear_order_has_nothing_to_condense():
    """P = 1: no interior modes, S is the assembled matrix itself."""
    ops, mats, l2g, ng, dm = _system((3, 2, 2), 1)
    c = Condensed(mats, l2g, ng, dm, 3, 1)
    A = oracle.assembled_matrix(mats, l2g, ng).toarray()
    np.testing.assert_array_equal(c.bdofs, np.arange(ng))
    assert np.abs(c.S.toarray() - A).max() <= 1e-15 * np.abs(A).max()


def test_schur_energy_is_the_minimum_over_interiors():
    """x_B . S x_B = min over interior values of x . A x, attained at the
    harmonic extension: every other interior choice has higher energy."""
    shape, P = (2, 2, 1), 3
    ops, mats, l2g, ng, dm = _system(shape, P)
    c = Condensed(mats, l2g, ng, dm, 3, P)
    A = oracle.assembled_matrix(mats, l2g, ng)
    xb = W.uniform(5, c.bdofs.size)
    eS = xb @ (c.S @ xb)
    x = c.interior_solution(xb * c.bfree + 0.0, np.zeros(ng))   # b = 0: harmonic extension
    xb0 = np.where(c.bfree, xb, 0.0)
    eS0 = xb0 @ (c.S @ xb0)
    assert abs(x @ (A @ x) - eS0) <= 1e-12 * abs(eS0)
    rng = np.random.default_rng(9)
    ii = l2g[:, interior_modes(3, P)].ravel()
    for _ in range(5):
        y = x.copy()
        y[ii] += 1e-3 * rng.standard_normal(ii.size)
        assert y @ (A @ y) > eS0
    assert eS > 0


def test_shared_interior_dof_is_rejected():
    """A map whose interior mode shares its DOF with another element cannot be
    condensed."""
    ops, mats, l2g, ng, dm = _system((2, 1, 1), 2)
    bad = l2g.copy()
    m = np.flatnonzero(interior_modes(3, 2))[0]
    bad[1, m] = bad[0, m]
    with pytest.raises(ValueError):
        Condensed(mats, bad, ng, dm, 3, 2)


def test_variable_order_condensation_equals_direct_solve_and_global_schur():
    """Section 4.2's spatially variable order (minimum-rule map, orders 2..6):
    the per-element condensation reproduces the direct solve, and its S is
    the assembled matrix's Schur complement onto the boundary DOFs."""
    from test_oracle import _varp_problem
    shape = (3, 2, 2)
    orders = [2, 5, 3, 4, 2, 6, 3, 3, 5, 2, 4, 6]
    perm, l2g, ng, dm, groups, mats = _varp_problem(shape, orders)
    c = Condensed(mats, l2g, ng, dm, 3, None)
    inner = np.concatenate([np.asarray(g)[interior_modes(3, int(round(len(g) ** (1 / 3))) - 1)]
                            for g in l2g])
    assert c.bdofs.size == ng - inner.size
    B, Sg = global_schur(mats, l2g, ng, inner)
    np.testing.assert_array_equal(B, c.bdofs)
    assert np.abs(c.S.toarray() - Sg).max() <= 1e-12 * np.abs(Sg).max()
    b = W.uniform(21, ng)
    b[dm.astype(bool)] = 0
    xd = direct_solve(mats, l2g, ng, dm, b)
    xc = c.solve(b)
    assert np.abs(xc - xd).max() <= 1e-11 * np.abs(xd).max()
