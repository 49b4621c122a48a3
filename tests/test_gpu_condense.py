"""GPU parity of static condensation (section 2.1): the boundary numbering,
the Jacobi preconditioner diag(S), the condensed operator S x_B against the oracle's assembled elemental Schur
complements (FP64 <= 1e-12: the interior blocks have condition numbers below
40 up to P = 6, so the dense inverse adds no more than the assembled
operator's rounding), the condensed solve against the oracle's direct solve
(true residual <= rtol recomputed by the oracle), the FP32-refined condensed
solve to an FP64 residual <= 1e-10, fewer CG iterations than the full
system, and the error paths."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import MaskedOperator, direct_solve
from oracle.condense import Condensed
from gpu_common import (FP64_RTOL, assert_close, assert_true_residual, jacobians, lib_points, nk,
                        rel_err, to_dev, torch_cuda)

pytestmark = pytest.mark.gpu


def _case(shape, P, signed=False, lam_seed=None, kappa_seed=None):
    Q = P + 2
    Jg, Jo, lat = jacobians(shape, P, W.WARP_AMPLITUDE)
    E = lat.nelem
    lam = None if lam_seed is None else np.random.default_rng(lam_seed).uniform(0.5, 2.0, E)
    kap = None if kappa_seed is None else W.uniform(kappa_seed, (E, Q ** 3), 0.5, 2.0)
    ops = oracle.ElementOps(3, P, Q, Jo, kappa=kap, lam=1.0 if lam is None else lam)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    sign = W.dof_signs(W.seed(0, 70) + P, l2g, ng) if signed else None
    m = nk()
    space = m.Space.create(3, P, Q, to_dev(Jg), kappa=to_dev(kap) if kap is not None else None)
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm),
                           lam=to_dev(lam) if lam is not None else None, lam0=1.0,
                           sign=to_dev(sign) if signed else None)
    mats = oracle.helmholtz_matrices(ops)
    return dict(P=P, l2g=l2g, ng=ng, dm=dm, sign=sign, mats=mats, space=space, sysm=sysm, ops=ops)


@pytest.mark.parametrize("P,shape,signed,lam", [(2, (3, 2, 2), False, None), (3, (3, 2, 2), True, 4),
                                                (4, (2, 3, 2), False, 5), (5, (2, 2, 2), True, None),
                                                (6, (2, 2, 2), False, 6)])
def test_condensed_operator_matches_oracle(P, shape, signed, lam):
    torch = torch_cuda()
    c = _case(shape, P, signed, lam)
    ref = Condensed(c["mats"], c["l2g"], c["ng"], c["dm"], 3, P, c["sign"])
    nb, bmap = c["sysm"].condense()
    assert nb == ref.bdofs.size
    np.testing.assert_array_equal(bmap.cpu().numpy(), ref.bdofs)
    # a second call reuses the built form; the preconditioner is diag(S)
    nb2, _, dS = c["sysm"].condense(with_map=False, with_diag=True)
    assert nb2 == nb
    dref = np.where(ref.bfree, ref.S.diagonal(), 1.0)
    assert_close(dS.cpu().numpy(), dref, FP64_RTOL, f"diag(S) P={P}")
    for k in range(2):
        xb = W.uniform(W.seed(0, 71) + 10 * P + k, nb)
        y = c["sysm"].condensed_apply(to_dev(xb)).cpu().numpy()
        assert_close(y, ref.apply(xb), FP64_RTOL, f"condensed apply P={P} call {k}")
    del torch


@pytest.mark.parametrize("P", [3, 6])
def test_condensed_operator_repeatable_to_rounding(P):
    """Repeated applications of S agree to rounding: the boundary scatter adds
    atomically, so the order of its additions may change between launches, and
    nothing else.  Two condensed solves of one right-hand side both meet rtol;
    the rounding differences steer the boundary CG a little (measured: 197 and
    199 iterations at P = 3), so their counts agree within 3% and their
    solutions within what two residuals of rtol allow for this small,
    well-conditioned system."""
    torch_cuda()
    m = nk()
    c = _case((3, 3, 2), P, signed=True)
    nb, _ = c["sysm"].condense(with_map=False)
    xb = to_dev(W.uniform(W.seed(0, 72) + P, nb))
    y0 = c["sysm"].condensed_apply(xb).cpu().numpy()
    for k in range(3):
        y = c["sysm"].condensed_apply(xb).cpu().numpy()
        assert rel_err(y, y0) <= 1e-14, (P, k, rel_err(y, y0))
    b = W.uniform(W.seed(0, 75) + P, c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    x1, i1 = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED)
    x2, i2 = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED)
    for i in (i1, i2):
        assert i[0]["status"] == 0 and i[0]["rel_resid"] <= 1e-10, i[0]
    assert abs(i1[0]["iters"] - i2[0]["iters"]) <= max(2, 0.03 * i1[0]["iters"]), (i1[0]["iters"], i2[0]["iters"])
    assert rel_err(x2.cpu().numpy(), x1.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("P,shape,signed,kappa", [(2, (3, 3, 2), False, None), (4, (3, 2, 2), True, None),
                                                  (6, (2, 2, 2), False, None), (5, (2, 3, 2), True, 12)])
def test_condensed_solve_matches_direct_solve(P, shape, signed, kappa):
    """NK_SOLVE_CONDENSED to 1e-12: the oracle's residual of the returned x,
    and x against the oracle's sparse direct solve (error <= cond(A) rtol);
    the last case has a per-point diffusion coefficient kappa in [0.5, 2]."""
    torch_cuda()
    m = nk()
    c = _case(shape, P, signed, lam_seed=7, kappa_seed=kappa)
    b = W.uniform(W.seed(0, 72) + P, c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    x, info = c["sysm"].solve(to_dev(b), rtol=1e-12, maxit=20000, mode=m.SOLVE_CONDENSED)
    xs = x.cpu().numpy()
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"], c["sign"])
    assert_true_residual(info[0], 1e-12, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, f"P={P}")
    assert info[0]["outer_iters"] >= 1 and info[0]["iters"] >= 1
    xref = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b, c["sign"])
    assert rel_err(xs, xref) < 1e-8
    # the condensed oracle agrees with the direct one (same x)
    xo = oracle.condensed_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b, 3, P, c["sign"])
    assert rel_err(xs, xo) < 1e-8


@pytest.mark.parametrize("P,shape,signed", [(3, (3, 3, 2), True), (6, (2, 2, 3), False)])
def test_condensed_f32_refined_true_residual(P, shape, signed):
    """NK_SOLVE_CONDENSED_F32_REFINED: the boundary system in FP32 (FP32
    factors and inverses) with FP64 reliable updates; the FP64 residual of the
    returned x, recomputed by the oracle, is <= 1e-10, and x agrees with the
    direct solve to cond(A) 1e-10."""
    torch_cuda()
    m = nk()
    c = _case(shape, P, signed, lam_seed=8)
    b = W.uniform(W.seed(0, 75) + P, c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    x, info = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED_F32_REFINED)
    xs = x.cpu().numpy()
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"], c["sign"])
    assert_true_residual(info[0], 1e-10, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, f"P={P}")
    xref = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b, c["sign"])
    assert rel_err(xs, xref) < 1e-5
    # the FP64 condensed solve of the same system after the FP32 one
    x64, info64 = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED)
    assert info64[0]["status"] == 0 and rel_err(x64.cpu().numpy(), xref) < 1e-5


@pytest.mark.parametrize("shape,orders", [((3, 2, 2), [2, 5, 3, 4, 2, 6, 3, 3, 5, 2, 4, 6]),
                                          ((4, 3, 2), [3, 6, 2, 4, 5, 6, 2, 3, 4, 5, 6, 2,
                                                       3, 3, 4, 4, 5, 5, 6, 6, 2, 2, 4, 6])])
def test_variable_order_condensation(shape, orders):
    """Section 4.2's spatially variable order (minimum-rule map, orders 2..6):
    the boundary numbering, diag(S) and S x against the oracle's per-element
    condensation, and both condensed solves against the direct solve."""
    torch_cuda()
    m = nk()
    from test_gpu_solve import _varp_case
    c = _varp_case(shape, orders)
    ref = Condensed(c["mats"], c["l2g"], c["ng"], c["dm"], 3, None)
    nb, bmap, dS = c["sysm"].condense(with_diag=True)
    assert nb == ref.bdofs.size
    np.testing.assert_array_equal(bmap.cpu().numpy(), ref.bdofs)
    assert_close(dS.cpu().numpy(), np.where(ref.bfree, ref.S.diagonal(), 1.0), FP64_RTOL, "varp diag(S)")
    xb = W.uniform(W.seed(0, 76), nb)
    assert_close(c["sysm"].condensed_apply(to_dev(xb)).cpu().numpy(), ref.apply(xb), FP64_RTOL,
                 "varp condensed apply")
    b = c["b"]
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"])
    xd = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b)
    for mode, rtol, tag in ((m.SOLVE_CONDENSED, 1e-12, "condensed"),
                            (m.SOLVE_CONDENSED_F32_REFINED, 1e-10, "condensed f32-refined")):
        x, info = c["sysm"].solve(to_dev(b), rtol=rtol, maxit=20000, mode=mode)
        xs = x.cpu().numpy()
        assert_true_residual(info[0], rtol, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, tag)
        assert rel_err(xs, xd) < (1e-8 if rtol < 1e-11 else 1e-5), tag


def test_condensed_solve_takes_fewer_iterations():
    """On a 4^3 curved lattice at P = 4 the boundary system needs fewer
    Jacobi-PCG iterations than the full one to the same full residual."""
    torch_cuda()
    m = nk()
    c = _case((4, 4, 4), 4)
    b = W.uniform(W.seed(0, 73), c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    xf, inf_f = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000)
    xc, inf_c = c["sysm"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED)
    assert inf_c[0]["status"] == 0 and inf_c[0]["rel_resid"] <= 1e-10
    assert inf_c[0]["iters"] < inf_f[0]["iters"], (inf_c[0]["iters"], inf_f[0]["iters"])
    assert rel_err(xc.cpu().numpy(), xf.cpu().numpy()) < 1e-6


def test_condensed_solve_initial_guess_and_zero_rhs():
    """An exact initial guess returns at once (no boundary solve); a zero
    right-hand side gives x = 0."""
    torch = torch_cuda()
    m = nk()
    c = _case((3, 2, 2), 3)
    b = W.uniform(W.seed(0, 74), c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    x, info = c["sysm"].solve(to_dev(b), rtol=1e-12, maxit=20000, mode=m.SOLVE_CONDENSED)
    x2, info2 = c["sysm"].solve(to_dev(b), x=x.clone(), rtol=1e-10, maxit=20000, mode=m.SOLVE_CONDENSED)
    assert info2[0]["status"] == 0 and info2[0]["iters"] == 0 and info2[0]["outer_iters"] == 0
    z = torch.zeros(c["ng"], dtype=torch.float64, device="cuda")
    x0, info0 = c["sysm"].solve(z, rtol=1e-10, maxit=100, mode=m.SOLVE_CONDENSED)
    assert info0[0]["status"] == 0 and float(x0.abs().max()) == 0.0


def test_condensed_error_paths():
    torch = torch_cuda()
    m = nk()
    # P = 1: no interior modes; a variable-order space with an order-1 group
    c1 = _case((2, 2, 2), 1)
    with pytest.raises(m.NkError) as ei:
        c1["sysm"].condense()
    assert ei.value.status == m.NK_EUNSUPPORTED
    from test_gpu_solve import _varp_case
    cv = _varp_case((2, 2, 1), [1, 3, 2, 4])
    with pytest.raises(m.NkError) as ei:
        cv["sysm"].condense()
    assert ei.value.status == m.NK_EUNSUPPORTED
    # condensed apply before the condensed form exists
    c = _case((2, 2, 1), 2)
    with pytest.raises(m.NkError) as ei:
        c["sysm"].condensed_apply(torch.zeros(8, dtype=torch.float64, device="cuda"))
    assert ei.value.status == m.NK_EINVAL
    # an interior mode sharing its DOF with another element
    l2g = c["l2g"].copy()
    inner = np.flatnonzero(oracle.interior_modes(3, 2))[0]
    l2g[1, inner] = l2g[0, inner]
    bad = m.System.create(c["space"], c["ng"], to_dev(l2g), to_dev(c["dm"]), lam0=1.0)
    with pytest.raises(m.NkError) as ei:
        bad.condense()
    assert ei.value.status == m.NK_EUNSUPPORTED
    # the batched solve does not take the condensed mode
    b = torch.zeros(c["ng"], dtype=torch.float64, device="cuda")
    with pytest.raises(m.NkError) as ei:
        m.solve_batched([c["sysm"]], [b], mode=m.SOLVE_CONDENSED)
    assert ei.value.status == m.NK_EUNSUPPORTED
    # an iteration budget too small for the tolerance: NK_ENOCONV, budget respected
    c3 = _case((3, 3, 2), 4)
    b3 = W.uniform(W.seed(0, 77), c3["ng"])
    b3[c3["dm"].astype(bool)] = 0.0
    for mode in (m.SOLVE_CONDENSED, m.SOLVE_CONDENSED_F32_REFINED):
        x, info = c3["sysm"].solve(to_dev(b3), rtol=1e-12, maxit=3, mode=mode, raise_on_fail=False)
        assert info[0]["status"] == m.NK_ENOCONV and info[0]["iters"] <= 3
        assert info[0]["rel_resid"] > 1e-12


@pytest.mark.parametrize("P", [4, 6])
def test_full_size_24c_condensed_solve_sampled_residuals(P):
    """The 24^3 curved-hex problem of the benchmark solved by condensation to
    1e-10: the library's true residual, the oracle's residual rows at a
    seeded sample of free DOFs (lattice vertices shared by eight elements,
    and random DOFs, interior ones included) each <= 1e-10 ||b||_2, and
    agreement with the full FP64 CG solution."""
    m = nk()
    torch_cuda()
    shape, Q = (24, 24, 24), P + 2
    lat = W.lattice(shape)
    space = m.Space.create(3, P, Q, to_dev(W.element_jacobians(lib_points(P, Q), lat, W.WARP_AMPLITUDE)))
    l2g, ng, dm = W.lattice_l2g(shape, P)
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam0=1.0)
    fixed = dm.astype(bool)
    b = W.uniform(W.seed(2, 1) + P, ng)
    b[fixed] = 0.0
    xc, info = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000, mode=m.SOLVE_CONDENSED)
    assert info[0]["status"] == 0 and info[0]["rel_resid"] <= 1e-10
    xr, infor = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000, mode=m.SOLVE_CONDENSED_F32_REFINED)
    assert infor[0]["status"] == 0 and infor[0]["rel_resid"] <= 1e-10
    xf, infof = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000)
    assert info[0]["iters"] < infof[0]["iters"]
    xs = xc.cpu().numpy().copy()
    xs[fixed] = 0.0
    assert rel_err(xs, xf.cpu().numpy()) < 1e-5
    assert rel_err(xr.cpu().numpy(), xf.cpu().numpy()) < 1e-5
    G = [s * P + 1 for s in shape]
    free = np.flatnonzero(~fixed)
    gx, gy, gz = free % G[0], (free // G[0]) % G[1], free // (G[0] * G[1])
    verts = free[(gx % P == 0) & (gy % P == 0) & (gz % P == 0)]
    inner = free[(gx % P != 0) & (gy % P != 0) & (gz % P != 0)]
    rng = np.random.default_rng(50 + P)
    sample = np.unique(np.concatenate([rng.choice(verts, 4, replace=False), rng.choice(inner, 4, replace=False),
                                       rng.choice(free, 6, replace=False)]))
    hits = {int(g): np.argwhere(l2g == g) for g in sample}
    elems = np.unique(np.concatenate([h[:, 0] for h in hits.values()]))
    pos = {int(e): k for k, e in enumerate(elems)}
    Jo = W.element_jacobians(oracle.gll(Q)[0], W.Lattice(lat.shape, lat.h, lat.origins[elems]), W.WARP_AMPLITUDE)
    ops = oracle.ElementOps(3, P, Q, Jo, lam=1.0)
    bn = np.linalg.norm(b)
    for xv, tag in ((xs, "condensed"), (xr.cpu().numpy(), "condensed f32-refined")):
        xv = xv.copy()
        xv[fixed] = 0.0
        y = ops.helmholtz_action(xv[l2g[elems]])
        for g, h in hits.items():
            Ag = sum(y[pos[int(e)], mm] for e, mm in h)
            assert abs(b[g] - Ag) <= 1e-10 * bn, (tag, g, abs(b[g] - Ag) / bn)
