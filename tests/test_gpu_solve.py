"""GPU parity of the assembled operator, assembly helpers and CG solves.

Assembled operator R A R x (FP64 <= 1e-12, FP32 <= 2e-6), Jacobi diagonal,
gather and scatter against the oracle; FP64 PCG against the oracle's sparse
direct solve; FP32-refined PCG to a true FP64 residual <= 1e-10 recomputed by
the oracle; many independent systems solved as one batch against individual
oracle solves; error paths (maxit, breakdown)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import MaskedOperator, jacobi_diagonal, direct_solve
from gpu_common import (FP32_RTOL, FP64_RTOL, assert_close, assert_true_residual, jacobians, nk,
                        rel_err, to_dev, torch_cuda)

pytestmark = pytest.mark.gpu


def _problem(shape, P, amp=W.WARP_AMPLITUDE, lam_seed=None):
    Q = P + 2
    Jg, Jo, lat = jacobians(shape, P, amp)
    E = lat.nelem
    lam = None if lam_seed is None else np.random.default_rng(lam_seed).uniform(0.5, 2.0, E)
    ops = oracle.ElementOps(3, P, Q, Jo, lam=1.0 if lam is None else lam)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    return dict(P=P, Q=Q, Jg=Jg, ops=ops, lat=lat, l2g=l2g, ng=ng, dm=dm, lam=lam)


def _gpu_system(pb):
    m = nk()
    space = m.Space.create(3, pb["P"], pb["Q"], to_dev(pb["Jg"]))
    lam = to_dev(pb["lam"]) if pb["lam"] is not None else None
    sysm = m.System.create(space, pb["ng"], to_dev(pb["l2g"]), to_dev(pb["dm"]), lam=lam, lam0=1.0)
    return space, sysm


def _rhs(pb):
    """Weak right-hand side of the manufactured sine (oracle side)."""
    ops, lat = pb["ops"], pb["lat"]
    U, dU = W.manufactured_ref_gradient(ops.x, lat)
    b = oracle.assemble_vector(ops.weak_rhs(U, dU), pb["l2g"], pb["ng"])
    b[pb["dm"].astype(bool)] = 0.0
    return b


@pytest.mark.parametrize("P,shape", [(2, (3, 2, 2)), (4, (3, 3, 2)), (6, (2, 2, 2))])
def test_assembled_operator_diag_gather_scatter(P, shape):
    torch = torch_cuda()
    m = nk()
    pb = _problem(shape, P, lam_seed=3)
    mats = oracle.helmholtz_matrices(pb["ops"])
    A = MaskedOperator(mats, pb["l2g"], pb["ng"], pb["dm"])
    space, sysm = _gpu_system(pb)
    x = np.random.default_rng(1).uniform(-1, 1, pb["ng"])
    ref = A(x)
    y = sysm.apply(to_dev(x)).cpu().numpy()
    assert_close(y, ref, FP64_RTOL, f"apply P={P}")
    y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
    assert_close(y32, ref, FP32_RTOL, f"apply32 P={P}")
    d = sysm.diagonal().cpu().numpy()
    assert_close(d, jacobi_diagonal(mats, pb["l2g"], pb["ng"], pb["dm"]), FP64_RTOL, "diag")
    xl = sysm.gather(to_dev(x)).cpu().numpy()
    np.testing.assert_array_equal(xl, oracle.gather(x, pb["l2g"]).ravel())
    yl = np.random.default_rng(2).uniform(-1, 1, xl.size)
    bref = oracle.assemble_vector(yl.reshape(pb["lat"].nelem, -1), pb["l2g"], pb["ng"])
    bref[pb["dm"].astype(bool)] = 0.0
    assert_close(sysm.assemble(to_dev(yl)).cpu().numpy(), bref, 1e-14, "assemble")


@pytest.mark.parametrize("P", [2, 4, 6])
def test_cg_f64_matches_direct_solve(P):
    torch_cuda()
    pb = _problem((3, 3, 3) if P < 6 else (2, 2, 3), P)
    b = _rhs(pb)
    mats = oracle.helmholtz_matrices(pb["ops"])
    xref = direct_solve(mats, pb["l2g"], pb["ng"], pb["dm"], b)
    _, sysm = _gpu_system(pb)
    x, info = sysm.solve(to_dev(b), rtol=1e-12, maxit=20000)
    assert info[0]["iters"] > 5
    xs = x.cpu().numpy()
    # the oracle's own residual of the GPU solution, and the solution error,
    # which is bounded by cond(A) * rtol (cond ~ 1e3 at P = 6)
    A = MaskedOperator(mats, pb["l2g"], pb["ng"], pb["dm"])
    assert_true_residual(info[0], 1e-12, A, mats, pb["l2g"], pb["ng"], pb["dm"], xs, b, f"P={P}")
    assert rel_err(xs, xref) < 1e-8


@pytest.mark.parametrize("P", [4, 6])
def test_cg_f32_refined_true_residual(P):
    """FP32 operator and vectors inside FP64 refinement: the FP64 residual of
    the returned x, recomputed by the oracle, is <= 1e-10."""
    m = nk()
    torch_cuda()
    pb = _problem((3, 3, 2), P, lam_seed=9)
    b = _rhs(pb)
    mats = oracle.helmholtz_matrices(pb["ops"])
    A = MaskedOperator(mats, pb["l2g"], pb["ng"], pb["dm"])
    _, sysm = _gpu_system(pb)
    x, info = sysm.solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_F32_REFINED)
    xs = x.cpu().numpy()
    assert_true_residual(info[0], 1e-10, A, mats, pb["l2g"], pb["ng"], pb["dm"], xs, b, f"P={P}")
    assert info[0]["outer_iters"] >= 2
    xref = direct_solve(mats, pb["l2g"], pb["ng"], pb["dm"], b)
    # the error is bounded by cond(A) * 1e-10 (cond ~ 1e4 at P = 6)
    assert rel_err(xs, xref) < 1e-5


def test_cg_initial_guess_and_zero_rhs():
    torch = torch_cuda()
    pb = _problem((2, 2, 2), 3)
    b = _rhs(pb)
    xref = direct_solve(oracle.helmholtz_matrices(pb["ops"]), pb["l2g"], pb["ng"], pb["dm"], b)
    _, sysm = _gpu_system(pb)
    x0 = to_dev(xref + 1e-3 * np.random.default_rng(0).standard_normal(pb["ng"]))
    x, info = sysm.solve(to_dev(b), x=x0, rtol=1e-12)
    assert rel_err(x.cpu().numpy(), xref) < 1e-8      # cond(A) * rtol
    # Dirichlet entries of the initial guess are forced to zero
    assert np.all(x.cpu().numpy()[pb["dm"].astype(bool)] == 0.0)
    z, info = sysm.solve(torch.zeros(pb["ng"], dtype=torch.float64, device="cuda"), rtol=1e-10)
    assert info[0]["iters"] == 0 and np.all(z.cpu().numpy() == 0.0)


def test_cg_maxit_reports_noconv():
    m = nk()
    torch_cuda()
    pb = _problem((3, 3, 3), 4)
    b = _rhs(pb)
    _, sysm = _gpu_system(pb)
    x, info = sysm.solve(to_dev(b), rtol=1e-14, maxit=7, raise_on_fail=False)
    assert info[0]["status"] == m.NK_ENOCONV
    assert info[0]["iters"] == 7


def test_cg_breakdown_on_indefinite_operator():
    """lambda = -1e4 makes A indefinite: breakdown or no convergence is
    reported, and the call returns normally."""
    m = nk()
    torch_cuda()
    pb = _problem((2, 2, 2), 3)
    b = _rhs(pb)
    space = m.Space.create(3, pb["P"], pb["Q"], to_dev(pb["Jg"]))
    sysm = m.System.create(space, pb["ng"], to_dev(pb["l2g"]), to_dev(pb["dm"]), lam0=-1e4)
    with pytest.raises(m.NkError) as ei:
        sysm.solve(to_dev(b), rtol=1e-12, maxit=500)
    assert ei.value.status in (5, 6)


def test_batched_independent_systems():
    """Systems of different sizes in one batched solve (one persistent
    operator launch per iteration, per-system CG scalars) equal the oracle's
    individual direct solves."""
    m = nk()
    torch = torch_cuda()
    P, Q = 3, 5
    boxes = [(1, 1, 1), (2, 3, 1), (3, 3, 3), (2, 2, 2), (4, 1, 2)]
    jg, l2gs, dms, bs, refs = [], [], [], [], []
    eoff, doff = [0], [0]
    for bx in boxes:
        pb = _problem(bx, P)
        b = _rhs(pb)
        refs.append(direct_solve(oracle.helmholtz_matrices(pb["ops"]), pb["l2g"], pb["ng"], pb["dm"], b))
        jg.append(pb["Jg"])
        l2gs.append(pb["l2g"] + doff[-1])
        dms.append(pb["dm"])
        bs.append(b)
        eoff.append(eoff[-1] + pb["lat"].nelem)
        doff.append(doff[-1] + pb["ng"])
    space = m.Space.create(3, P, Q, to_dev(np.concatenate(jg)))
    sysm = m.System.create_batched(space, eoff, doff, to_dev(np.concatenate(l2gs).astype(np.int32)),
                                   to_dev(np.concatenate(dms)), lam0=1.0)
    for mode, tol in ((m.SOLVE_F64, 1e-12), (m.SOLVE_F32_REFINED, 1e-10)):
        x, info = sysm.solve(to_dev(np.concatenate(bs)), rtol=tol, mode=mode)
        xs = x.cpu().numpy()
        assert len(info) == len(boxes)
        for k, ref in enumerate(refs):
            assert info[k]["status"] == 0 and info[k]["rel_resid"] <= tol
            err = rel_err(xs[doff[k]:doff[k + 1]], ref)
            assert err < (1e-9 if mode == m.SOLVE_F64 else 1e-6), (k, mode, err)


@pytest.mark.parametrize("P", [4, 6])
def test_assembled_operator_and_cg_matrix_core_variant(P):
    """The matrix-core (MFMA) variant of the assembled operator, selected as
    the last Helmholtz tile, against the oracle; and a CG solve with it."""
    torch = torch_cuda()
    m = nk()
    nt = m.tile_count(m.OP_HELM, 3, P)
    assert m.tile_config(m.OP_HELM, 3, P, m.F64) != ""
    try:
        for dt in (m.F64, m.F32):
            m.set_tile_config(m.OP_HELM, 3, P, dt, nt - 1)
        assert m.tile_config(m.OP_HELM, 3, P, m.F64).startswith("mfma")
        pb = _problem((3, 2, 2), P, lam_seed=5)
        mats = oracle.helmholtz_matrices(pb["ops"])
        A = MaskedOperator(mats, pb["l2g"], pb["ng"], pb["dm"])
        _, sysm = _gpu_system(pb)
        x = np.random.default_rng(3).uniform(-1, 1, pb["ng"])
        ref = A(x)
        assert_close(sysm.apply(to_dev(x)).cpu().numpy(), ref, FP64_RTOL, f"mfma apply P={P}")
        y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
        assert_close(y32, ref, FP32_RTOL, f"mfma apply32 P={P}")
        b = _rhs(pb)
        xs, info = sysm.solve(to_dev(b), rtol=1e-12)
        assert_true_residual(info[0], 1e-12, A, mats, pb["l2g"], pb["ng"], pb["dm"],
                             xs.cpu().numpy(), b, f"mfma P={P}")
        xr, info = sysm.solve(to_dev(b), rtol=1e-10, mode=m.SOLVE_F32_REFINED)
        assert_true_residual(info[0], 1e-10, A, mats, pb["l2g"], pb["ng"], pb["dm"],
                             xr.cpu().numpy(), b, f"mfma refined P={P}")
    finally:
        for dt in (m.F64, m.F32):
            m.set_tile_config(m.OP_HELM, 3, P, dt, 0)


# ------------------------------------------- mixed-order (conforming) systems

def _varp_case(shape, orders, amp=W.WARP_AMPLITUDE):
    """Mixed-order space (groups by ascending order), its conforming map and
    the oracle's elemental matrices in the same element order."""
    from gpu_common import lib_points
    m = nk()
    perm, l2g, ng, dm = W.varp_lattice_l2g(shape, orders)
    lat = W.lattice(shape)
    ords = np.asarray(orders)[perm]
    Ps = sorted(set(ords.tolist()))
    jacs, mats, rhs_loc = [], [], []
    for P in Ps:
        idx = perm[ords == P]
        Q = P + 2
        sub = W.Lattice(lat.shape, lat.h, lat.origins[idx])
        jacs.append(to_dev(np.ascontiguousarray(W.element_jacobians(lib_points(P, Q), sub, amp))))
        ops = oracle.ElementOps(3, P, Q, W.element_jacobians(oracle.gll(Q)[0], sub, amp), lam=1.0)
        mats += oracle.helmholtz_matrices(ops)
        U, dU = W.manufactured_ref_gradient(ops.x, sub)
        rhs_loc += list(ops.weak_rhs(U, dU))
    space = m.Space.create_varp(3, Ps, [P + 2 for P in Ps], jacs)
    sysm = m.System.create(space, ng, to_dev(np.concatenate(l2g)), to_dev(dm), lam0=1.0)
    b = oracle.assemble_vector(rhs_loc, l2g, ng)
    b[dm.astype(bool)] = 0.0
    return dict(space=space, sysm=sysm, l2g=l2g, ng=ng, dm=dm, mats=mats, b=b)


@pytest.mark.parametrize("shape,orders", [((3, 2, 2), [2, 5, 3, 4, 2, 6, 3, 3, 5, 2, 4, 6]),
                                          ((2, 2, 2), [1, 8, 2, 7, 3, 6, 4, 10])])
def test_mixed_order_assembled_operator_and_solves(shape, orders):
    """Conforming variable-order system (minimum rule): the assembled operator
    against the oracle's, FP64 and FP32-refined CG against the sparse direct
    solve (residual recomputed by the oracle), gather and assembly."""
    torch = torch_cuda()
    m = nk()
    c = _varp_case(shape, orders)
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"])
    x = np.random.default_rng(11).uniform(-1, 1, c["ng"])
    ref = A(x)
    assert_close(c["sysm"].apply(to_dev(x)).cpu().numpy(), ref, FP64_RTOL, "varp apply")
    y32 = c["sysm"].apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
    assert_close(y32, ref, FP32_RTOL, "varp apply32")
    d = c["sysm"].diagonal().cpu().numpy()
    assert_close(d, jacobi_diagonal(c["mats"], c["l2g"], c["ng"], c["dm"]), FP64_RTOL, "varp diag")
    b = c["b"]
    xs, info = c["sysm"].solve(to_dev(b), rtol=1e-12)
    xs = xs.cpu().numpy()
    assert_true_residual(info[0], 1e-12, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, "varp")
    xd = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b)
    assert rel_err(xs, xd) < 1e-8
    xr, info = c["sysm"].solve(to_dev(b), rtol=1e-10, mode=m.SOLVE_F32_REFINED)
    assert_true_residual(info[0], 1e-10, A, c["mats"], c["l2g"], c["ng"], c["dm"],
                         xr.cpu().numpy(), b, "varp refined")
    # gather / assemble through the ragged map
    xl = c["sysm"].gather(to_dev(x)).cpu().numpy()
    np.testing.assert_array_equal(xl, np.concatenate(oracle.gather(x, c["l2g"])))
    yl = np.random.default_rng(12).uniform(-1, 1, xl.size)
    sizes = np.cumsum([0] + [len(g) for g in c["l2g"]])
    ylist = [yl[sizes[k]:sizes[k + 1]] for k in range(len(c["l2g"]))]
    got = c["sysm"].assemble(to_dev(yl)).cpu().numpy()
    want = oracle.assemble_vector(ylist, c["l2g"], c["ng"])
    want[c["dm"].astype(bool)] = 0.0        # Dirichlet rows (and the zero DOF) receive nothing
    assert_close(got, want, FP64_RTOL, "varp assemble")


# ----------------------------------------- the Neumann filter equation (3)

def test_filter_equation_neumann_solve():
    """u** - alpha^2 lap u** = u*, du**/dn = 0 on curved hexes: the GPU's
    modified forward transform (assembled IProductWRTBase of u*, CG on the
    Helmholtz system with kappa = alpha^2, lambda = 1, no Dirichlet DOF)
    against the oracle's sparse direct solve of the same problem; and, on an
    affine lattice, the exact recovery of a polynomial with zero normal
    derivative from its strong-form right-hand side."""
    torch = torch_cuda()
    m = nk()
    P, shape, alpha = 5, (2, 2, 2), 0.15
    Q = P + 2
    Jg, Jo, lat = jacobians(shape, P, W.WARP_AMPLITUDE)
    E, nq = lat.nelem, Q ** 3
    kap = np.full((E, nq), alpha ** 2)
    ops = oracle.ElementOps(3, P, Q, Jo, kappa=kap, lam=1.0)
    l2g, ng, _ = W.lattice_l2g(shape, P)
    none = np.zeros(ng, np.uint8)
    space = m.Space.create(3, P, Q, to_dev(Jg), kappa=to_dev(kap))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(none), lam0=1.0)
    ustar = W.uniform(W.seed(2, 1) + 3, (E, nq))
    x, info = m.filtered_fwd_trans(space, sysm, to_dev(ustar.ravel()), rtol=1e-12)
    x = x.cpu().numpy()
    mats = oracle.helmholtz_matrices(ops)
    b = oracle.assemble_vector(ops.iprod(ustar), l2g, ng)
    A = MaskedOperator(mats, l2g, ng, none)
    assert_true_residual(info[0], 1e-12, A, mats, l2g, ng, none, x, b, "filter")
    assert rel_err(x, direct_solve(mats, l2g, ng, none, b)) < 1e-9
    # polynomial with zero normal derivative, affine lattice, P = 4
    P, Q = 4, 6
    Jg, _, lat = jacobians(shape, P, 0.0)
    kap = np.full((E, Q ** 3), alpha ** 2)
    space = m.Space.create(3, P, Q, to_dev(Jg), kappa=to_dev(kap))
    l2g, ng, _ = W.lattice_l2g(shape, P)
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(np.zeros(ng, np.uint8)), lam0=1.0)
    X = W.lattice_points(m.basis_tables(P, Q)[0], lat)
    g = X ** 2 * (1 - X) ** 2
    d2g = 2 - 12 * X + 12 * X ** 2
    U = g.prod(axis=1)
    lapU = d2g[:, 0] * g[:, 1] * g[:, 2] + g[:, 0] * d2g[:, 1] * g[:, 2] + g[:, 0] * g[:, 1] * d2g[:, 2]
    x, _ = m.filtered_fwd_trans(space, sysm, to_dev((U - alpha ** 2 * lapU).ravel()), rtol=1e-13)
    u = m.bwd_trans(space, sysm.gather(x)).cpu().numpy()
    assert np.abs(u - U.ravel()).max() < 1e-12


# ------------------------------------------- orientation signs on quadrilaterals and hexahedra

@pytest.mark.parametrize("dim,P,tile", [(3, 4, "vector"), (3, 6, "vector"), (3, 6, "mfma"), (2, 5, "vector")])
def test_signed_assembled_operator(dim, P, tile):
    """Random +-1 signs per local mode (the general signed assembly
    sum_e S_e A_e^T H_e A_e S_e) through the hexahedral vector and matrix-core
    kernels and the quadrilateral kernel, against the oracle; the Jacobi
    diagonal is sign-free."""
    torch = torch_cuda()
    m = nk()
    shape = (3, 2, 2) if dim == 3 else (4, 3)
    Q = P + 2
    Jg, Jo, lat = jacobians(shape, P, W.WARP_AMPLITUDE if dim == 3 else 0.0)
    ops = oracle.ElementOps(dim, P, Q, Jo, lam=1.0)
    mats = oracle.helmholtz_matrices(ops)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    sign = np.where(np.random.default_rng(P + dim).uniform(size=l2g.shape) < 0.5, -1, 1).astype(np.int8)
    A = MaskedOperator(mats, l2g, ng, dm, sign)
    nt = m.tile_count(m.OP_HELM, dim, P)
    try:
        if tile == "mfma":
            for dt in (m.F64, m.F32):
                m.set_tile_config(m.OP_HELM, dim, P, dt, nt - 1)
        space = m.Space.create(dim, P, Q, to_dev(Jg))
        sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), sign=to_dev(sign))
        x = np.random.default_rng(7).uniform(-1, 1, ng)
        ref = A(x)
        assert_close(sysm.apply(to_dev(x)).cpu().numpy(), ref, FP64_RTOL, f"signed apply d={dim} P={P}")
        y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
        assert_close(y32, ref, FP32_RTOL, f"signed apply32 d={dim} P={P}")
        assert_close(sysm.diagonal().cpu().numpy(), jacobi_diagonal(mats, l2g, ng, dm), FP64_RTOL, "diag")
        np.testing.assert_array_equal(sysm.gather(to_dev(x)).cpu().numpy(),
                                      oracle.gather(x, l2g, sign).ravel())
    finally:
        if tile == "mfma":
            for dt in (m.F64, m.F32):
                m.set_tile_config(m.OP_HELM, dim, P, dt, 0)


@pytest.mark.parametrize("P", [2, 4, 7])
def test_interior_last_numbering_operator_and_solve(P):
    """The boundary-interior renumbering of the lattice (element interiors as
    contiguous blocks): the assembled operator and the FP64 and FP32-refined
    solves against the oracle with the same numbering."""
    torch = torch_cuda()
    m = nk()
    shape = (3, 2, 2)
    pb = _problem(shape, P, lam_seed=11)
    l2g, ng, dm = W.lattice_l2g(shape, P, interior_last=True)
    mats = oracle.helmholtz_matrices(pb["ops"])
    A = MaskedOperator(mats, l2g, ng, dm)
    space = m.Space.create(3, P, P + 2, to_dev(pb["Jg"]))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam=to_dev(pb["lam"]))
    x = np.random.default_rng(5).uniform(-1, 1, ng)
    assert_close(sysm.apply(to_dev(x)).cpu().numpy(), A(x), FP64_RTOL, f"interior-last apply P={P}")
    y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
    assert_close(y32, A(x), FP32_RTOL, f"interior-last apply32 P={P}")
    b = np.random.default_rng(6).uniform(-1, 1, ng)
    b[dm.astype(bool)] = 0.0
    # a rough random right-hand side: the recursive residual CG stops on
    # drifts from the true one by O(cond(A) eps) ~ 1e-11 at P = 7, so the
    # solve restarts from its iterate until the true residual meets rtol
    xs, info = sysm.solve(to_dev(b), rtol=1e-12)
    assert_true_residual(info[0], 1e-12, A, mats, l2g, ng, dm, xs.cpu().numpy(), b, f"P={P}")
    xref = direct_solve(mats, l2g, ng, dm, b)
    assert rel_err(xs.cpu().numpy(), xref) < 1e-8
    xr, info = sysm.solve(to_dev(b), rtol=1e-10, mode=m.SOLVE_F32_REFINED)
    assert_true_residual(info[0], 1e-10, A, mats, l2g, ng, dm, xr.cpu().numpy(), b, f"refined P={P}")


@pytest.mark.parametrize("P", [4, 6, 8])
def test_full_size_24c_cg_sampled_residuals(P):
    """The 24^3 curved-hex CG problem of the benchmark at full size, in its
    launch configuration (the system's own tuned tile): FP64 PCG and the
    FP32-refined solve to 1e-10 on a seeded right-hand side.  The oracle
    recomputes (A x)_g at a seeded sample of free global DOFs (lattice
    vertices, shared by eight elements, and random DOFs) from the elements
    that hold them: every sampled residual obeys |b_g - (A x)_g| <= 1e-10
    ||b||_2 (implied by the 2-norm criterion), and the GPU's own A x agrees
    with the oracle's there to 1e-12 of the largest output of the elements
    involved (the scale of the rounding in a sum with cancellation)."""
    from gpu_common import lib_points
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
    x64, info = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000)
    assert info[0]["status"] == 0
    x32, info = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000, mode=m.SOLVE_F32_REFINED)
    assert info[0]["status"] == 0
    Ax = sysm.apply(x64).cpu().numpy()
    G = [s * P + 1 for s in shape]
    free = np.flatnonzero(~fixed)
    gx, gy, gz = free % G[0], (free // G[0]) % G[1], free // (G[0] * G[1])
    verts = free[(gx % P == 0) & (gy % P == 0) & (gz % P == 0)]
    rng = np.random.default_rng(40 + P)
    sample = np.unique(np.concatenate([rng.choice(verts, 4, replace=False), rng.choice(free, 8, replace=False)]))
    hits = {int(g): np.argwhere(l2g == g) for g in sample}          # (e, local mode) pairs
    elems = np.unique(np.concatenate([h[:, 0] for h in hits.values()]))
    assert max(len(h) for h in hits.values()) == 8
    pos = {int(e): k for k, e in enumerate(elems)}
    Jo = W.element_jacobians(oracle.gll(Q)[0], W.Lattice(lat.shape, lat.h, lat.origins[elems]), W.WARP_AMPLITUDE)
    ops = oracle.ElementOps(3, P, Q, Jo, lam=1.0)
    bn = np.linalg.norm(b)
    for x, tag in ((x64, "f64"), (x32, "f32-refined")):
        xs = x.cpu().numpy().copy()
        xs[fixed] = 0.0
        y = ops.helmholtz_action(xs[l2g[elems]])
        for g, h in hits.items():
            parts = np.array([y[pos[int(e)], mm] for e, mm in h])
            Ag = parts.sum()
            assert abs(b[g] - Ag) <= 1e-10 * bn, (tag, g, abs(b[g] - Ag) / bn)
            if tag == "f64":
                scale = sum(np.abs(y[pos[int(e)]]).max() for e, _ in h)
                assert abs(Ax[g] - Ag) <= 1e-12 * scale, (g, Ax[g], Ag, scale)


def test_system_size_limit_rejected():
    """Bit 30 of an internal l2g entry carries the orientation sign, so a
    system holds fewer than 2^30 DOFs both as given and after each system's
    DOF range is padded to whole reduction blocks. Both limits are rejected
    with NK_EINVAL on the host before any device allocation."""
    torch = torch_cuda()
    m = nk()
    P, Q = 1, 3
    Jg, _, _ = jacobians((1, 1, 1), P, 0.0)
    space = m.Space.create(3, P, Q, to_dev(Jg))
    l2g = to_dev(np.arange(8, dtype=np.int32).reshape(1, 8))
    small = torch.zeros(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(m.NkError) as ei:
        m.System.create(space, 1 << 30, l2g, small)
    assert ei.value.status == m.NK_EINVAL
    assert "too many global DOFs" in str(ei.value)
    ng = (1 << 30) - 1
    dm = torch.zeros(ng, dtype=torch.uint8, device="cuda")
    with pytest.raises(m.NkError) as ei:
        m.System.create(space, ng, l2g, dm)
    assert ei.value.status == m.NK_EINVAL
    assert "padded system too large" in str(ei.value)
    del dm
    torch.cuda.empty_cache()


# ------------------------------------ separately created systems in one call

def test_cg_solve_batched_separate_systems():
    """nk_cg_solve_batched over systems created separately, each with its own
    space: two P=3 boxes (one with per-element lambda), two P=5 boxes, one
    P=7 box and a conforming mixed-order system.  The P=3 and P=5 pairs run
    as batched unions, the others as lanes of their own.  Every system's
    solution matches the oracle's direct solve, its true residual meets rtol
    (library value exactly, oracle value up to rounding), a second call
    reuses the cached unions, and destroying a member drops them."""
    m = nk()
    torch = torch_cuda()
    specs = [((2, 2, 1), 3, None), ((3, 2, 2), 3, 31), ((2, 2, 2), 5, None), ((1, 2, 2), 5, 32),
             ((2, 1, 2), 7, None)]
    cases = []
    for shape, P, ls in specs:
        pb = _problem(shape, P, lam_seed=ls)
        mats = oracle.helmholtz_matrices(pb["ops"])
        b = _rhs(pb)
        _, sysm = _gpu_system(pb)
        cases.append(dict(sys=sysm, mats=mats, l2g=pb["l2g"], ng=pb["ng"], dm=pb["dm"], b=b,
                          xref=direct_solve(mats, pb["l2g"], pb["ng"], pb["dm"], b)))
    vc = _varp_case((2, 2, 1), [2, 4, 3, 5])
    cases.append(dict(sys=vc["sysm"], mats=vc["mats"], l2g=vc["l2g"], ng=vc["ng"], dm=vc["dm"],
                      b=vc["b"], xref=direct_solve(vc["mats"], vc["l2g"], vc["ng"], vc["dm"], vc["b"])))

    def check(cs, mode, tol, err_tol, what):
        xs, info = m.solve_batched([c["sys"] for c in cs], [to_dev(c["b"]) for c in cs], rtol=tol,
                                   mode=mode)
        assert len(info) == len(cs)
        for k, c in enumerate(cs):
            A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"])
            x = xs[k].cpu().numpy()
            assert_true_residual(info[k], tol, A, c["mats"], c["l2g"], c["ng"], c["dm"], x, c["b"],
                                 f"{what} system {k}")
            assert rel_err(x, c["xref"]) < err_tol, (what, k, rel_err(x, c["xref"]))
        return xs

    for rep in range(2):
        check(cases, m.SOLVE_F64, 1e-12, 1e-8, f"f64 call {rep}")
        check(cases, m.SOLVE_F32_REFINED, 1e-10, 1e-6, f"refined call {rep}")
    # a single system through the batched call equals nk_cg_solve's contract
    check(cases[4:5], m.SOLVE_F64, 1e-12, 1e-8, "one system")
    # destroying a member drops its union; the rest still solve
    cases[0]["sys"].destroy()
    check(cases[1:], m.SOLVE_F64, 1e-12, 1e-8, "after destroy")
    # a system may appear once per call
    with pytest.raises(m.NkError) as ei:
        m.solve_batched([cases[1]["sys"], cases[1]["sys"]], [to_dev(cases[1]["b"])] * 2)
    assert ei.value.status == m.NK_EINVAL
