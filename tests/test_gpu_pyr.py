"""GPU parity of the pyramid operators (BwdTrans, IProductWRTBase, Helmholtz
with per-point kappa and per-element lambda) against the oracle's dense
elemental matrices, on the curved pyramidal mesh of the unit cube; FP64
1e-12 and FP32 2e-6 relative 2-norm, as for the other operators."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import collapsed as C
from gpu_common import (FP32_RTOL, FP64_RTOL, assert_close, assert_true_residual, nk, rel_err, to_dev,
                        torch_cuda)

pytestmark = pytest.mark.gpu


def _jacobians(P, n, amp=W.WARP_AMPLITUDE, elems=None):
    """(J at the library's points, J at the oracle's points)."""
    m = nk()
    Q = P + 2
    xg = m.basis_tables(P, Q)[0]
    e3g = m.tet_points(Q)[4]
    Jg = W.pyr_lattice_jacobians(n, xg, xg, e3g, amp, elems)
    x, _ = oracle.gll(Q)
    x3, _ = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    Jo = W.pyr_lattice_jacobians(n, x, x, x3, amp, elems)
    return Jg, Jo


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_pyramid_operators_match_oracle(P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, Jo = _jacobians(P, 2 if P <= 5 else 1)
    E, nq = Jg.shape[0], Q * Q * (Q - 1)
    nm = (P + 1) * (P + 2) * (2 * P + 3) // 6
    rng = np.random.default_rng(370 + P)
    kap = rng.uniform(0.5, 2.0, (E, nq))
    lam = rng.uniform(0.5, 2.0, E)
    ops = C.PyrOps(P, Q, Jo, kappa=kap, lam=lam)
    space = m.Space.create_pyr(P, Q, to_dev(Jg), kappa=to_dev(kap))
    c = W.uniform(W.seed(0, 0) + 600 + P, (E, nm))
    f = W.uniform(W.seed(0, 1) + 600 + P, (E, nq))
    ref = [ops.bwd(c), ops.iprod(f), ops.helmholtz(c)]
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        got = [m.bwd_trans(space, to_dev(c.ravel(), td), dtype=dt),
               m.iprod_wrt_base(space, to_dev(f.ravel(), td), dtype=dt),
               m.helmholtz(space, to_dev(c.ravel(), td), lam=to_dev(lam), dtype=dt)]
        for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
            assert_close(g.double().cpu().numpy(), r.ravel(), tol, f"pyr {name} P={P} dt={dt}")


def test_pyramid_helmholtz_constant_symmetry_and_errors():
    """L 1 = 0 and x^T H y = y^T H x on the GPU at P = 4; an empty space;
    derivative calls are rejected; a mirrored element too."""
    torch = torch_cuda()
    m = nk()
    P, Q = 4, 6
    Jg, _ = _jacobians(P, 2)
    E = Jg.shape[0]
    modes = C.pyr_modes(P)
    one = np.array([1.0 if (p < 0 or (p in (0, P) and q in (0, P) and r == 0)) else 0.0
                    for p, q, s, r in modes])
    space = m.Space.create_pyr(P, Q, to_dev(Jg))
    y = m.helmholtz(space, to_dev(np.tile(one, E)), lam0=0.0).cpu().numpy()
    assert np.abs(y).max() < 1e-12
    rng = np.random.default_rng(1)
    a, b = rng.uniform(-1, 1, (2, E * len(modes)))
    Ha = m.helmholtz(space, to_dev(a)).cpu().numpy()
    Hb = m.helmholtz(space, to_dev(b)).cpu().numpy()
    assert abs(b @ Ha - a @ Hb) < 1e-12 * abs(b @ Ha)
    nq = Q * Q * (Q - 1)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert m.helmholtz(m.Space.create_pyr(P, Q, to_dev(np.zeros((0, 3, 3, nq)))), e).numel() == 0
    with pytest.raises(m.NkError) as ei:
        m.fwd_trans(space, torch.zeros(E * nq, dtype=torch.float64, device="cuda"))
    assert ei.value.status == m.NK_EUNSUPPORTED
    bad = Jg.copy()
    bad[0, :, 1] *= -1.0
    with pytest.raises(m.NkError):
        m.Space.create_pyr(P, Q, to_dev(bad))


def test_full_size_pyramids_p4_sampled():
    """The pyramidal workload the benchmark times (6 x 20^3 = 48 000 curved
    pyramids, P=4, Q=6) at full size and in the same launch configuration;
    the oracle checks a seeded sample of elements in FP64 and FP32."""
    torch = torch_cuda()
    m = nk()
    n, P = 20, 4
    Q = P + 2
    E, nq, nm = 6 * n ** 3, Q * Q * (Q - 1), (P + 1) * (P + 2) * (2 * P + 3) // 6
    xg = m.basis_tables(P, Q)[0]
    space = m.Space.create_pyr(P, Q, to_dev(W.pyr_lattice_jacobians(n, xg, xg, m.tet_points(Q)[4])))
    c = W.uniform(W.seed(1, 0), E * nm)
    f = W.uniform(W.seed(1, 1), E * nq)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(10).choice(E, 10, replace=False)]))
    _, Jo = _jacobians(P, n, elems=sample)
    ops = C.PyrOps(P, Q, Jo)
    cs, fs = c.reshape(E, nm)[sample], f.reshape(E, nq)[sample]
    ref = [ops.bwd(cs), ops.iprod(fs), ops.helmholtz(cs)]
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        got = [m.bwd_trans(space, to_dev(c, td), dtype=dt).double().cpu().numpy().reshape(E, nq),
               m.iprod_wrt_base(space, to_dev(f, td), dtype=dt).double().cpu().numpy().reshape(E, nm),
               m.helmholtz(space, to_dev(c, td), lam0=1.0, dtype=dt).double().cpu().numpy().reshape(E, nm)]
        for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
            assert_close(g[sample], r, tol, f"full-size pyr {name} dt={dt}")


# ------------------------------ assembled pyramidal systems (no signs needed)

def _pyr_system_case(P, n=2, amp=W.WARP_AMPLITUDE):
    """Curved pyramidal mesh with per-point kappa and per-element lambda; the
    oracle's elemental matrices and the GPU system built from the same
    numbering (base modes transposed where an element's b and d swap)."""
    m = nk()
    Q = P + 2
    Jg, Jo = _jacobians(P, n, amp)
    l2g, ng, dm = W.pyr_lattice_l2g(n, P)
    E, nq = Jg.shape[0], Q * Q * (Q - 1)
    rng = np.random.default_rng(400 + P)
    kap = rng.uniform(0.5, 2.0, (E, nq))
    lam = rng.uniform(0.5, 2.0, E)
    ops = C.PyrOps(P, Q, Jo, kappa=kap, lam=lam)
    mats = [ops.helmholtz_matrix(e) for e in range(E)]
    space = m.Space.create_pyr(P, Q, to_dev(Jg), kappa=to_dev(kap))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam=to_dev(lam))
    return dict(ops=ops, mats=mats, l2g=l2g, ng=ng, dm=dm, space=space, sys=sysm, E=E)


@pytest.mark.parametrize("P", [1, 2, 3, 5, 7])
def test_pyramidal_system_operator_diag_gather_assemble(P):
    """The assembled pyramidal operator (gather, elemental Helmholtz,
    scatter-add, Dirichlet rows masked), its Jacobi diagonal, gather and
    assembly against the oracle."""
    from oracle.assembly import MaskedOperator, jacobi_diagonal
    torch = torch_cuda()
    m = nk()
    c = _pyr_system_case(P, n=2 if P <= 5 else 1)
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"])
    x = np.random.default_rng(P).uniform(-1, 1, c["ng"])
    ref = A(x)
    sysm = c["sys"]
    assert_close(sysm.apply(to_dev(x)).cpu().numpy(), ref, FP64_RTOL, f"pyr apply P={P}")
    y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
    assert_close(y32, ref, FP32_RTOL, f"pyr apply32 P={P}")
    dref = jacobi_diagonal(c["mats"], c["l2g"], c["ng"], c["dm"])
    assert_close(sysm.diagonal().cpu().numpy(), dref, FP64_RTOL, f"pyr diag P={P}")
    xl = sysm.gather(to_dev(x)).cpu().numpy()
    np.testing.assert_array_equal(xl, oracle.gather(x, c["l2g"]).ravel())
    yl = np.random.default_rng(P + 1).uniform(-1, 1, xl.size)
    bref = oracle.assemble_vector(yl.reshape(c["E"], -1), c["l2g"], c["ng"])
    bref[c["dm"].astype(bool)] = 0.0
    assert_close(sysm.assemble(to_dev(yl)).cpu().numpy(), bref, 1e-14, f"pyr assemble P={P}")


@pytest.mark.parametrize("P", [2, 4])
def test_pyramidal_cg_solves_match_direct_solve(P):
    """FP64 PCG to 1e-12 and the FP32-refined solve to 1e-10 on the curved
    pyramidal mesh, against the oracle's sparse direct solve."""
    from oracle.assembly import MaskedOperator, direct_solve
    m = nk()
    torch_cuda()
    c = _pyr_system_case(P, n=2)
    b = np.random.default_rng(405 + P).uniform(-1, 1, c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"])
    xref = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b)
    x, info = c["sys"].solve(to_dev(b), rtol=1e-12, maxit=20000)
    xs = x.cpu().numpy()
    assert_true_residual(info[0], 1e-12, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, "f64")
    assert rel_err(xs, xref) < 1e-8
    xr, info = c["sys"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_F32_REFINED)
    assert_true_residual(info[0], 1e-10, A, c["mats"], c["l2g"], c["ng"], c["dm"],
                         xr.cpu().numpy(), b, "refined")
