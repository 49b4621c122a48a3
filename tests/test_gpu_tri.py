"""GPU parity of the collapsed-coordinate triangle operators (BwdTrans,
IProductWRTBase, Helmholtz with per-point kappa and per-element lambda)
against the oracle's dense elemental matrices, on a curved triangle mesh;
FP64 1e-12 and FP32 2e-6 relative 2-norm, as for the other operators."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import collapsed as C
from gpu_common import (FP32_RTOL, FP64_RTOL, assert_close, assert_true_residual, nk, rel_err, to_dev,
                        torch_cuda)

pytestmark = pytest.mark.gpu


def _case(P, n=3, amp=0.05):
    m = nk()
    Q = P + 2
    e1g, _, e2g, _ = m.tri_points(Q)
    Jg = W.tri_lattice_jacobians(n, e1g, e2g, amp)
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    Jo = W.tri_lattice_jacobians(n, oracle.gll(Q)[0], x1, amp)
    return Jg, Jo


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_triangle_operators_match_oracle(P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, Jo = _case(P)
    E, nq = Jg.shape[0], Q * (Q - 1)
    nm = (P + 1) * (P + 2) // 2
    rng = np.random.default_rng(70 + P)
    kap = rng.uniform(0.5, 2.0, (E, nq))
    lam = rng.uniform(0.5, 2.0, E)
    ops = C.TriOps(P, Q, Jo, kappa=kap, lam=lam)
    space = m.Space.create_tri(P, Q, to_dev(Jg), kappa=to_dev(kap))
    c = W.uniform(W.seed(0, 0) + 300 + P, (E, nm))
    f = W.uniform(W.seed(0, 1) + 300 + P, (E, nq))
    ref = [ops.bwd(c), ops.iprod(f), ops.helmholtz(c)]
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        got = [m.bwd_trans(space, to_dev(c.ravel(), td), dtype=dt),
               m.iprod_wrt_base(space, to_dev(f.ravel(), td), dtype=dt),
               m.helmholtz(space, to_dev(c.ravel(), td), lam=to_dev(lam), dtype=dt)]
        for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
            assert_close(g.double().cpu().numpy(), r.ravel(), tol, f"tri {name} P={P} dt={dt}")


def test_triangle_space_rejects_unsupported_calls():
    torch = torch_cuda()
    m = nk()
    P, Q = 3, 5
    Jg, _ = _case(P, n=1)
    space = m.Space.create_tri(P, Q, to_dev(Jg))
    with pytest.raises(m.NkError) as ei:
        m.phys_deriv(space, torch.zeros(2 * Q * (Q - 1), dtype=torch.float64, device="cuda"))
    assert ei.value.status == m.NK_EUNSUPPORTED
    bad = Jg.copy()
    bad[0, 0, 0] *= -1.0          # inverted element
    bad[0, 0, 1] *= -1.0
    with pytest.raises(m.NkError):
        m.Space.create_tri(P, Q, to_dev(bad))


def test_empty_triangle_space():
    torch = torch_cuda()
    m = nk()
    P, Q = 4, 6
    space = m.Space.create_tri(P, Q, to_dev(np.zeros((0, 2, 2, Q * (Q - 1)))))
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert m.bwd_trans(space, e).numel() == 0
    assert m.iprod_wrt_base(space, e).numel() == 0
    assert m.helmholtz(space, e).numel() == 0


def test_full_size_131072_triangles_p6_sampled():
    """The curved-triangle workload the benchmark times (256 x 256 squares,
    131072 triangles, P=6, Q=8) at full size and in the same launch
    configuration; the oracle checks a seeded sample of elements (first,
    last and 10 random) of all three operators in FP64 and FP32."""
    torch = torch_cuda()
    m = nk()
    n, P = 256, 6
    Q = P + 2
    e1g, _, e2g, _ = m.tri_points(Q)
    space = m.Space.create_tri(P, Q, to_dev(W.tri_lattice_jacobians(n, e1g, e2g, 0.05)))
    E, nq, nm = 2 * n * n, Q * (Q - 1), (P + 1) * (P + 2) // 2
    c = W.uniform(W.seed(1, 0), E * nm)
    f = W.uniform(W.seed(1, 1), E * nq)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(7).choice(E, 10, replace=False)]))
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    Jo = W.tri_lattice_jacobians(n, oracle.gll(Q)[0], x1, 0.05)[sample]
    ops = C.TriOps(P, Q, Jo)
    cs, fs = c.reshape(E, nm)[sample], f.reshape(E, nq)[sample]
    ref = [ops.bwd(cs), ops.iprod(fs), ops.helmholtz(cs)]
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        got = [m.bwd_trans(space, to_dev(c, td), dtype=dt).double().cpu().numpy().reshape(E, nq),
               m.iprod_wrt_base(space, to_dev(f, td), dtype=dt).double().cpu().numpy().reshape(E, nm),
               m.helmholtz(space, to_dev(c, td), lam0=1.0, dtype=dt).double().cpu().numpy().reshape(E, nm)]
        for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
            assert_close(g[sample], r, tol, f"full-size tri {name} dt={dt}")


# ------------------------------------------- assembled triangle systems with orientation signs

def _tri_system_case(P, n=4, amp=0.05):
    """Curved triangle mesh with rotated local vertex orders, per-point kappa
    and per-element lambda; the oracle's elemental matrices and the GPU
    system built from the same signed numbering."""
    m = nk()
    Q = P + 2
    E = 2 * n * n
    rot = W.tri_rotations(40 + P, E)
    e1g, _, e2g, _ = m.tri_points(Q)
    Jg = W.tri_lattice_jacobians(n, e1g, e2g, amp, rot)
    x1, _ = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    Jo = W.tri_lattice_jacobians(n, oracle.gll(Q)[0], x1, amp, rot)
    l2g, sign, ng, dm = W.tri_lattice_l2g(n, P, rot)
    rng = np.random.default_rng(80 + P)
    kap = rng.uniform(0.5, 2.0, (E, Q * (Q - 1)))
    lam = rng.uniform(0.5, 2.0, E)
    ops = C.TriOps(P, Q, Jo, kappa=kap, lam=lam)
    mats = [ops.helmholtz_matrix(e) for e in range(E)]
    space = m.Space.create_tri(P, Q, to_dev(Jg), kappa=to_dev(kap))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam=to_dev(lam), sign=to_dev(sign))
    return dict(ops=ops, mats=mats, l2g=l2g, sign=sign, ng=ng, dm=dm, space=space, sys=sysm, E=E)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 6, 8, 10])
def test_triangle_system_operator_diag_gather_assemble(P):
    """The signed assembled triangle operator (gather with signs, elemental
    Helmholtz, signed scatter-add, Dirichlet rows masked), its Jacobi
    diagonal, gather and assembly against the oracle's signed assembly."""
    from oracle.assembly import MaskedOperator, jacobi_diagonal
    torch = torch_cuda()
    m = nk()
    c = _tri_system_case(P)
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"], c["sign"])
    x = np.random.default_rng(P).uniform(-1, 1, c["ng"])
    ref = A(x)
    sysm = c["sys"]
    assert_close(sysm.apply(to_dev(x)).cpu().numpy(), ref, FP64_RTOL, f"tri apply P={P}")
    y32 = sysm.apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
    assert_close(y32, ref, FP32_RTOL, f"tri apply32 P={P}")
    dref = jacobi_diagonal(c["mats"], c["l2g"], c["ng"], c["dm"], c["sign"])
    assert_close(sysm.diagonal().cpu().numpy(), dref, FP64_RTOL, f"tri diag P={P}")
    xl = sysm.gather(to_dev(x)).cpu().numpy()
    np.testing.assert_array_equal(xl, oracle.gather(x, c["l2g"], c["sign"]).ravel())
    yl = np.random.default_rng(P + 1).uniform(-1, 1, xl.size)
    bref = oracle.assemble_vector(yl.reshape(c["E"], -1), c["l2g"], c["ng"], c["sign"])
    bref[c["dm"].astype(bool)] = 0.0
    assert_close(sysm.assemble(to_dev(yl)).cpu().numpy(), bref, 1e-14, f"tri assemble P={P}")


@pytest.mark.parametrize("P", [2, 4, 6])
def test_triangle_cg_solves_match_direct_solve(P):
    """FP64 PCG to 1e-12 and the FP32-refined solve to 1e-10 on the signed
    curved triangle mesh, against the oracle's sparse direct solve."""
    from oracle.assembly import MaskedOperator, direct_solve
    m = nk()
    torch_cuda()
    c = _tri_system_case(P, n=6)
    b = np.random.default_rng(90 + P).uniform(-1, 1, c["ng"])
    b[c["dm"].astype(bool)] = 0.0
    A = MaskedOperator(c["mats"], c["l2g"], c["ng"], c["dm"], c["sign"])
    xref = direct_solve(c["mats"], c["l2g"], c["ng"], c["dm"], b, c["sign"])
    x, info = c["sys"].solve(to_dev(b), rtol=1e-12, maxit=20000)
    xs = x.cpu().numpy()
    assert_true_residual(info[0], 1e-12, A, c["mats"], c["l2g"], c["ng"], c["dm"], xs, b, "f64")
    assert rel_err(xs, xref) < 1e-8
    xr, info = c["sys"].solve(to_dev(b), rtol=1e-10, maxit=20000, mode=m.SOLVE_F32_REFINED)
    assert_true_residual(info[0], 1e-10, A, c["mats"], c["l2g"], c["ng"], c["dm"],
                         xr.cpu().numpy(), b, "refined")


def test_signed_system_rejects_bad_signs_and_keeps_unsigned_behaviour():
    """Signs other than +-1 are rejected; an all-+1 sign array gives the same
    operator as the unsigned create call."""
    torch = torch_cuda()
    m = nk()
    c = _tri_system_case(3, n=2)
    bad = c["sign"].copy()
    bad[0, 0] = 2
    with pytest.raises(m.NkError) as ei:
        m.System.create(c["space"], c["ng"], to_dev(c["l2g"]), to_dev(c["dm"]), sign=to_dev(bad))
    assert ei.value.status == m.NK_EINVAL
    ones = np.ones_like(c["sign"])
    s1 = m.System.create(c["space"], c["ng"], to_dev(c["l2g"]), to_dev(c["dm"]), sign=to_dev(ones))
    s0 = m.System.create(c["space"], c["ng"], to_dev(c["l2g"]), to_dev(c["dm"]))
    x = to_dev(np.random.default_rng(4).uniform(-1, 1, c["ng"]))
    assert torch.equal(s1.apply(x), s0.apply(x))
