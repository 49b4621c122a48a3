"""GPU parity of the collapsed-coordinate triangle operators (BwdTrans,
IProductWRTBase, Helmholtz with per-point kappa and per-element lambda)
against the oracle's dense elemental matrices, on a curved triangle mesh;
FP64 1e-12 and FP32 2e-6 relative 2-norm, as for the other operators."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import collapsed as C
from gpu_common import FP32_RTOL, FP64_RTOL, assert_close, nk, to_dev, torch_cuda

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
