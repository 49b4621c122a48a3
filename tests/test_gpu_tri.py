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
