"""GPU parity of PhysDeriv, IProductWRTDerivBase and FwdTrans against the
oracle (dense collocation derivative with the chain rule, dense D_a B
products, dense elemental mass solves), on warped hexes and affine quads.

Tolerances.  FP64 operators: 1e-12 relative 2-norm, as for the other
operators.  FP32 PhysDeriv and IProductWRTDerivBase: 1e-5; each output is a
sum of Q products of the collocation (or D_a B) entries, which alternate in
sign and exceed the result by up to ~Q^2/2 at Q <= 12, so the FP32 rounding
of 6e-8 per term grows to a few 1e-6 normwise.  FwdTrans solves with M_e,
whose condition number reaches ~1e7 at P=6 in the modified basis: the result
is checked by its FP64 residual as the oracle recomputes it (<= 1e-12 of the
right-hand side), by the mass-norm distance to the oracle's dense solution
(the physical-space error, bounded by residual x sqrt(cond) ~ 1e-13 x 3e3),
and by coefficients within cond x 1e-16 ~ 1e-8 (looser: both solves round).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import FP64_RTOL, assert_close, jacobians, nk, rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

FP32_DERIV_RTOL = 1e-5


def _mesh(dim, P, shape=None, amp=None):
    shape = shape or ((2, 2, 1) if dim == 3 else (3, 2))
    amp = (W.WARP_AMPLITUDE if dim == 3 else 0.0) if amp is None else amp
    Jg, Jo, lat = jacobians(shape, P, amp)
    return Jg, Jo, lat


@pytest.mark.parametrize("dim,P", [(3, 1), (3, 2), (3, 3), (3, 5), (3, 6), (3, 7), (3, 8), (3, 10),
                                   (2, 2), (2, 4), (2, 7), (2, 10)])
def test_phys_deriv_and_iprod_deriv_match_oracle(dim, P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, Jo, lat = _mesh(dim, P)
    E, nq = lat.nelem, Q ** dim
    ops = oracle.ElementOps(dim, P, Q, Jo)
    u = W.uniform(W.seed(0, 1) + P, (E, nq))
    f = W.uniform(W.seed(0, 1) + 50 + P, (E, dim, nq))
    space = m.Space.create(dim, P, Q, to_dev(Jg))
    du_ref = ops.phys_deriv(u)
    ip_ref = ops.iprod_deriv(f)
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_DERIV_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        du = m.phys_deriv(space, to_dev(u.ravel(), td), dtype=dt)
        assert_close(du.double().cpu().numpy(), du_ref.ravel(), tol, f"phys_deriv P={P} dt={dt}")
        ip = m.iprod_wrt_deriv_base(space, to_dev(f.ravel(), td), dtype=dt)
        assert_close(ip.double().cpu().numpy(), ip_ref.ravel(), tol, f"iprod_deriv P={P} dt={dt}")


def test_iprod_deriv_of_phys_deriv_is_the_laplacian_on_gpu():
    """Composed on the GPU: IProductWRTDerivBase(PhysDeriv(BwdTrans c)) equals
    the local Helmholtz operator with lambda = 0 (kappa = 1) applied to c."""
    torch = torch_cuda()
    m = nk()
    P, Q = 5, 7
    Jg, _, lat = _mesh(3, P, shape=(2, 2, 2))
    c = to_dev(W.uniform(W.seed(0, 0) + 7, (lat.nelem, (P + 1) ** 3)).ravel())
    space = m.Space.create(3, P, Q, to_dev(Jg))
    lap = m.helmholtz(space, c, lam0=0.0)
    got = m.iprod_wrt_deriv_base(space, m.phys_deriv(space, m.bwd_trans(space, c)))
    assert_close(got.cpu().numpy(), lap.cpu().numpy(), 1e-11, "div grad")


def _mass_norm(ops, d):
    return np.sqrt(sum(d[e] @ ops.mass_matrix(e) @ d[e] for e in range(ops.nelem)))


@pytest.mark.parametrize("P", [1, 2, 3, 4, 6, 7, 8, 10])
def test_fwd_trans_matches_oracle(P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, Jo, lat = _mesh(3, P, shape=(2, 1, 2))
    E = lat.nelem
    ops = oracle.ElementOps(3, P, Q, Jo)
    f = W.uniform(W.seed(0, 1) + 100 + P, (E, Q ** 3))
    ref = ops.fwd(f)
    rhs = ops.iprod(f)
    space = m.Space.create(3, P, Q, to_dev(Jg))
    x = m.fwd_trans(space, to_dev(f.ravel())).cpu().numpy().reshape(E, -1)
    res = np.stack([rhs[e] - ops.mass_matrix(e) @ x[e] for e in range(E)])
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(rhs)
    assert _mass_norm(ops, x - ref) <= 1e-10 * _mass_norm(ops, ref)
    assert rel_err(x, ref) <= 1e-7
    # FP32: the projection in physical space (mass norm) to FP32 accuracy
    x32 = m.fwd_trans(space, to_dev(f.ravel(), torch.float32), dtype=m.F32)
    x32 = x32.double().cpu().numpy().reshape(E, -1)
    assert _mass_norm(ops, x32 - ref) <= 2e-5 * _mass_norm(ops, ref)


def test_fwd_trans_inverts_bwd_trans_on_gpu():
    torch = torch_cuda()
    m = nk()
    P, Q = 6, 8
    Jg, _, lat = _mesh(3, P, shape=(3, 2, 2))
    c = W.uniform(W.seed(0, 0) + 9, (lat.nelem, (P + 1) ** 3))
    space = m.Space.create(3, P, Q, to_dev(Jg))
    got = m.fwd_trans(space, m.bwd_trans(space, to_dev(c.ravel()))).cpu().numpy()
    assert rel_err(got, c) <= 1e-8


@pytest.mark.parametrize("P", [1, 3, 4, 7, 10])
def test_fwd_trans_2d_matches_oracle(P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, Jo, lat = _mesh(2, P, shape=(3, 2))
    E = lat.nelem
    ops = oracle.ElementOps(2, P, Q, Jo)
    f = W.uniform(W.seed(0, 1) + 200 + P, (E, Q ** 2))
    ref = ops.fwd(f)
    rhs = ops.iprod(f)
    space = m.Space.create(2, P, Q, to_dev(Jg))
    x = m.fwd_trans(space, to_dev(f.ravel())).cpu().numpy().reshape(E, -1)
    res = np.stack([rhs[e] - ops.mass_matrix(e) @ x[e] for e in range(E)])
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(rhs)
    assert _mass_norm(ops, x - ref) <= 1e-10 * _mass_norm(ops, ref)
    x32 = m.fwd_trans(space, to_dev(f.ravel(), torch.float32), dtype=m.F32)
    x32 = x32.double().cpu().numpy().reshape(E, -1)
    assert _mass_norm(ops, x32 - ref) <= 2e-5 * _mass_norm(ops, ref)


def test_listing_projection_and_integral_on_gpu():
    """The listing of section 3.5 on the GPU: one standard quadrilateral
    [-1,1]^2, 8 modes (P=7) and 9 GLL points per direction, f = cos x cos y.
    Its integral (the sum of the four vertex-mode entries of
    IProductWRTBase(f), since the vertex modes sum to 1) is 4 sin^2(1), the
    value the text prints (tests/golden); FwdTrans(f) is the Galerkin
    projection: the oracle finds I(f - BwdTrans(FwdTrans f)) = 0 and the
    projection's integral equals the integral of f."""
    import os
    torch = torch_cuda()
    m = nk()
    with open(os.path.join(os.path.dirname(__file__), "golden", "listing1_integral.txt")) as fh:
        nm, npts, exact = [l for l in fh if not l.startswith("#")][0].split()
    P, Q, exact = int(nm) - 1, int(npts), float(exact)
    xg = m.basis_tables(P, Q)[0]
    J = np.zeros((1, 2, 2, Q * Q))
    J[0, 0, 0] = J[0, 1, 1] = 1.0
    space = m.Space.create(2, P, Q, to_dev(J))
    X, Y = np.meshgrid(xg, xg, indexing="ij")
    f = (np.cos(X) * np.cos(Y)).T.ravel()          # point q = i + Q j
    n = P + 1
    vert = [0, P, P * n, P * n + P]
    I = m.iprod_wrt_base(space, to_dev(f)).cpu().numpy()
    assert abs(I[vert].sum() - exact) < 1e-14
    c = m.fwd_trans(space, to_dev(f))
    Ic = m.iprod_wrt_base(space, m.bwd_trans(space, c)).cpu().numpy()
    assert abs(Ic[vert].sum() - exact) < 1e-13
    ops = oracle.ElementOps(2, P, Q, J)
    r = ops.iprod(f[None] - ops.bwd(c.cpu().numpy()[None]))
    assert np.abs(r).max() < 1e-14


def test_empty_space_derivative_operators():
    torch = torch_cuda()
    m = nk()
    P = 3
    J0 = np.zeros((0, 3, 3, (P + 2) ** 3))
    s0 = m.Space.create(3, P, P + 2, to_dev(J0))
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert m.phys_deriv(s0, e).numel() == 0
    assert m.iprod_wrt_deriv_base(s0, e).numel() == 0
    assert m.fwd_trans(s0, e).numel() == 0


def test_full_size_32cube_p6_sampled():
    """The 32^3, P=6 curved workload at full size in the launch configuration
    the benchmark times; the oracle checks a seeded sample of elements (first,
    last and 10 random) for all three operators."""
    torch = torch_cuda()
    m = nk()
    cfg = W.CONFIGS[1]
    P, Q = cfg["P"], cfg["Q"]
    lat = W.lattice(cfg["shape"])
    E = lat.nelem
    space = m.Space.create(3, P, Q, to_dev(W.element_jacobians(m.basis_tables(P, Q)[0], lat, cfg["warp"])))
    u = W.uniform(W.seed(1, 1), (E, Q ** 3))
    f = W.uniform(W.seed(1, 1) + 10, (E, 3, Q ** 3))
    du = m.phys_deriv(space, to_dev(u.ravel())).cpu().numpy().reshape(E, 3, -1)
    ip = m.iprod_wrt_deriv_base(space, to_dev(f.ravel())).cpu().numpy().reshape(E, -1)
    fw = m.fwd_trans(space, to_dev(u.ravel())).cpu().numpy().reshape(E, -1)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(6).choice(E, 10, replace=False)]))
    Jo = W.element_jacobians(oracle.gll(Q)[0], W.Lattice(lat.shape, lat.h, lat.origins[sample]), cfg["warp"])
    ops = oracle.ElementOps(3, P, Q, Jo)
    assert_close(du[sample], ops.phys_deriv(u[sample]), FP64_RTOL, "full-size phys_deriv")
    assert_close(ip[sample], ops.iprod_deriv(f[sample]), FP64_RTOL, "full-size iprod_deriv")
    ref = ops.fwd(u[sample])
    assert _mass_norm(ops, fw[sample] - ref) <= 1e-10 * _mass_norm(ops, ref)
