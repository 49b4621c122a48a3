"""GPU parity of the elemental operators against the FP64 oracle.

BwdTrans, IProductWRTBase and the local Helmholtz operator through the C ABI,
FP64 (<= 1e-12 relative) and FP32 (<= 2e-6 relative), for 2-D quads and
curved 3-D hexes at every compiled order, every tile configuration, ragged
element counts, per-element lambda and per-point kappa; the mixed-order
persistent launch; the weak right-hand side; full-size sampled checks on the
32^3, P=6 workload."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import (FP32_RTOL, FP64_RTOL, assert_close, jacobians, nk, to_dev,
                        torch_cuda)

pytestmark = pytest.mark.gpu


def _run_all(space, dim, P, coeffs, f, lam, dtype):
    torch = torch_cuda()
    m = nk()
    td = torch.float64 if dtype == m.F64 else torch.float32
    c = to_dev(coeffs, td).reshape(-1)
    ff = to_dev(f, td).reshape(-1)
    lamd = to_dev(lam) if lam is not None else None
    u = m.bwd_trans(space, c, dtype=dtype)
    ip = m.iprod_wrt_base(space, ff, dtype=dtype)
    h = m.helmholtz(space, c, lam=lamd, lam0=1.0, dtype=dtype)
    torch.cuda.synchronize()
    return [t.double().cpu().numpy() for t in (u, ip, h)]


def _oracle_all(ops, coeffs, f):
    return ops.bwd(coeffs).ravel(), ops.iprod(f).ravel(), ops.helmholtz(coeffs).ravel()


def test_config0_quads_2d():
    """8x8 affine quads on [0,1]^2, P=4, Q=6, lambda=1 (the 2-D workload)."""
    torch_cuda()
    m = nk()
    cfg = W.CONFIGS[0]
    P, Q = cfg["P"], cfg["Q"]
    Jg, Jo, lat = jacobians(cfg["shape"], P, 0.0)
    E = lat.nelem
    coeffs = W.uniform(W.seed(0, 0), (E, (P + 1) ** 2))
    f = W.uniform(W.seed(0, 1), (E, Q ** 2))
    ops = oracle.ElementOps(2, P, Q, Jo, lam=1.0)
    ref = _oracle_all(ops, coeffs, f)
    space = m.Space.create(2, P, Q, to_dev(Jg))
    for dtype, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        got = _run_all(space, 2, P, coeffs, f, None, dtype)
        for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
            assert_close(g, r, tol, f"2d {name} dtype={dtype}")


# elements per order: > largest tile + ragged tail, bounded by oracle cost
_N3 = {1: 61, 2: 35, 3: 23, 4: 17, 5: 13, 6: 9, 7: 7, 8: 5, 9: 5, 10: 3}


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_curved_hex_all_orders_all_tiles(P):
    torch_cuda()
    m = nk()
    Q = P + 2
    E = _N3[P]
    Jg, Jo, lat = jacobians((4, 4, 4), P, W.WARP_AMPLITUDE, nelem=E)
    rng = np.random.default_rng(100 + P)
    coeffs = rng.uniform(-1, 1, (E, (P + 1) ** 3))
    f = rng.uniform(-1, 1, (E, Q ** 3))
    lam = rng.uniform(0.5, 2.0, E)
    kap = rng.uniform(0.5, 2.0, (E, Q ** 3))
    ops = oracle.ElementOps(3, P, Q, Jo, kappa=kap, lam=lam)
    ref = _oracle_all(ops, coeffs, f)
    space = m.Space.create(3, P, Q, to_dev(Jg), kappa=to_dev(kap))
    for dtype, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        for op in (m.OP_BWD, m.OP_IPROD, m.OP_HELM):
            nt = m.tile_count(op, 3, P)
            assert nt >= 1
        ntiles = max(m.tile_count(op, 3, P) for op in (0, 1, 2))
        for tile in range(ntiles):
            for op in (0, 1, 2):
                m.set_tile_config(op, 3, P, dtype, min(tile, m.tile_count(op, 3, P) - 1))
            got = _run_all(space, 3, P, coeffs, f, lam, dtype)
            for name, g, r in zip(("bwd", "iprod", "helm"), got, ref):
                assert_close(g, r, tol, f"P={P} tile={tile} {name} dtype={dtype}")
        for op in (0, 1, 2):
            m.set_tile_config(op, 3, P, dtype, 0)


def test_empty_space_is_noop():
    torch = torch_cuda()
    m = nk()
    J = torch.zeros((0, 3, 3, 512), dtype=torch.float64, device="cuda")
    space = m.Space.create(3, 6, 8, J)
    assert space.sizes() == (0, 0, 0)
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    y = m.helmholtz(space, x, torch.zeros(1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert y.shape == (1,)


def test_invalid_jacobian_rejected():
    torch = torch_cuda()
    m = nk()
    Jg, _, _ = jacobians((1, 1, 2), 2, 0.0)
    Jg[1, 0, 0, 3] = -1.0           # one point with negative detJ
    with pytest.raises(m.NkError) as ei:
        m.Space.create(3, 2, 4, to_dev(Jg))
    assert ei.value.status == 1       # NK_EINVAL


def test_mixed_order_single_launch():
    """Elements of orders 2..10 in one persistent launch == per-element oracle."""
    torch = torch_cuda()
    m = nk()
    Ps = [10, 2, 7, 5, 3, 9, 4, 8, 6]          # deliberately unsorted
    counts = {2: 37, 3: 21, 4: 15, 5: 11, 6: 9, 7: 5, 8: 3, 9: 3, 10: 2}
    rng = np.random.default_rng(7)
    jg, coeffs, refs, lams = [], [], [], []
    for P in Ps:
        Jg, Jo, _ = jacobians((4, 4, 4), P, W.WARP_AMPLITUDE, nelem=counts[P])
        E = counts[P]
        c = rng.uniform(-1, 1, (E, (P + 1) ** 3))
        lam = rng.uniform(0.5, 2.0, E)
        ops = oracle.ElementOps(3, P, P + 2, Jo, lam=lam)
        refs.append(ops.helmholtz(c).ravel())
        jg.append(to_dev(Jg))
        coeffs.append(c.ravel())
        lams.append(lam)
    space = m.Space.create_varp(3, Ps, [p + 2 for p in Ps], jg)
    x = to_dev(np.concatenate(coeffs))
    lam = to_dev(np.concatenate(lams))
    for dtype, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dtype == m.F64 else torch.float32
        for strategy in range(4):
            space.set_strategy(dtype, strategy)
            y = m.helmholtz(space, x.to(td), lam=lam, dtype=dtype).double().cpu().numpy()
            off = 0
            for P, r in zip(Ps, refs):
                assert_close(y[off:off + r.size], r, tol, f"varp P={P} dtype={dtype} strategy={strategy}")
                off += r.size
            assert off == y.size
    # BwdTrans on the mixed-order space (concurrent per-group launches)
    c64 = x
    u = m.bwd_trans(space, c64).cpu().numpy()
    off_c = off_u = 0
    for P in Ps:
        Jg, Jo, _ = jacobians((4, 4, 4), P, W.WARP_AMPLITUDE, nelem=counts[P])
        n3, q3 = (P + 1) ** 3, (P + 2) ** 3
        c = x[off_c:off_c + counts[P] * n3].cpu().numpy().reshape(counts[P], n3)
        ref = oracle.ElementOps(3, P, P + 2, Jo).bwd(c).ravel()
        assert_close(u[off_u:off_u + ref.size], ref, FP64_RTOL, f"varp bwd P={P}")
        off_c += counts[P] * n3
        off_u += ref.size


def test_weak_rhs_matches_oracle():
    torch = torch_cuda()
    m = nk()
    P, Q = 4, 6
    Jg, Jo, lat = jacobians((3, 2, 2), P, W.WARP_AMPLITUDE)
    E = lat.nelem
    rng = np.random.default_rng(11)
    lam = rng.uniform(0.5, 2, E)
    U, dU = W.manufactured_ref_gradient(oracle.gll(Q)[0], lat)
    Ug, dUg = W.manufactured_ref_gradient(m.basis_tables(P, Q)[0], lat)
    ops = oracle.ElementOps(3, P, Q, Jo, lam=lam)
    ref = ops.weak_rhs(U, dU).ravel()
    space = m.Space.create(3, P, Q, to_dev(Jg))
    y = m.helmholtz_weak_rhs(space, to_dev(Ug).reshape(-1), to_dev(dUg).reshape(-1), lam=to_dev(lam))
    assert_close(y.cpu().numpy(), ref, FP64_RTOL, "weak rhs")


def test_full_size_32cube_p6_sampled():
    """The 32^3, P=6 curved workload at full size; oracle on sampled elements
    (first, last, and a seeded random sample)."""
    torch = torch_cuda()
    m = nk()
    cfg = W.CONFIGS[1]
    P, Q = cfg["P"], cfg["Q"]
    lat = W.lattice(cfg["shape"])
    E = lat.nelem
    Jg = W.element_jacobians(m.basis_tables(P, Q)[0], lat, cfg["warp"])
    coeffs = W.uniform(W.seed(1, 0), (E, (P + 1) ** 3))
    f = W.uniform(W.seed(1, 1), (E, Q ** 3))
    space = m.Space.create(3, P, Q, to_dev(Jg))
    del Jg
    got = _run_all(space, 3, P, coeffs, f, None, m.F64)
    got32 = _run_all(space, 3, P, coeffs, f, None, m.F32)
    sample = np.unique(np.concatenate([[0, 1, E - 1], np.random.default_rng(5).choice(E, 13, replace=False)]))
    Jo = W.element_jacobians(oracle.gll(Q)[0], W.Lattice(lat.shape, lat.h, lat.origins[sample]), cfg["warp"])
    ops = oracle.ElementOps(3, P, Q, Jo, lam=cfg["lam"])
    ref = [ops.bwd(coeffs[sample]), ops.iprod(f[sample]), ops.helmholtz(coeffs[sample])]
    nq, nm = Q ** 3, (P + 1) ** 3
    for k, (name, g, r) in enumerate(zip(("bwd", "iprod", "helm"), got, ref)):
        width = nq if k == 0 else nm
        gs = g.reshape(E, width)[sample]
        assert_close(gs, r, FP64_RTOL, f"full-size {name}")
        assert_close(got32[k].reshape(E, width)[sample], r, FP32_RTOL, f"full-size {name} f32")
