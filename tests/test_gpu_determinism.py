"""Repeatability and tile agreement of the GPU kernels.

Kernels without atomics (every elemental operator: BwdTrans,
IProductWRTBase, local Helmholtz, PhysDeriv, IProductWRTDerivBase,
FwdTrans; the triangle and collapsed 3-D operators; the mixed-order launch)
give bit-identical results when run twice on the same input.  Every tile
configuration of a 3-D operator, the matrix-core Helmholtz included, agrees
with the first tile to 1e-13 relative in FP64 (the tiles reorder no sums
except the matrix-core form, which pads its contractions).  The assembled
operator adds its element contributions with atomics, so two runs may differ
in the order of those additions: within 1e-14 relative."""
import numpy as np
import pytest

import workloads as W
from gpu_common import jacobians, lib_points, nk, rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _twice(fn):
    torch = torch_cuda()
    a = fn().clone()
    b = fn().clone()
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("P", [2, 5, 6, 8, 10])
def test_hex_operators_bitwise_repeatable(P):
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, _, lat = jacobians((5, 4, 3), P, W.WARP_AMPLITUDE)
    E = lat.nelem
    rng = np.random.default_rng(700 + P)
    space = m.Space.create(3, P, Q, to_dev(Jg))
    for dt, td in ((m.F64, torch.float64), (m.F32, torch.float32)):
        c = to_dev(rng.uniform(-1, 1, E * (P + 1) ** 3), td)
        f = to_dev(rng.uniform(-1, 1, E * Q ** 3), td)
        g = to_dev(rng.uniform(-1, 1, 3 * E * Q ** 3), td)
        for name, fn in (("bwd", lambda: m.bwd_trans(space, c, dtype=dt)),
                         ("iprod", lambda: m.iprod_wrt_base(space, f, dtype=dt)),
                         ("helm", lambda: m.helmholtz(space, c, lam0=1.3, dtype=dt)),
                         ("deriv", lambda: m.phys_deriv(space, f, dtype=dt)),
                         ("iprod_deriv", lambda: m.iprod_wrt_deriv_base(space, g, dtype=dt)),
                         ("fwd", lambda: m.fwd_trans(space, f, dtype=dt))):
            a, b = _twice(fn)
            assert np.array_equal(a, b), f"{name} P={P} dtype={dt} not bitwise repeatable"


@pytest.mark.parametrize("P", [3, 4, 6, 8])
def test_hex_tiles_agree(P):
    """Each tile of BwdTrans, IProductWRTBase and Helmholtz against tile 0,
    FP64 to 1e-13 and FP32 to 1e-6 relative."""
    torch = torch_cuda()
    m = nk()
    Q = P + 2
    Jg, _, lat = jacobians((5, 3, 3), P, W.WARP_AMPLITUDE)
    E = lat.nelem
    rng = np.random.default_rng(800 + P)
    lam = to_dev(rng.uniform(0.5, 2.0, E))
    space = m.Space.create(3, P, Q, to_dev(Jg))
    try:
        for dt, td, tol in ((m.F64, torch.float64, 1e-13), (m.F32, torch.float32, 1e-6)):
            c = to_dev(rng.uniform(-1, 1, E * (P + 1) ** 3), td)
            f = to_dev(rng.uniform(-1, 1, E * Q ** 3), td)
            runs = {m.OP_BWD: lambda: m.bwd_trans(space, c, dtype=dt),
                    m.OP_IPROD: lambda: m.iprod_wrt_base(space, f, dtype=dt),
                    m.OP_HELM: lambda: m.helmholtz(space, c, lam=lam, dtype=dt)}
            for op, fn in runs.items():
                m.set_tile_config(op, 3, P, dt, 0)
                ref = fn().double().cpu().numpy()
                for tile in range(1, m.tile_count(op, 3, P)):
                    m.set_tile_config(op, 3, P, dt, tile)
                    got = fn().double().cpu().numpy()
                    e = rel_err(got, ref)
                    assert e <= tol, (op, P, dt, m.tile_config(op, 3, P, dt), e)
                m.set_tile_config(op, 3, P, dt, 0)
    finally:
        for dt in (m.F64, m.F32):
            for op in (m.OP_BWD, m.OP_IPROD, m.OP_HELM):
                m.set_tile_config(op, 3, P, dt, 0)


@pytest.mark.parametrize("shape", ["tri", "tet", "prism", "pyr"])
def test_collapsed_operators_bitwise_repeatable(shape):
    torch = torch_cuda()
    m = nk()
    P = 5
    Q = P + 2
    if shape == "tri":
        e1, _, e2, _ = m.tri_points(Q)
        space = m.Space.create_tri(P, Q, to_dev(W.tri_lattice_jacobians(6, e1, e2, 0.05)))
        nm, npt = (P + 1) * (P + 2) // 2, Q * (Q - 1)
    elif shape == "tet":
        e1, _, e2, _, e3, _ = m.tet_points(Q)
        space = m.Space.create_tet(P, Q, to_dev(W.tet_lattice_jacobians(3, e1, e2, e3)))
        nm, npt = (P + 1) * (P + 2) * (P + 3) // 6, Q * (Q - 1) ** 2
    elif shape == "prism":
        e1, _, e2, _ = m.tri_points(Q)
        space = m.Space.create_prism(P, Q, to_dev(W.prism_lattice_jacobians(3, e1, e2, e1)))
        nm, npt = (P + 1) ** 2 * (P + 2) // 2, Q * Q * (Q - 1)
    else:
        xg = lib_points(P, Q)
        space = m.Space.create_pyr(P, Q, to_dev(W.pyr_lattice_jacobians(3, xg, xg, m.tet_points(Q)[4])))
        nm, npt = (P + 1) * (P + 2) * (2 * P + 3) // 6, Q * Q * (Q - 1)
    E = space.sizes()[0]
    rng = np.random.default_rng(900)
    for dt, td in ((m.F64, torch.float64), (m.F32, torch.float32)):
        c = to_dev(rng.uniform(-1, 1, E * nm), td)
        f = to_dev(rng.uniform(-1, 1, E * npt), td)
        for name, fn in (("bwd", lambda: m.bwd_trans(space, c, dtype=dt)),
                         ("iprod", lambda: m.iprod_wrt_base(space, f, dtype=dt)),
                         ("helm", lambda: m.helmholtz(space, c, lam0=0.7, dtype=dt))):
            a, b = _twice(fn)
            assert np.array_equal(a, b), f"{shape} {name} dtype={dt} not bitwise repeatable"


def test_mixed_order_launch_repeatable_and_strategies_agree():
    """The mixed-order space: each strategy twice gives identical bits, and
    the strategies agree with each other to 1e-13 (the per-order launches
    use each order's tuned tile)."""
    torch = torch_cuda()
    m = nk()
    Ps = [2, 3, 5, 7, 10]
    jacs, xs = [], []
    for k, P in enumerate(Ps):
        Jg, _, lat = jacobians((3, 2, 2), P, W.WARP_AMPLITUDE)
        jacs.append(to_dev(Jg))
        xs.append(np.random.default_rng(950 + k).uniform(-1, 1, lat.nelem * (P + 1) ** 3))
    space = m.Space.create_varp(3, Ps, [P + 2 for P in Ps], jacs)
    x = to_dev(np.concatenate(xs))
    ref = None
    for strategy in range(4):
        space.set_strategy(m.F64, strategy)
        a, b = _twice(lambda: m.helmholtz(space, x, lam0=1.0))
        assert np.array_equal(a, b), f"strategy {strategy} not bitwise repeatable"
        if ref is None:
            ref = a
        assert rel_err(a, ref) <= 1e-13, f"strategy {strategy} differs from strategy 0"


def test_assembled_operator_repeatable_to_rounding():
    """Atomic scatter-add: two applications agree to 1e-14 relative."""
    torch = torch_cuda()
    m = nk()
    P, shape = 5, (4, 3, 3)
    Jg, _, _ = jacobians(shape, P, W.WARP_AMPLITUDE)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    space = m.Space.create(3, P, P + 2, to_dev(Jg))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam0=1.0)
    x = to_dev(np.random.default_rng(990).uniform(-1, 1, ng))
    a, b = _twice(lambda: sysm.apply(x))
    assert rel_err(a, b) <= 1e-14
