"""GPU parity at the benchmark's full sizes, on sampled outputs the oracle
computes one element (or one global DOF) at a time, in the launch
configurations the benchmark times:

* the 20x20x50 curved lattice with per-element orders 2..10 (20 000 hexes):
  Helmholtz of every mixed-order strategy, FP64 and FP32, on sampled elements
  of every order;
* the 256 independent P=5 solves (~250 000 hexes in one batched system):
  the smallest systems against the oracle's sparse direct solves, the largest
  through oracle residuals at sampled DOFs;
* the adjoint gradient kernel on the 16^3 P=6 workload with per-point kappa
  and per-element lambda, on sampled elements;
* the assembled triangle, tetrahedron, prism and pyramid solves at the
  benchmark's mesh sizes, through oracle residuals at sampled DOFs.

The 32^3 operators and the 24^3 CG solves are covered the same way in
test_gpu_ops.py and test_gpu_solve.py."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import direct_solve
from gpu_common import FP32_RTOL, FP64_RTOL, assert_close, lib_points, nk, rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_full_size_20000_mixed_orders_sampled():
    torch = torch_cuda()
    m = nk()
    cfg = W.CONFIGS[3]
    lat = W.lattice(cfg["varp_shape"])
    Pe = W.varp_orders(W.seed(3, 4), lat.nelem, *cfg["varp_P"])
    Ps = sorted(set(int(p) for p in Pe))
    jacs, xs, sels = [], [], []
    for P in Ps:
        sel = np.flatnonzero(Pe == P)
        sub = W.Lattice(lat.shape, lat.h, lat.origins[sel])
        jacs.append(to_dev(W.element_jacobians(lib_points(P, P + 2), sub, cfg["warp"])))
        xs.append(W.uniform(W.seed(3, 0) + P, (sel.size, (P + 1) ** 3)))
        sels.append(sel)
    space = m.Space.create_varp(3, Ps, [p + 2 for p in Ps], jacs)
    x = np.concatenate([v.ravel() for v in xs])
    rng = np.random.default_rng(33)
    refs, picks = [], []
    for P, sel, v in zip(Ps, sels, xs):
        pick = np.unique(np.concatenate([[0, sel.size - 1], rng.choice(sel.size, 3, replace=False)]))
        sub = W.Lattice(lat.shape, lat.h, lat.origins[sel[pick]])
        ops = oracle.ElementOps(3, P, P + 2, W.element_jacobians(oracle.gll(P + 2)[0], sub, cfg["warp"]),
                                lam=cfg["lam"])
        refs.append(ops.helmholtz_action(v[pick]))
        picks.append(pick)
    for dt, tol in ((m.F64, FP64_RTOL), (m.F32, FP32_RTOL)):
        td = torch.float64 if dt == m.F64 else torch.float32
        for strategy in range(4):
            space.set_strategy(dt, strategy)
            y = m.helmholtz(space, to_dev(x, td), lam0=1.0, dtype=dt).double().cpu().numpy()
            off = 0
            for P, sel, pick, ref in zip(Ps, sels, picks, refs):
                nm = (P + 1) ** 3
                got = y[off:off + sel.size * nm].reshape(sel.size, nm)[pick]
                assert_close(got, ref, tol, f"mixed order P={P} strategy={strategy} dt={dt}")
                off += sel.size * nm
            assert off == y.size


def _check_256(xs, info, mode, tol, err_tol, ctx):
    """NK_OK and the library's true residual <= tol for every system; the two
    smallest systems against the oracle's direct solves; the largest by
    oracle residuals at sampled free DOFs."""
    P, Q, cfg, boxes, l2gs, dms, doff, b, small, large = ctx
    assert len(info) == len(boxes)
    worst = max(i["rel_resid"] for i in info)
    assert all(i["status"] == 0 for i in info) and worst <= tol, (mode, worst)
    for k in small:
        lat = W.lattice(boxes[k])
        ops = oracle.ElementOps(3, P, Q, W.element_jacobians(oracle.gll(Q)[0], lat, cfg["warp"]), lam=1.0)
        bk = b[doff[k]:doff[k + 1]]
        ref = direct_solve(oracle.helmholtz_matrices(ops), l2gs[k], doff[k + 1] - doff[k], dms[k], bk)
        assert rel_err(xs[doff[k]:doff[k + 1]], ref) < err_tol, (k, mode)
    # the largest system: oracle residuals at sampled free DOFs
    k = large
    lat = W.lattice(boxes[k])
    bk, xk, l2g, fixed = b[doff[k]:doff[k + 1]], xs[doff[k]:doff[k + 1]].copy(), l2gs[k], dms[k].astype(bool)
    xk[fixed] = 0.0
    sample = np.random.default_rng(44).choice(np.flatnonzero(~fixed), 10, replace=False)
    hits = {int(g): np.argwhere(l2g == g) for g in sample}
    elems = np.unique(np.concatenate([h[:, 0] for h in hits.values()]))
    pos = {int(e): j for j, e in enumerate(elems)}
    ops = oracle.ElementOps(3, P, Q, W.element_jacobians(
        oracle.gll(Q)[0], W.Lattice(lat.shape, lat.h, lat.origins[elems]), cfg["warp"]), lam=1.0)
    y = ops.helmholtz_action(xk[l2g[elems]])
    habs = [np.abs(ops.helmholtz_matrix(j)) for j in range(len(elems))]
    bn = np.linalg.norm(bk)
    for g, h in hits.items():
        Ag = sum(y[pos[int(e)], mm] for e, mm in h)
        # |r_g| <= ||r||_2 <= tol ||b||_2, plus the rounding of the
        # oracle's own sum (sqrt(k) u (|A||x|)_g, k = 8 n^3 terms)
        absAg = sum((habs[pos[int(e)]] @ np.abs(xk[l2g[e]]))[mm] for e, mm in h)
        allow = 2.0 * np.sqrt(8 * (P + 1) ** 3) * 2.0 ** -53 * absAg
        assert abs(bk[g] - Ag) <= tol * bn + allow, (mode, g, abs(bk[g] - Ag) / bn)


def test_full_size_256_solves_sampled():
    """The 256 independent P=5 solves of the benchmark (log-uniform 64..4096
    hexes each) at full size, in both launch configurations it times: one
    batched system over one space, and the 256 systems created separately
    (each its own space) passed to nk_cg_solve_batched; FP64 and FP32-refined
    to 1e-10."""
    torch = torch_cuda()
    m = nk()
    cfg = W.CONFIGS[3]
    P, Q = cfg["solve_P"], cfg["solve_P"] + 2
    boxes = W.solve_boxes(W.seed(3, 5), cfg["nsolves"], *cfg["solve_sizes"])
    xq = lib_points(P, Q)
    nel = [a * b * c for a, b, c in boxes]
    E = int(sum(nel))
    J = torch.empty((E, 3, 3, Q ** 3), dtype=torch.float64, device="cuda")
    l2gs, dms, eoff, doff = [], [], [0], [0]
    for bx in boxes:
        lat = W.lattice(bx)
        J[eoff[-1]:eoff[-1] + lat.nelem] = torch.from_numpy(W.element_jacobians(xq, lat, cfg["warp"]))
        l2g, ng, dm = W.lattice_l2g(bx, P)
        l2gs.append(l2g)
        dms.append(dm)
        eoff.append(eoff[-1] + lat.nelem)
        doff.append(doff[-1] + ng)
    space = m.Space.create(3, P, Q, J)
    sysb = m.System.create_batched(space, eoff, doff,
                                   to_dev(np.concatenate([l + o for l, o in zip(l2gs, doff[:-1])]).astype(np.int32)),
                                   to_dev(np.concatenate(dms)), lam0=1.0)
    b = W.uniform(W.seed(3, 1), doff[-1])
    b[np.concatenate(dms).astype(bool)] = 0.0
    order = np.argsort(nel)
    ctx = (P, Q, cfg, boxes, l2gs, dms, doff, b, [int(k) for k in order[:2]], int(order[-1]))
    # error <= cond(A) times the residual: 1e-6 leaves room for cond(A) up to 1e4
    for mode in (m.SOLVE_F64, m.SOLVE_F32_REFINED):
        x, info = sysb.solve(to_dev(b), rtol=1e-10, maxit=50000, mode=mode)
        _check_256(x.cpu().numpy(), info, mode, 1e-10, 1e-6, ctx)
    # separately created systems in one nk_cg_solve_batched call
    singles = [m.System.create(m.Space.create(3, P, Q, J[eoff[k]:eoff[k + 1]]), doff[k + 1] - doff[k],
                               to_dev(l2gs[k]), to_dev(dms[k]), lam0=1.0) for k in range(len(boxes))]
    del J
    bs = [to_dev(b[doff[k]:doff[k + 1]]) for k in range(len(boxes))]
    for mode in (m.SOLVE_F64, m.SOLVE_F32_REFINED):
        xs, info = m.solve_batched(singles, bs, rtol=1e-10, maxit=50000, mode=mode)
        _check_256(torch.cat(xs).cpu().numpy(), info, mode, 1e-10, 1e-6, ctx)


def test_full_size_16c_gradient_kernel_sampled():
    torch_cuda()
    m = nk()
    cfg = W.CONFIGS[4]
    P, Q = cfg["P"], cfg["Q"]
    lat = W.lattice(cfg["shape"])
    E, nq, nm = lat.nelem, Q ** 3, (P + 1) ** 3
    kap = W.uniform(W.seed(4, 3), (E, nq), *cfg["coef_range"])
    lam = W.uniform(W.seed(4, 2), (E,), *cfg["coef_range"])
    space = m.Space.create(3, P, Q, to_dev(W.element_jacobians(lib_points(P, Q), lat, cfg["warp"])),
                           kappa=to_dev(kap))
    ul = W.uniform(W.seed(4, 0), (E, nm))
    zl = W.uniform(W.seed(4, 1), (E, nm))
    dk, dl = m.param_grad(space, to_dev(zl.ravel()), to_dev(ul.ravel()))
    dk = dk.cpu().numpy().reshape(E, nq)
    dl = dl.cpu().numpy()
    pick = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(45).choice(E, 3, replace=False)]))
    sub = W.Lattice(lat.shape, lat.h, lat.origins[pick])
    ops = oracle.ElementOps(3, P, Q, W.element_jacobians(oracle.gll(Q)[0], sub, cfg["warp"]),
                            kappa=kap[pick], lam=lam[pick])
    loc = np.arange(pick.size * nm).reshape(pick.size, nm)
    dk_ref, dl_ref = oracle.param_grad(ops, loc, ul[pick].ravel(), zl[pick].ravel())
    assert_close(dk[pick], dk_ref, FP64_RTOL, "full-size dkappa")
    assert_close(dl[pick], dl_ref, FP64_RTOL, "full-size dlambda")


# ------------------- collapsed-shape solves at the benchmark's mesh sizes

def _collapsed_case(shape, P):
    """(space, system, l2g, sign, nglobal, dirichlet, oracle-ops factory over
    element subsets) for the benchmark's triangle, tetrahedron, prism and
    pyramid solve meshes."""
    from oracle import collapsed as C
    m = nk()
    Q = P + 2
    g = oracle.gll(Q)[0]
    r1 = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)[0]
    r2 = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)[0]
    sign = None
    if shape == "tri":
        n = 128
        rot = W.tri_rotations(W.seed(5, 7), 2 * n * n)
        e1, _, e2, _ = m.tri_points(Q)
        space = m.Space.create_tri(P, Q, to_dev(W.tri_lattice_jacobians(n, e1, e2, 0.05, rot)))
        l2g, sign, ng, dm = W.tri_lattice_l2g(n, P, rot)
        Jo = W.tri_lattice_jacobians(n, g, r1, 0.05, rot)
        factory = lambda el: C.TriOps(P, Q, Jo[el])
    elif shape == "tet":
        n = 12
        e1, _, e2, _, e3, _ = m.tet_points(Q)
        space = m.Space.create_tet(P, Q, to_dev(W.tet_lattice_jacobians(n, e1, e2, e3, sorted_ids=True)))
        l2g, ng, dm = W.tet_lattice_l2g(n, P)
        factory = lambda el: C.TetOps(P, Q, W.tet_lattice_jacobians(n, g, r1, r2, elems=el, sorted_ids=True))
    elif shape == "prism":
        n = 16
        rot = W.tri_rotations(W.seed(2, 7), 2 * n * n)
        e1, _, e2, _ = m.tri_points(Q)
        space = m.Space.create_prism(P, Q, to_dev(W.prism_lattice_jacobians(n, e1, e2, e1, rot=rot)))
        l2g, sign, ng, dm = W.prism_lattice_l2g(n, P, rot)
        factory = lambda el: C.PrismOps(P, Q, W.prism_lattice_jacobians(n, g, r1, g, elems=el, rot=rot))
    else:
        n = 10
        xg = m.basis_tables(P, Q)[0]
        space = m.Space.create_pyr(P, Q, to_dev(W.pyr_lattice_jacobians(n, xg, xg, m.tet_points(Q)[4])))
        l2g, ng, dm = W.pyr_lattice_l2g(n, P)
        factory = lambda el: C.PyrOps(P, Q, W.pyr_lattice_jacobians(n, g, g, r2, elems=el))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam0=1.0,
                           sign=None if sign is None else to_dev(sign))
    return space, sysm, l2g, sign, ng, dm, factory


@pytest.mark.parametrize("shape", ["tri", "tet", "prism", "pyr"])
@pytest.mark.parametrize("P", [4, 6])
def test_full_size_collapsed_solves_sampled_residuals(shape, P):
    """The benchmark's assembled triangle (32 768), tetrahedron (10 368),
    prism (8 192) and pyramid (6 000) solves at full size, FP64 and
    FP32-refined to 1e-10 on a seeded right-hand side: the oracle recomputes
    (A x)_g from the dense elemental matrices of the elements that hold a
    seeded sample of free DOFs (with orientation signs), and every sampled
    residual obeys |b_g - (A x)_g| <= 1e-10 ||b||_2 (implied by NK_OK) up to
    the rounding of the oracle's own sum."""
    m = nk()
    torch_cuda()
    space, sysm, l2g, sign, ng, dm, factory = _collapsed_case(shape, P)
    fixed = dm.astype(bool)
    b = W.uniform(W.seed(2, 3) + P, ng)
    b[fixed] = 0.0
    free = np.flatnonzero(~fixed)
    sample = np.random.default_rng(50 + P).choice(free, 12, replace=False)
    hits = {int(gd): np.argwhere(l2g == gd) for gd in sample}
    elems = np.unique(np.concatenate([h[:, 0] for h in hits.values()]))
    pos = {int(e): k for k, e in enumerate(elems)}
    ops = factory(elems)
    mats = [ops.helmholtz_matrix(k) for k in range(len(elems))]
    sg = np.ones_like(l2g, dtype=np.float64) if sign is None else sign.astype(np.float64)
    bn = np.linalg.norm(b)
    for mode in (m.SOLVE_F64, m.SOLVE_F32_REFINED):
        x, info = sysm.solve(to_dev(b), rtol=1e-10, maxit=50000, mode=mode)
        assert info[0]["status"] == 0 and info[0]["rel_resid"] <= 1e-10
        xs = x.cpu().numpy().copy()
        xs[fixed] = 0.0
        for gd, h in hits.items():
            Ag = absAg = 0.0
            for e, mm in h:
                k = pos[int(e)]
                ye = mats[k] @ (sg[e] * xs[l2g[e]])
                Ag += sg[e, mm] * ye[mm]
                absAg += (np.abs(mats[k]) @ np.abs(xs[l2g[e]]))[mm]
            # rounding of the oracle's own sum: sqrt(k) u (|A||x|)_g
            allow = 2.0 * np.sqrt(8 * mats[0].shape[1]) * 2.0 ** -53 * absAg
            assert abs(b[gd] - Ag) <= 1e-10 * bn + allow, (shape, P, mode, gd, abs(b[gd] - Ag) / bn)
