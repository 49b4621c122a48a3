#!/usr/bin/env python3
"""Benchmark of the matrix-free spectral/hp hot path on one MI355X.

Timed steps: one FP64 Helmholtz application (matrix-free, sum-factorised,
per-point geometric factors) over 32^3 curved hexahedra at P=6 (Q=8 GLL
points), 11 239 424 local DOF, inputs resident in HBM.  `value` is local
GDOF/s of that step.  The same JSON line carries measured sections for the
other operators (BwdTrans, IProductWRTBase, FP32 Helmholtz), the assembled CG
solves at P=4, 6, 8 on 24^3 curved hexes in FP64 and FP32-refined modes, the
mixed-order single launch and the batched solves, the adjoint gradient, the
roofline of the dominant kernel and the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Helmholtz op GDOF/s & CG solve time, FP64 vs FP32-refined, P=4..8 hexes; % roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def helm_bytes_per_elem(P, Q, s=8):
    """Algorithmic bytes of one Helmholtz element: coefficients in and out
    (2 n^3) and 7 per-point geometric factors (7 Q^3)."""
    n = P + 1
    return s * (2 * n ** 3 + 7 * Q ** 3)


def bwd_bytes_per_elem(P, Q, s=8):
    return s * ((P + 1) ** 3 + Q ** 3)


def iprod_bytes_per_elem(P, Q, s=8):
    return s * ((P + 1) ** 3 + 2 * Q ** 3)


KERNEL_SOURCES = ["paper_1906_03489_amd/csrc/engine.h", "paper_1906_03489_amd/csrc/ops3d_inst.hip",
                  "paper_1906_03489_amd/csrc/tiles.h", "paper_1906_03489_amd/csrc/tables.h"]
PMC_SUMMARY = "profiles/helmholtz_f64_32c_P6_pmc.txt"


def measured_traffic():
    """HBM bytes per launch of the FP64 Helmholtz kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None if
    the kernel sources changed since those counters were taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        vals, digest = {}, None
        with open(os.path.join(ROOT, PMC_SUMMARY)) as fh:
            for line in fh:
                if "kernel sources hash" in line:
                    digest = line.split(":")[-1].strip()
                elif line.strip() and not line.startswith("#"):
                    k, v = line.split()
                    vals[k] = float(v)
        if digest != h.hexdigest()[:16]:
            return None
        return int(vals["helm_traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


FWD_FLOPS_SUMMARY = "profiles/fwd_trans_32c_P6_flops.txt"
FWD_SOURCES = ["paper_1906_03489_amd/csrc/deriv.hip", "paper_1906_03489_amd/csrc/engine.h",
               "paper_1906_03489_amd/csrc/tables.h", "paper_1906_03489_amd/csrc/tiles.h"]
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def fwd_trans_flops():
    """Issued lane-flops per element of FwdTrans (32^3, P=6) per dtype from
    the committed rocprofv3 flop-counter summary, or {} once the kernel
    sources changed since those counters were taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in FWD_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        vals, digest = {}, None
        with open(os.path.join(ROOT, FWD_FLOPS_SUMMARY)) as fh:
            for line in fh:
                if "kernel sources hash" in line:
                    digest = line.split(":")[-1].strip()
                elif line.strip() and not line.startswith("#"):
                    k, v = line.split()
                    vals[k] = float(v)
        if digest != h.hexdigest()[:16]:
            return {}
        return {"f64": vals["flops_per_elem_f64"], "f32": vals["flops_per_elem_f32"]}
    except (OSError, KeyError, ValueError):
        return {}


def time_launches(fn, n, torch):
    """Average ms per call of fn over n back-to-back calls, HIP events on
    the current stream (the stream the kernels are launched on)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def device_copy_gbs(torch, n=1 << 28, reps=10):
    """Achievable HBM rate of a streaming copy (2 GiB read + 2 GiB written
    per pass, far beyond the 256 MB cache), as the practical ceiling beside
    the 8 TB/s datasheet peak: the better of a device-to-device memcpy and an
    elementwise kernel that reads one array and writes another (the latter
    is faster on this chip: ~5.7 vs ~4.8 TB/s)."""
    src = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = 0.0
    for f in (lambda: dst.copy_(src), lambda: torch.mul(src, 1.0, out=dst)):
        for _ in range(2):
            f()
        ms = time_launches(f, reps, torch)
        best = max(best, 2 * n * 8 / (ms * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def make_space(nk, W, shape, P, amp, torch, kappa=None):
    Q = P + 2
    lat = W.lattice(shape)
    J = W.element_jacobians(nk.basis_tables(P, Q)[0], lat, amp)
    Jd = torch.from_numpy(J).cuda()
    del J
    sp = nk.Space.create(3, P, Q, Jd, kappa=kappa)
    del Jd
    return sp, lat


ROTATE_BYTES = 640e6   # rotation working set per operator: beyond the 256 MB Infinity Cache


def rotation_count(bytes_per_launch, floor=3, cap=64):
    """Buffer sets (or spaces) to rotate over so that the data of one launch
    is not in the 256 MB Infinity Cache when its set comes round again."""
    return int(min(cap, max(floor, -(-ROTATE_BYTES // max(bytes_per_launch, 1)))))


def time_elementwise_ops(nk, W, torch, spaces_fn, E, nm, npt, nfac, reps):
    """BwdTrans / IProductWRTBase / Helmholtz of a collapsed-shape space,
    FP64 and FP32.  Each operator is timed over a rotation of rotation_count
    launches whose data are all distinct: buffer sets, and for the operators
    that read the geometric factors, spaces built from the same Jacobians
    (spaces_fn(k) returns k of them), so the rotation spans at least
    ROTATE_BYTES.  Algorithmic bytes per element (s bytes per scalar):
    BwdTrans s(nm + np), IProductWRTBase s(nm + 2 np) (values and w detJ),
    Helmholtz s(2 nm + nfac np)."""
    res = {}
    # the factor-reading operator with the fewest bytes per launch sets the space count
    nsp = rotation_count(4 * (2 * npt + nm) * E)
    spaces = spaces_fn(nsp)
    for dt, name, s in ((nk.F64, "f64", 8), (nk.F32, "f32", 4)):
        td = torch.float64 if dt == nk.F64 else torch.float32
        ops = (("bwd_trans", s * (nm + npt)), ("iprod_wrt_base", s * (2 * npt + nm)),
               ("helmholtz", s * (2 * nm + nfac * npt)))
        nb = max(rotation_count(b * E) for _, b in ops)
        cs = [torch.from_numpy(W.uniform(W.seed(1, 0) + k, E * nm)).to(td).cuda() for k in range(nb)]
        fs = [torch.from_numpy(W.uniform(W.seed(1, 1) + k, E * npt)).to(td).cuda() for k in range(nb)]
        us = [torch.empty(E * npt, dtype=td, device="cuda") for _ in range(nb)]
        ys = [torch.empty(E * nm, dtype=td, device="cuda") for _ in range(nb)]
        fns = {"bwd_trans": lambda k: nk.bwd_trans(spaces[k % nsp], cs[k], us[k], dtype=dt),
               "iprod_wrt_base": lambda k: nk.iprod_wrt_base(spaces[k % nsp], fs[k], ys[k], dtype=dt),
               "helmholtz": lambda k: nk.helmholtz(spaces[k % nsp], cs[k], ys[k], lam0=1.0, dtype=dt)}
        for op, bpe in ops:
            nrot = rotation_count(bpe * E)
            fn = fns[op]
            for k in range(nrot):
                fn(k)
            cnt = [0]

            def step():
                fn(cnt[0] % nrot)
                cnt[0] += 1
            ms = time_launches(step, max(reps, nrot), torch)
            gbs = bpe * E / (ms * 1e-3) / 1e9
            res[f"{op}_{name}"] = {"ms": round(ms, 5), "gdof_s": round(E * nm / (ms * 1e-3) / 1e9, 3),
                                   "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "rotation": nrot, "rotation_MB": round(nrot * bpe * E / 1e6, 1)}
        del cs, fs, us, ys
    del spaces
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------ sections

def section_ops(nk, W, torch, space, lat, P, Q, reps):
    """BwdTrans, IProductWRTBase and Helmholtz on the 32^3 workload, FP64
    and FP32; inputs rotate over enough buffers to exceed the 256 MB cache."""
    E = lat.nelem
    n3, q3 = (P + 1) ** 3, Q ** 3
    out = {}
    for dt, name, s in ((nk.F64, "f64", 8), (nk.F32, "f32", 4)):
        td = torch.float64 if dt == nk.F64 else torch.float32
        nset = 3
        cs = [torch.from_numpy(W.uniform(W.seed(1, 0) + k, E * n3)).to(td).cuda() for k in range(nset)]
        fs = [torch.from_numpy(W.uniform(W.seed(1, 1) + k, E * q3)).to(td).cuda() for k in range(nset)]
        us = [torch.empty(E * q3, dtype=td, device="cuda") for _ in range(nset)]
        ys = [torch.empty(E * n3, dtype=td, device="cuda") for _ in range(nset)]
        for op, bpe, fn in (
            ("bwd_trans", bwd_bytes_per_elem(P, Q, s), lambda k: nk.bwd_trans(space, cs[k], us[k], dtype=dt)),
            ("iprod_wrt_base", iprod_bytes_per_elem(P, Q, s),
             lambda k: nk.iprod_wrt_base(space, fs[k], ys[k], dtype=dt)),
            ("helmholtz", helm_bytes_per_elem(P, Q, s),
             lambda k: nk.helmholtz(space, cs[k], ys[k], lam0=1.0, dtype=dt)),
        ):
            for k in range(nset):
                fn(k)
            cnt = [0]

            def step():
                fn(cnt[0] % nset)
                cnt[0] += 1
            ms = time_launches(step, reps, torch)
            gbs = bpe * E / (ms * 1e-3) / 1e9
            out[f"{op}_{name}"] = {"ms": round(ms, 5), "gdof_s": round(E * n3 / (ms * 1e-3) / 1e9, 3),
                                   "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "tile": nk.tile_config({"bwd_trans": 0, "iprod_wrt_base": 1,
                                                           "helmholtz": 2}[op], 3, P, dt)}
        # every compiled Helmholtz candidate (vector tiles and the matrix-core variant)
        chosen = None
        nt = nk.tile_count(2, 3, P)
        per_tile = {}
        for k in range(nt):
            nk.set_tile_config(2, 3, P, dt, k)
            name_k = nk.tile_config(2, 3, P, dt)
            nk.helmholtz(space, cs[0], ys[0], lam0=1.0, dtype=dt)
            cnt = [0]

            def step_t():
                nk.helmholtz(space, cs[cnt[0] % nset], ys[cnt[0] % nset], lam0=1.0, dtype=dt)
                cnt[0] += 1
            ms = time_launches(step_t, reps, torch)
            gbs = helm_bytes_per_elem(P, Q, s) * E / (ms * 1e-3) / 1e9
            per_tile[name_k] = {"ms": round(ms, 5), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        out[f"helmholtz_all_tiles_{name}"] = per_tile
        nk.autotune(space, 0b100)
        del cs, fs, us, ys
        torch.cuda.empty_cache()
    return out


def section_deriv(nk, W, torch, space, lat, P, Q, reps):
    """PhysDeriv, IProductWRTDerivBase and FwdTrans on the 32^3 workload,
    FP64 and FP32, inputs rotating over buffer sets larger than the 256 MB
    cache.  Algorithmic bytes per element: PhysDeriv s(Q^3 + 3Q^3 + 9Q^3)
    (values, gradient, J^{-1}); IProductWRTDerivBase s(3Q^3 + 10Q^3 + n^3)
    (field, J^{-1} and w detJ, coefficients); FwdTrans s(2Q^3 + n^3) (values,
    w detJ, coefficients): its CG iterations run on chip, so it is bound by
    arithmetic, not HBM, and hbm_frac only says how far; its "alu" roofline
    takes the issued flops per element from the committed counter summary
    against the vector peak.  gdof_s counts the element's n^3 modes per
    second for all three."""
    E = lat.nelem
    n3, q3 = (P + 1) ** 3, Q ** 3
    fwd_flops = fwd_trans_flops() if (P, Q, E) == (6, 8, 32768) else {}
    out = {}
    for dt, name, s in ((nk.F64, "f64", 8), (nk.F32, "f32", 4)):
        td = torch.float64 if dt == nk.F64 else torch.float32
        nset = 3
        us = [torch.from_numpy(W.uniform(W.seed(1, 1) + k, E * q3)).to(td).cuda() for k in range(nset)]
        fs = [torch.from_numpy(W.uniform(W.seed(1, 1) + 10 + k, 3 * E * q3)).to(td).cuda()
              for k in range(nset)]
        dus = [torch.empty(3 * E * q3, dtype=td, device="cuda") for _ in range(nset)]
        cs = [torch.empty(E * n3, dtype=td, device="cuda") for _ in range(nset)]
        for op, bpe, bound, fn in (
            ("phys_deriv", s * 13 * q3, "hbm", lambda k: nk.phys_deriv(space, us[k], dus[k], dtype=dt)),
            ("iprod_wrt_deriv_base", s * (13 * q3 + n3), "hbm",
             lambda k: nk.iprod_wrt_deriv_base(space, fs[k], cs[k], dtype=dt)),
            ("fwd_trans", s * (2 * q3 + n3), "alu", lambda k: nk.fwd_trans(space, us[k], cs[k], dtype=dt)),
        ):
            for k in range(nset):
                fn(k)
            cnt = [0]

            def step():
                fn(cnt[0] % nset)
                cnt[0] += 1
            r = reps if bound == "hbm" else max(4, reps // 4)
            ms = time_launches(step, r, torch)
            gbs = bpe * E / (ms * 1e-3) / 1e9
            out[f"{op}_{name}"] = {"ms": round(ms, 5), "gdof_s": round(E * n3 / (ms * 1e-3) / 1e9, 3),
                                   "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "bound": bound}
            if bound == "alu":
                fl = fwd_flops.get(name)
                tf = fl * E / (ms * 1e-3) / 1e12 if fl else None
                out[f"{op}_{name}"]["alu"] = {
                    "flops_per_elem": fl, "achieved_TFLOPs": round(tf, 2) if tf else None,
                    "peak_TFLOPs": VALU_PEAK_TFLOPS[name],
                    "frac": round(tf / VALU_PEAK_TFLOPS[name], 4) if tf else None}
        del us, fs, dus, cs
        torch.cuda.empty_cache()
    return out


def section_tri(nk, W, torch, n=256, orders=(4, 6, 8), reps=40):
    """Collapsed-coordinate triangles: 2 n^2 curved triangles of the unit
    square, BwdTrans / IProductWRTBase / Helmholtz per order, FP64 and FP32.
    Algorithmic bytes per element (nm modes, np = Q(Q-1) points, s bytes):
    BwdTrans s(nm + np), IProductWRTBase s(2 np + nm), Helmholtz s(2 nm + 4 np)
    (4 factors per point)."""
    out = {"nelem": 2 * n * n}
    for P in orders:
        Q = P + 2
        e1, _, e2, _ = nk.tri_points(Q)
        J = torch.from_numpy(W.tri_lattice_jacobians(n, e1, e2, 0.05)).cuda()
        E = 2 * n * n
        nm, npt = (P + 1) * (P + 2) // 2, Q * (Q - 1)
        res = time_elementwise_ops(nk, W, torch, lambda k: [nk.Space.create_tri(P, Q, J) for _ in range(k)],
                                   E, nm, npt, 4, reps)
        del J
        out[f"P{P}"] = res
        log(f"tri P={P}: helmholtz f64 {res['helmholtz_f64']['ms'] * 1e3:.1f} us "
            f"({res['helmholtz_f64']['hbm_frac']:.1%} HBM)")
        torch.cuda.empty_cache()
    return out


def build_cg_problem(nk, W, torch, shape, P, amp):
    """Curved lattice, assembled system, weak RHS of the manufactured sine
    (built on the GPU with the library's own operators)."""
    Q = P + 2
    space, lat = make_space(nk, W, shape, P, amp, torch)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda(), lam0=1.0)
    U, dU = W.manufactured_ref_gradient(nk.basis_tables(P, Q)[0], lat)
    Ud = torch.from_numpy(U).cuda().reshape(-1)
    dUd = torch.from_numpy(dU).cuda().reshape(-1)
    del U, dU
    yl = nk.helmholtz_weak_rhs(space, Ud, dUd, lam0=1.0)
    b = sysm.assemble(yl)
    del Ud, dUd, yl
    return space, sysm, b, ng, lat


def section_cg(nk, W, torch, orders, shape=(24, 24, 24)):
    out = {}
    for P in orders:
        space, sysm, b, ng, lat = build_cg_problem(nk, W, torch, shape, P, W.WARP_AMPLITUDE)
        # warm the graphs
        sysm.solve(b, rtol=1e-2, maxit=64)
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_F32_REFINED)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = sysm.solve(b, rtol=1e-10, maxit=50000)
        t64 = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x32, i32 = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_F32_REFINED)
        t32 = (time.perf_counter() - t) * 1e3
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        nel = lat.nelem
        n3, q3 = (P + 1) ** 3, (P + 2) ** 3
        # algorithmic bytes of one PCG iteration: factors, the l2g map, and
        # 9 global vectors (operator in and out, x, r, p read and written,
        # the diagonal); the implementation streams 12 (its s = A p
        # recurrence and the reset of w), reported separately
        it_bytes64 = 8 * 7 * q3 * nel + 4 * n3 * nel + 8 * 9 * ng
        impl_bytes64 = 8 * 7 * q3 * nel + 4 * n3 * nel + 8 * 12 * ng
        ms_it64 = t64 / max(i64[0]["iters"], 1)
        gbs64 = it_bytes64 / (ms_it64 * 1e-3) / 1e9
        out[f"P{P}"] = {
            "nglobal": ng, "nelem": nel,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(ms_it64, 4),
                    "GB_s_per_iter": round(gbs64, 1), "hbm_frac_per_iter": round(gbs64 / HBM_PEAK_GBS, 4),
                    "impl_GB_s_per_iter": round(impl_bytes64 / (ms_it64 * 1e-3) / 1e9, 1)},
            "f32_refined": {"ms": round(t32, 2), "inner_iters": i32[0]["iters"],
                            "outer_iters": i32[0]["outer_iters"], "rel_resid": i32[0]["rel_resid"],
                            "rel_diff_vs_f64": diff},
            "speedup_refined_vs_f64": round(t64 / t32, 3),
        }
        log(f"cg P={P}: f64 {t64:.1f} ms ({i64[0]['iters']} it), refined {t32:.1f} ms "
            f"({i32[0]['outer_iters']} outer, {i32[0]['iters']} inner) resid {i32[0]['rel_resid']:.2e}")
        del space, sysm, b, x64, x32
        torch.cuda.empty_cache()
    return out


def section_condensed(nk, W, torch, orders=(4, 6), shape=(24, 24, 24)):
    """Static condensation (section 2.1) against the full FP64 PCG on the 24^3
    problem: setup of the boundary system and interior inverses, the
    condensed operator S x_B alone, boundary CG iterations, time per iteration
    and per solve."""
    out = {}
    for P in orders:
        space, sysm, b, ng, lat = build_cg_problem(nk, W, torch, shape, P, W.WARP_AMPLITUDE)
        sysm.solve(b, rtol=1e-2, maxit=64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        nb, _ = sysm.condense(with_map=False)
        setup_ms = (time.perf_counter() - t) * 1e3
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_CONDENSED)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xf, inf_f = sysm.solve(b, rtol=1e-10, maxit=50000)
        tf = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        xc, inf_c = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_CONDENSED)
        tc = (time.perf_counter() - t) * 1e3
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_CONDENSED_F32_REFINED)   # FP32 copy, graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        xr, inf_r = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_CONDENSED_F32_REFINED)
        tr = (time.perf_counter() - t) * 1e3
        nel, n3, q3, ni = lat.nelem, (P + 1) ** 3, (P + 2) ** 3, (P - 1) ** 3
        # algorithmic bytes of one boundary iteration: one read of the factors
        # and the map (the fused kernel's second pass reads them again; the
        # counters show that re-read reaching memory), the interior inverses
        # in their diagonal storage, 9 boundary vectors
        el_bytes = nel * (8 * 7 * q3 + 4 * n3 + 8 * (ni // 2 + 1) * ni)
        it_bytes = el_bytes + 8 * 9 * nb
        # S x_B alone: nk_condensed_apply calls (each pads x_B, launches the
        # fused kernel and synchronises), HIP events over 20 calls
        xb = torch.from_numpy(W.uniform(3, nb)).cuda()
        yb = torch.empty_like(xb)
        for _ in range(3):
            sysm.condensed_apply(xb, yb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            sysm.condensed_apply(xb, yb)
        e1.record()
        torch.cuda.synchronize()
        ap_ms = e0.elapsed_time(e1) / 20
        ap_gbs = (el_bytes + 16 * nb) / (ap_ms * 1e-3) / 1e9
        del xb, yb
        ms_it = tc / max(inf_c[0]["iters"], 1)
        gbs = it_bytes / (ms_it * 1e-3) / 1e9
        out[f"P{P}"] = {
            "nglobal": ng, "nboundary": nb, "nelem": nel, "setup_ms": round(setup_ms, 1),
            "apply_f64_per_call": {"ms": round(ap_ms, 4), "GB_s": round(ap_gbs, 1)},
            "full_f64": {"ms": round(tf, 2), "iters": inf_f[0]["iters"],
                         "ms_per_iter": round(tf / max(inf_f[0]["iters"], 1), 4)},
            "condensed": {"ms": round(tc, 2), "iters": inf_c[0]["iters"], "passes": inf_c[0]["outer_iters"],
                          "rel_resid": inf_c[0]["rel_resid"], "ms_per_iter": round(ms_it, 4),
                          "GB_s_per_iter": round(gbs, 1), "hbm_frac_per_iter": round(gbs / HBM_PEAK_GBS, 4)},
            "condensed_f32_refined": {"ms": round(tr, 2), "iters": inf_r[0]["iters"],
                                      "passes": inf_r[0]["outer_iters"], "rel_resid": inf_r[0]["rel_resid"],
                                      "rel_diff": float(torch.linalg.norm(xr - xf) / torch.linalg.norm(xf))},
            "speedup_condensed_vs_full": round(tf / tc, 3),
            "speedup_condensed_f32_refined_vs_full": round(tf / tr, 3),
            "rel_diff": float(torch.linalg.norm(xc - xf) / torch.linalg.norm(xf)),
        }
        log(f"condensed P={P}: setup {setup_ms:.1f} ms, full {tf:.1f} ms ({inf_f[0]['iters']} it), "
            f"condensed {tc:.1f} ms ({inf_c[0]['iters']} it, {inf_c[0]['outer_iters']} passes, "
            f"{ms_it * 1e3:.1f} us/it), condensed f32-refined {tr:.1f} ms ({inf_r[0]['iters']} it, "
            f"{inf_r[0]['outer_iters']} passes); S x_B {ap_ms * 1e3:.1f} us per call")
        del space, sysm, b, xf, xc, xr
        torch.cuda.empty_cache()
    return out


def section_tet(nk, W, torch, cases=((20, 4), (20, 6), (20, 8)), reps=30, shape="tet"):
    """Collapsed-coordinate tetrahedra (the unit cube split into n^3 cubes of
    six curved tetrahedra each), prisms (the triangle mesh of the unit
    square extruded into n layers, 2 n^3 curved prisms) or pyramids (six per
    cube, apex at its centre): BwdTrans /
    IProductWRTBase / Helmholtz per order, FP64 and FP32.  Algorithmic bytes
    per element (nm modes, np points, s bytes): BwdTrans s(nm + np),
    IProductWRTBase s(2 np + nm), Helmholtz s(2 nm + 7 np) (7 factors per
    point)."""
    out = {}
    for n, P in cases:
        Q = P + 2
        if shape == "tet":
            e1, _, e2, _, e3, _ = nk.tet_points(Q)
            J = torch.from_numpy(W.tet_lattice_jacobians(n, e1, e2, e3)).cuda()
            mk = nk.Space.create_tet
            E = 6 * n ** 3
            nm, npt = (P + 1) * (P + 2) * (P + 3) // 6, Q * (Q - 1) ** 2
        elif shape == "prism":
            e1, _, e2, _ = nk.tri_points(Q)
            J = torch.from_numpy(W.prism_lattice_jacobians(n, e1, e2, e1)).cuda()
            mk = nk.Space.create_prism
            E = 2 * n ** 3
            nm, npt = (P + 1) ** 2 * (P + 2) // 2, Q * Q * (Q - 1)
        else:   # pyramids: 6 per cube
            xg = nk.basis_tables(P, Q)[0]
            J = torch.from_numpy(W.pyr_lattice_jacobians(n, xg, xg, nk.tet_points(Q)[4])).cuda()
            mk = nk.Space.create_pyr
            E = 6 * n ** 3
            nm, npt = (P + 1) * (P + 2) * (2 * P + 3) // 6, Q * Q * (Q - 1)
        res = {"nelem": E}
        res.update(time_elementwise_ops(nk, W, torch, lambda k: [mk(P, Q, J) for _ in range(k)],
                                        E, nm, npt, 7, reps))
        del J
        out[f"P{P}"] = res
        log(f"{shape} P={P} ({E} elements): helmholtz f64 {res['helmholtz_f64']['ms'] * 1e3:.1f} us "
            f"({res['helmholtz_f64']['hbm_frac']:.1%} HBM), bwd {res['bwd_trans_f64']['hbm_frac']:.1%}, "
            f"iprod {res['iprod_wrt_base_f64']['hbm_frac']:.1%}")
        torch.cuda.empty_cache()
    return out


def section_tri_solve(nk, W, torch, n=128, orders=(4, 6)):
    """Assembled C0 solve on 2 n^2 curved triangles of the unit square with
    rotated local vertex orders (orientation signs on the shared edges),
    Dirichlet boundary, lambda = 1: -lap u + u = 1 (right-hand side the
    assembled IProductWRTBase of f = 1), FP64 vs FP32-refined to 1e-10."""
    out = {}
    E = 2 * n * n
    rot = W.tri_rotations(W.seed(5, 7), E)
    for P in orders:
        Q = P + 2
        e1, _, e2, _ = nk.tri_points(Q)
        J = torch.from_numpy(W.tri_lattice_jacobians(n, e1, e2, 0.05, rot)).cuda()
        space = nk.Space.create_tri(P, Q, J)
        del J
        l2g, sign, ng, dm = W.tri_lattice_l2g(n, P, rot)
        sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda(),
                                lam0=1.0, sign=torch.from_numpy(sign).cuda())
        ones = torch.ones(E * Q * (Q - 1), dtype=torch.float64, device="cuda")
        b = sysm.assemble(nk.iprod_wrt_base(space, ones))
        # warm the graphs (these short solves stop at maxit)
        sysm.solve(b, rtol=1e-2, maxit=64, raise_on_fail=False)
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_F32_REFINED, raise_on_fail=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = sysm.solve(b, rtol=1e-10, maxit=50000)
        t64 = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x32, i32 = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_F32_REFINED)
        t32 = (time.perf_counter() - t) * 1e3
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        out[f"P{P}"] = {
            "nglobal": int(ng), "nelem": E,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(t64 / max(i64[0]["iters"], 1), 4)},
            "f32_refined": {"ms": round(t32, 2), "inner_iters": i32[0]["iters"],
                            "outer_iters": i32[0]["outer_iters"], "rel_resid": i32[0]["rel_resid"],
                            "rel_diff_vs_f64": diff},
            "speedup_refined_vs_f64": round(t64 / t32, 3),
        }
        log(f"tri solve P={P}: {ng} DOF, f64 {t64:.1f} ms ({i64[0]['iters']} it), refined {t32:.1f} ms")
        del space, sysm, b, x64, x32, ones
        torch.cuda.empty_cache()
    return out


def section_tet_solve(nk, W, torch, n=12, orders=(4, 6)):
    """Assembled C0 solve on 6 n^3 curved tetrahedra of the unit cube with
    sorted vertex orders (half of them left-handed), Dirichlet boundary,
    lambda = 1: -lap u + u = 1 (right-hand side the assembled
    IProductWRTBase of f = 1), FP64 vs FP32-refined to 1e-10."""
    out = {}
    E = 6 * n ** 3
    for P in orders:
        Q = P + 2
        e1, _, e2, _, e3, _ = nk.tet_points(Q)
        J = torch.from_numpy(W.tet_lattice_jacobians(n, e1, e2, e3, sorted_ids=True)).cuda()
        space = nk.Space.create_tet(P, Q, J)
        del J
        l2g, ng, dm = W.tet_lattice_l2g(n, P)
        sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda(), lam0=1.0)
        ones = torch.ones(E * Q * (Q - 1) ** 2, dtype=torch.float64, device="cuda")
        b = sysm.assemble(nk.iprod_wrt_base(space, ones))
        sysm.solve(b, rtol=1e-2, maxit=64, raise_on_fail=False)
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_F32_REFINED, raise_on_fail=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = sysm.solve(b, rtol=1e-10, maxit=50000)
        t64 = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x32, i32 = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_F32_REFINED)
        t32 = (time.perf_counter() - t) * 1e3
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        out[f"P{P}"] = {
            "nglobal": int(ng), "nelem": E,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(t64 / max(i64[0]["iters"], 1), 4)},
            "f32_refined": {"ms": round(t32, 2), "inner_iters": i32[0]["iters"],
                            "outer_iters": i32[0]["outer_iters"], "rel_resid": i32[0]["rel_resid"],
                            "rel_diff_vs_f64": diff},
            "speedup_refined_vs_f64": round(t64 / t32, 3),
        }
        log(f"tet solve P={P}: {ng} DOF, f64 {t64:.1f} ms ({i64[0]['iters']} it), refined {t32:.1f} ms")
        del space, sysm, b, x64, x32, ones
        torch.cuda.empty_cache()
    return out


def section_prism_solve(nk, W, torch, n=16, orders=(4, 6)):
    """Assembled C0 solve on 2 n^3 curved prisms of the unit cube (the
    triangle mesh extruded in n layers, triangle vertex orders rotated per
    column, so edges carry orientation signs), Dirichlet boundary,
    lambda = 1: -lap u + u = 1, FP64 vs FP32-refined to 1e-10."""
    out = {}
    E = 2 * n ** 3
    rot = W.tri_rotations(W.seed(2, 7), 2 * n * n)
    for P in orders:
        Q = P + 2
        e1, _, e2, _ = nk.tri_points(Q)
        J = torch.from_numpy(W.prism_lattice_jacobians(n, e1, e2, e1, rot=rot)).cuda()
        space = nk.Space.create_prism(P, Q, J)
        del J
        l2g, sign, ng, dm = W.prism_lattice_l2g(n, P, rot)
        sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda(),
                                lam0=1.0, sign=torch.from_numpy(sign).cuda())
        ones = torch.ones(E * Q * Q * (Q - 1), dtype=torch.float64, device="cuda")
        b = sysm.assemble(nk.iprod_wrt_base(space, ones))
        sysm.solve(b, rtol=1e-2, maxit=64, raise_on_fail=False)
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_F32_REFINED, raise_on_fail=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = sysm.solve(b, rtol=1e-10, maxit=50000)
        t64 = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x32, i32 = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_F32_REFINED)
        t32 = (time.perf_counter() - t) * 1e3
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        out[f"P{P}"] = {
            "nglobal": int(ng), "nelem": E,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(t64 / max(i64[0]["iters"], 1), 4)},
            "f32_refined": {"ms": round(t32, 2), "inner_iters": i32[0]["iters"],
                            "outer_iters": i32[0]["outer_iters"], "rel_resid": i32[0]["rel_resid"],
                            "rel_diff_vs_f64": diff},
            "speedup_refined_vs_f64": round(t64 / t32, 3),
        }
        log(f"prism solve P={P}: {ng} DOF, f64 {t64:.1f} ms ({i64[0]['iters']} it), refined {t32:.1f} ms")
        del space, sysm, b, x64, x32, ones
        torch.cuda.empty_cache()
    return out


def section_pyr_solve(nk, W, torch, n=10, orders=(4, 6)):
    """Assembled C0 solve on 6 n^3 curved pyramids of the unit cube (each cube
    split into six pyramids around its centre), Dirichlet boundary,
    lambda = 1: -lap u + u = 1, FP64 vs FP32-refined to 1e-10."""
    out = {}
    E = 6 * n ** 3
    for P in orders:
        Q = P + 2
        xg = nk.basis_tables(P, Q)[0]
        J = torch.from_numpy(W.pyr_lattice_jacobians(n, xg, xg, nk.tet_points(Q)[4])).cuda()
        space = nk.Space.create_pyr(P, Q, J)
        del J
        l2g, ng, dm = W.pyr_lattice_l2g(n, P)
        sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda(), lam0=1.0)
        ones = torch.ones(E * Q * Q * (Q - 1), dtype=torch.float64, device="cuda")
        b = sysm.assemble(nk.iprod_wrt_base(space, ones))
        sysm.solve(b, rtol=1e-2, maxit=64, raise_on_fail=False)
        sysm.solve(b, rtol=1e-2, maxit=64, mode=nk.SOLVE_F32_REFINED, raise_on_fail=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = sysm.solve(b, rtol=1e-10, maxit=50000)
        t64 = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x32, i32 = sysm.solve(b, rtol=1e-10, maxit=50000, mode=nk.SOLVE_F32_REFINED)
        t32 = (time.perf_counter() - t) * 1e3
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        out[f"P{P}"] = {
            "nglobal": int(ng), "nelem": E,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(t64 / max(i64[0]["iters"], 1), 4)},
            "f32_refined": {"ms": round(t32, 2), "inner_iters": i32[0]["iters"],
                            "outer_iters": i32[0]["outer_iters"], "rel_resid": i32[0]["rel_resid"],
                            "rel_diff_vs_f64": diff},
            "speedup_refined_vs_f64": round(t64 / t32, 3),
        }
        log(f"pyramid solve P={P}: {ng} DOF, f64 {t64:.1f} ms ({i64[0]['iters']} it), refined {t32:.1f} ms")
        del space, sysm, b, x64, x32, ones
        torch.cuda.empty_cache()
    return out


def section_varp(nk, W, torch, reps=20):
    """20 000 hexes (20x20x50 curved lattice) with per-element order drawn from
    {2..10}: one persistent mixed-order launch vs one launch per order group."""
    cfg = W.CONFIGS[3]
    lat = W.lattice(cfg["varp_shape"])
    Pe = W.varp_orders(W.seed(3, 4), lat.nelem, *cfg["varp_P"])
    Ps = sorted(set(int(p) for p in Pe))
    jacs, xs, nbytes, ndof = [], [], 0, 0
    for P in Ps:
        sel = np.flatnonzero(Pe == P)
        sub = W.Lattice(lat.shape, lat.h, lat.origins[sel])
        jacs.append(torch.from_numpy(W.element_jacobians(nk.basis_tables(P, P + 2)[0], sub, cfg["warp"])).cuda())
        n3 = (P + 1) ** 3
        xs.append(torch.from_numpy(W.uniform(W.seed(3, 0) + P, sel.size * n3)).cuda())
        nbytes += helm_bytes_per_elem(P, P + 2) * sel.size
        ndof += sel.size * n3
    space = nk.Space.create_varp(3, Ps, [p + 2 for p in Ps], jacs)
    singles = [nk.Space.create(3, P, P + 2, j) for P, j in zip(Ps, jacs)]
    x = torch.cat(xs)
    out = {"nelem": int(lat.nelem), "local_dof": int(ndof), "orders": Ps}
    names = {0: "persistent", 1: "persistent_2bpc", 2: "concurrent", 3: "sequential"}
    for dt, name in ((nk.F64, "f64"), (nk.F32, "f32")):
        td = torch.float64 if dt == nk.F64 else torch.float32
        xd = x.to(td)
        y = torch.empty_like(xd)
        xg = [t.to(td) for t in xs]
        yg = [torch.empty_like(t) for t in xg]

        def per_group():
            for sp, xi, yi in zip(singles, xg, yg):
                nk.helmholtz(sp, xi, yi, lam0=1.0, dtype=dt)
        per_group()
        ms_grp = time_launches(per_group, reps, torch)
        ref = torch.cat(yg)
        res = {"per_group_separate_spaces_ms": round(ms_grp, 4)}
        for k, sname in names.items():
            space.set_strategy(dt, k)
            nk.helmholtz(space, xd, y, lam0=1.0, dtype=dt)
            ms = time_launches(lambda: nk.helmholtz(space, xd, y, lam0=1.0, dtype=dt), reps, torch)
            err = float(torch.linalg.norm(y - ref) / torch.linalg.norm(ref))
            s = 8 if dt == nk.F64 else 4
            gbs = nbytes * s / 8 / (ms * 1e-3) / 1e9
            res[sname] = {"ms": round(ms, 4), "speedup_vs_per_group": round(ms_grp / ms, 3),
                          "gdof_s": round(ndof / (ms * 1e-3) / 1e9, 2), "GB_s": round(gbs, 1),
                          "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "rel_diff_vs_per_group": err}
            log(f"varp {name} {sname}: {ms * 1e3:.1f} us vs per-group {ms_grp * 1e3:.1f} us")
        # the autotuner's choice
        nk.autotune(space, 0b100)
        res["autotuned"] = names[space.get_strategy(dt)]
        out[name] = res
    return out


def section_varp_solve(nk, W, torch, shape=(12, 12, 12), orders=(2, 8)):
    """A conforming variable-order solve: curved lattice with per-element
    order drawn from {orders[0]..orders[1]}, C0 map by the minimum rule,
    manufactured-sine weak right-hand side, FP64 CG and the FP32-refined
    solve to 1e-10; with every order at most 6 also both condensed solves
    (setup timed on its own)."""
    cfg = W.CONFIGS[3]
    lat = W.lattice(shape)
    Pe = W.varp_orders(W.seed(3, 4) + 1, lat.nelem, *orders)
    perm, l2g, ng, dm = W.varp_lattice_l2g(shape, Pe)
    ords = Pe[perm]
    Ps = sorted(set(int(p) for p in ords))
    jacs, Us, dUs = [], [], []
    for P in Ps:
        sub = W.Lattice(lat.shape, lat.h, lat.origins[perm[ords == P]])
        xq = nk.basis_tables(P, P + 2)[0]
        jacs.append(torch.from_numpy(W.element_jacobians(xq, sub, cfg["warp"])).cuda())
        U, dU = W.manufactured_ref_gradient(xq, sub)
        Us.append(U.ravel())
        dUs.append(dU.ravel())
    space = nk.Space.create_varp(3, Ps, [p + 2 for p in Ps], jacs)
    sysm = nk.System.create(space, ng, torch.from_numpy(np.concatenate(l2g)).cuda(),
                            torch.from_numpy(dm).cuda(), lam0=1.0)
    yl = nk.helmholtz_weak_rhs(space, torch.from_numpy(np.concatenate(Us)).cuda(),
                               torch.from_numpy(np.concatenate(dUs)).cuda(), lam0=1.0)
    b = sysm.assemble(yl)
    out = {"shape": list(shape), "orders": Ps, "nelem": int(lat.nelem), "nglobal": int(ng),
           "local_dof": int(sum((P + 1) ** 3 for P in ords))}
    modes = [(nk.SOLVE_F64, "f64"), (nk.SOLVE_F32_REFINED, "f32_refined")]
    if max(Ps) <= 6:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sysm.condense(with_map=False)
        out["condense_setup_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        modes += [(nk.SOLVE_CONDENSED, "condensed"), (nk.SOLVE_CONDENSED_F32_REFINED, "condensed_f32_refined")]
    for mode, name in modes:
        sysm.solve(b, rtol=1e-10, mode=mode)         # graphs and tiles warmed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = sysm.solve(b, rtol=1e-10, mode=mode)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms": round(ms, 2), "iters": info[0]["iters"],
                     "outer_iters": info[0]["outer_iters"], "rel_resid": info[0]["rel_resid"]}
        log(f"varp solve {name}: {ms:.1f} ms, {info[0]['iters']} it")
    return out


def section_filter(nk, W, torch, shape=(24, 24, 24), P=6):
    """The modified forward transform of Eq. (3), u** - alpha^2 lap u** = u*
    with du**/dn = 0, on the 24^3 curved lattice at P=6; filter width two
    element sizes, alpha = 2h / (2 pi).  Right-hand side: assembled
    IProductWRTBase of a seeded point field; FP64 CG and FP32-refined."""
    Q = P + 2
    lat = W.lattice(shape)
    alpha = 2.0 * lat.h[0] / (2.0 * math.pi)
    nq = Q ** 3
    kap = torch.full((lat.nelem * nq,), alpha ** 2, dtype=torch.float64, device="cuda")
    space, _ = make_space(nk, W, shape, P, W.WARP_AMPLITUDE, torch, kappa=kap)
    l2g, ng, _ = W.lattice_l2g(shape, P)
    sysm = nk.System.create(space, ng, torch.from_numpy(l2g).cuda(),
                            torch.zeros(ng, dtype=torch.uint8, device="cuda"), lam0=1.0)
    ustar = torch.from_numpy(W.uniform(W.seed(2, 1), lat.nelem * nq)).cuda()
    out = {"alpha": alpha, "nglobal": int(ng)}
    for mode, name in ((nk.SOLVE_F64, "f64"), (nk.SOLVE_F32_REFINED, "f32_refined")):
        nk.filtered_fwd_trans(space, sysm, ustar, rtol=1e-10, mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = nk.filtered_fwd_trans(space, sysm, ustar, rtol=1e-10, mode=mode)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms": round(ms, 2), "iters": info[0]["iters"], "rel_resid": info[0]["rel_resid"]}
        log(f"filter {name}: {ms:.1f} ms, {info[0]['iters']} it")
    return out


def section_many_solves(nk, W, torch):
    """256 independent P=5 Helmholtz solves on curved boxes of 64..4096 hexes
    (log-uniform sizes): one batched solve (one operator launch per CG
    iteration for all systems, captured in graphs) vs the systems solved one
    by one, FP64 and FP32-refined."""
    cfg = W.CONFIGS[3]
    P, Q = cfg["solve_P"], cfg["solve_P"] + 2
    boxes = W.solve_boxes(W.seed(3, 5), cfg["nsolves"], *cfg["solve_sizes"])
    xq = nk.basis_tables(P, Q)[0]
    n3, q3 = (P + 1) ** 3, Q ** 3
    nel = [a * b * c for a, b, c in boxes]
    E = int(sum(nel))
    J = torch.empty((E, 3, 3, q3), dtype=torch.float64, device="cuda")
    U = torch.empty((E, q3), dtype=torch.float64, device="cuda")
    dU = torch.empty((E, 3, q3), dtype=torch.float64, device="cuda")
    l2gs, dms, eoff, doff, ngs = [], [], [0], [0], []
    for bx in boxes:
        lat = W.lattice(bx)
        e0, e1 = eoff[-1], eoff[-1] + lat.nelem
        J[e0:e1] = torch.from_numpy(W.element_jacobians(xq, lat, cfg["warp"]))
        u_, du_ = W.manufactured_ref_gradient(xq, lat)
        U[e0:e1] = torch.from_numpy(u_)
        dU[e0:e1] = torch.from_numpy(du_)
        l2g, ng, dm = W.lattice_l2g(bx, P)
        l2gs.append(l2g)
        dms.append(dm)
        ngs.append(ng)
        eoff.append(e1)
        doff.append(doff[-1] + ng)
    space = nk.Space.create(3, P, Q, J)
    l2g_u = torch.from_numpy(np.concatenate([l + o for l, o in zip(l2gs, doff[:-1])]).astype(np.int32)).cuda()
    dm_u = torch.from_numpy(np.concatenate(dms)).cuda()
    sysb = nk.System.create_batched(space, eoff, doff, l2g_u, dm_u, lam0=1.0)
    yl = nk.helmholtz_weak_rhs(space, U.reshape(-1), dU.reshape(-1), lam0=1.0)
    b = sysb.assemble(yl)
    del U, dU, yl
    out = {"nsys": len(boxes), "nelem_total": E, "nglobal_total": int(doff[-1]),
           "min_elems": int(min(nel)), "max_elems": int(max(nel))}
    for mode, name in ((nk.SOLVE_F64, "f64"), (nk.SOLVE_F32_REFINED, "f32_refined")):
        sysb.solve(b, rtol=1e-2, maxit=50000, mode=mode)      # capture graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        xb, info = sysb.solve(b, rtol=1e-10, maxit=50000, mode=mode)
        tb = (time.perf_counter() - t) * 1e3
        its = [i["iters"] for i in info]
        out[name] = {"batched_ms": round(tb, 2), "iters_min": min(its), "iters_max": max(its),
                     "max_rel_resid": max(i["rel_resid"] for i in info)}
        log(f"256 solves {name}: batched {tb:.1f} ms (iters {min(its)}..{max(its)})")
    # one by one (same kernels, one system per solve)
    singles = []
    for k in range(len(boxes)):
        sp = nk.Space.create(3, P, Q, J[eoff[k]:eoff[k + 1]])
        sy = nk.System.create(sp, ngs[k], torch.from_numpy(l2gs[k]).cuda(), torch.from_numpy(dms[k]).cuda(),
                              lam0=1.0)
        singles.append((sp, sy, b[doff[k]:doff[k + 1]].contiguous()))
    for mode, name in ((nk.SOLVE_F64, "f64"), (nk.SOLVE_F32_REFINED, "f32_refined")):
        for sp, sy, bk in singles:
            sy.solve(bk, rtol=1e-2, maxit=50000, mode=mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xs = [sy.solve(bk, rtol=1e-10, maxit=50000, mode=mode)[0] for sp, sy, bk in singles]
        ti = (time.perf_counter() - t) * 1e3
        xb, _ = sysb.solve(b, rtol=1e-10, maxit=50000, mode=mode)
        diff = float(torch.linalg.norm(xb - torch.cat(xs)) / torch.linalg.norm(xb))
        out[name].update({"one_by_one_ms": round(ti, 2),
                          "speedup_batched": round(ti / out[name]["batched_ms"], 2),
                          "rel_diff_batched_vs_one_by_one": diff})
        log(f"256 solves {name}: one by one {ti:.1f} ms")
    # the same 256 separately created systems in one nk_cg_solve_batched call
    # (the library batches them into a cached union on the first call)
    sys_list = [sy for sp, sy, bk in singles]
    b_list = [bk for sp, sy, bk in singles]
    for mode, name in ((nk.SOLVE_F64, "f64"), (nk.SOLVE_F32_REFINED, "f32_refined")):
        torch.cuda.synchronize()
        t = time.perf_counter()
        nk.solve_batched(sys_list, b_list, rtol=1e-2, maxit=50000, mode=mode)
        tfirst = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        xs, info = nk.solve_batched(sys_list, b_list, rtol=1e-10, maxit=50000, mode=mode)
        tsep = (time.perf_counter() - t) * 1e3
        xb, _ = sysb.solve(b, rtol=1e-10, maxit=50000, mode=mode)
        diff = float(torch.linalg.norm(torch.cat(xs) - xb) / torch.linalg.norm(xb))
        out[name].update({"separate_systems_batched_ms": round(tsep, 2),
                          "separate_systems_first_call_ms": round(tfirst, 2),
                          "separate_systems_max_rel_resid": max(i["rel_resid"] for i in info),
                          "rel_diff_separate_vs_batched": diff,
                          "speedup_separate_batched_vs_one_by_one": round(out[name]["one_by_one_ms"] / tsep, 2)})
        log(f"256 solves {name}: separate systems batched {tsep:.1f} ms (first call {tfirst:.1f} ms)")
    out["speedup_f32_refined_vs_f64_batched"] = round(out["f64"]["batched_ms"] / out["f32_refined"]["batched_ms"], 3)
    return out


def section_grad(nk, W, torch):
    """Loss 0.5 ||u(kappa, lambda) - u_t||^2 on 16^3 curved hexes at P=6 with
    kappa per quadrature point and lambda per element drawn from [0.5, 2]:
    forward solve and adjoint backward through torch.autograd, plus a
    central-difference check along a seeded direction."""
    from paper_1906_03489_amd.autograd import HelmholtzProblem, helmholtz_solve
    cfg = W.CONFIGS[4]
    P, Q, shape = cfg["P"], cfg["Q"], cfg["shape"]
    lat = W.lattice(shape)
    E, q3 = lat.nelem, Q ** 3
    xq = nk.basis_tables(P, Q)[0]
    J = torch.from_numpy(W.element_jacobians(xq, lat, cfg["warp"])).cuda()
    l2g, ng, dm = W.lattice_l2g(shape, P)
    l2g, dm = torch.from_numpy(l2g).cuda(), torch.from_numpy(dm).cuda()
    sp1 = nk.Space.create(3, P, Q, J)
    sy1 = nk.System.create(sp1, ng, l2g, dm, lam0=1.0)
    U, dU = W.manufactured_ref_gradient(xq, lat)
    b = sy1.assemble(nk.helmholtz_weak_rhs(sp1, torch.from_numpy(U).cuda().reshape(-1),
                                           torch.from_numpy(dU).cuda().reshape(-1), lam0=1.0))
    ut, _ = sy1.solve(b, rtol=1e-12)
    pb = HelmholtzProblem(3, P, Q, J, l2g, ng, dm, b, rtol=1e-12)
    lo, hi = cfg["coef_range"]
    kap = torch.from_numpy(W.uniform(W.seed(4, 3), (E, q3), lo, hi)).cuda().requires_grad_(True)
    lam = torch.from_numpy(W.uniform(W.seed(4, 2), E, lo, hi)).cuda().requires_grad_(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    u = helmholtz_solve(kap, lam, pb)
    loss = 0.5 * torch.sum((u - ut) ** 2)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t_bwd = (time.perf_counter() - t) * 1e3
    rng = np.random.default_rng(W.seed(4, 6))
    vk = torch.from_numpy(rng.standard_normal((E, q3))).cuda()
    vl = torch.from_numpy(rng.standard_normal(E)).cuda()
    eps = 1e-4
    with torch.no_grad():
        lp = 0.5 * torch.sum((helmholtz_solve(kap + eps * vk, lam + eps * vl, pb) - ut) ** 2)
        lm = 0.5 * torch.sum((helmholtz_solve(kap - eps * vk, lam - eps * vl, pb) - ut) ** 2)
    fd = float((lp - lm) / (2 * eps))
    an = float(torch.sum(kap.grad * vk) + torch.sum(lam.grad * vl))
    log(f"grad: forward {t_fwd:.1f} ms, backward {t_bwd:.1f} ms, fd {fd:.6e} vs adjoint {an:.6e}")
    return {"nelem": E, "n_kappa": E * q3, "n_lambda": E, "loss": float(loss),
            "forward_ms": round(t_fwd, 2), "backward_ms": round(t_bwd, 2),
            "fd_directional": fd, "adjoint_directional": an,
            "fd_rel_diff": abs(fd - an) / abs(an)}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(W, budget_s=5.0, apply_s=3.0):
    """The plain FP64 oracle on a bounded sample of the 32^3, P=6 workload:
    (1) dense elemental matrices built and applied (the headline value);
    (2) apply only: 256 prebuilt H_e applied as one batched matmul."""
    import oracle
    threads = _blas_threads()
    P, Q = 6, 8
    n3 = (P + 1) ** 3
    lat = W.lattice((32, 32, 32))
    rng = np.random.default_rng(W.seed(1, 6))
    idx = np.sort(rng.choice(lat.nelem, 4096, replace=False))
    x = W.uniform(W.seed(1, 0), (lat.nelem, n3))
    done = 0
    t0 = time.perf_counter()
    chunk = 8
    while time.perf_counter() - t0 < budget_s and done < idx.size:
        sel = idx[done:done + chunk]
        sub = W.Lattice(lat.shape, lat.h, lat.origins[sel])
        J = W.element_jacobians(oracle.gll(Q)[0], sub, W.WARP_AMPLITUDE)
        ops = oracle.ElementOps(3, P, Q, J, lam=1.0)
        ops.helmholtz(x[sel])
        done += sel.size
    dt = time.perf_counter() - t0
    # apply only
    sel = idx[:256]
    sub = W.Lattice(lat.shape, lat.h, lat.origins[sel])
    ops = oracle.ElementOps(3, P, Q, W.element_jacobians(oracle.gll(Q)[0], sub, W.WARP_AMPLITUDE), lam=1.0)
    H = np.stack(oracle.helmholtz_matrices(ops))
    xs = x[sel][:, :, None]
    reps = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < apply_s:
        np.matmul(H, xs)
        reps += 1
    da = time.perf_counter() - t1
    return {"value": round(done * n3 / dt / 1e9, 6), "unit": "GDOF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done} of 32768 elements of the 32^3 P=6 workload, dense H_e build + apply, "
                      f"{dt:.1f} s",
            "apply_only": {"value": round(reps * 256 * n3 / da / 1e9, 6), "unit": "GDOF/s",
                           "cores": threads,
                           "sample": f"256 prebuilt H_e (343 x 343) applied as one batched matmul, "
                                     f"{reps} times in {da:.1f} s"}}


def cpu_oracle_pcg(W, P=4, shape=(24, 24, 24), rtol=1e-10, maxit=None, iters_ref=None):
    """The oracle's Jacobi PCG on the 24^3 curved-hex problem of the GPU's
    CG section (same right-hand side construction: weak form of the
    manufactured sine), as the oracle stands: prebuilt dense H_e applied by
    its masked operator.  Time to solution on the host's cores (about a
    minute of CPU work).  With maxit, a bounded sample: the setup and maxit
    iterations are timed, and the time to solution is the setup plus
    iters_ref (the iteration count of the same textbook PCG to rtol, e.g. the
    GPU's FP64 count for this problem) times the measured iteration."""
    import oracle
    from oracle.assembly import MaskedOperator, jacobi_diagonal
    threads = _blas_threads()
    Q = P + 2
    lat = W.lattice(shape)
    t0 = time.perf_counter()
    Jo = W.element_jacobians(oracle.gll(Q)[0], lat, W.WARP_AMPLITUDE)
    ops = oracle.ElementOps(3, P, Q, Jo, lam=1.0)
    # the oracle's dense H_e element by element (what helmholtz_matrices
    # does), with a progress line every 1000 elements
    mats = []
    for e in range(ops.nelem):
        mats.append(ops.helmholtz_matrix(e))
        if (e + 1) % 1000 == 0:
            log(f"oracle pcg setup: {e + 1} of {ops.nelem} H_e, {time.perf_counter() - t0:.0f} s")
    l2g, ng, dm = W.lattice_l2g(shape, P)
    U, dU = W.manufactured_ref_gradient(ops.x, lat)
    b = oracle.assemble_vector(ops.weak_rhs(U, dU), l2g, ng)
    b[dm.astype(bool)] = 0.0
    diag = jacobi_diagonal(mats, l2g, ng, dm)
    A = MaskedOperator(mats, l2g, ng, dm)
    t_setup = time.perf_counter() - t0
    log(f"oracle pcg setup {t_setup:.1f} s ({lat.nelem} dense H_e)")
    calls = [0]

    def apply(v):
        # the oracle's operator, with a progress line every 100 applications
        calls[0] += 1
        if calls[0] % 100 == 0:
            log(f"oracle pcg: {calls[0]} operator applications, {time.perf_counter() - t1:.0f} s")
        return A(v)
    t1 = time.perf_counter()
    x, its, res = oracle.pcg(apply, b, diag, rtol=rtol, maxit=maxit if maxit else 100000)
    t_solve = time.perf_counter() - t1
    out = {"P": P, "nglobal": int(ng), "nelem": int(lat.nelem), "iters": int(its), "rel_resid": float(res),
           "setup_s": round(t_setup, 2), "solve_s": round(t_solve, 2),
           "s_per_iter": round(t_solve / max(its, 1), 4), "cores": threads}
    if maxit:
        out["sample"] = f"setup and the first {its} of the PCG iterations timed"
        if iters_ref:
            out["time_to_solution_s"] = round(t_setup + iters_ref * t_solve / max(its, 1), 1)
            out["iters_to_solution"] = int(iters_ref)
            out["sample"] += (f"; time to solution = setup + {iters_ref} iterations (the GPU FP64 "
                              f"PCG's count for the same problem and rtol)")
    return out


# --------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sections", default="ops,deriv,tri,tet,cg,batch,grad,cpu",
                    help="comma list of ops,deriv,tri,tet,cg,cond,batch,grad,cpu,cpu_pcg (or 'none'; "
                         "cond: the static-condensation comparison alone, also part of cg); "
                         "cpu_pcg (the oracle's 24^3 P=4 PCG, minutes of CPU) and cpu_pcg6 (a sample of "
                         "its P=6 PCG, 13 GB of host memory) are not in the default")
    ap.add_argument("--cg-orders", default="4,6,8")
    ap.add_argument("--calib", action="store_true",
                    help="after the timed region, one 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1906_03489_amd import nk
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    secs = set(s for s in args.sections.split(",") if s and s != "none")

    cfg = W.CONFIGS[1]
    P, Q = cfg["P"], cfg["Q"]
    log("building 32^3 P=6 curved space ...")
    space, lat = make_space(nk, W, cfg["shape"], P, cfg["warp"], torch)
    E = lat.nelem
    ndof = E * (P + 1) ** 3
    x = torch.from_numpy(W.uniform(W.seed(1, 0), ndof)).cuda()
    y = torch.empty_like(x)
    nk.autotune(space, 0b111)
    log("tiles:", nk.tile_config(2, 3, P, nk.F64), nk.tile_config(2, 3, P, nk.F32))
    for _ in range(args.warmup):
        nk.helmholtz(space, x, y, lam0=1.0)
    torch.cuda.synchronize()
    # timed region: exactly `steps` Helmholtz applications
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        nk.helmholtz(space, x, y, lam0=1.0)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    gdof = ndof / (ms * 1e-3) / 1e9
    bpl = helm_bytes_per_elem(P, Q) * E
    achieved = bpl / (ms * 1e-3) / 1e9
    # the practical HBM ceiling (measured before the calibration copy, which
    # the counter summaries take as the last 1 GiB copy of the run)
    copy_gbs = device_copy_gbs(torch)
    if args.calib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the counters of the Helmholtz kernel in the same run
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"helmholtz f64: {ms * 1e3:.1f} us/launch, {gdof:.2f} GDOF/s, {achieved:.0f} GB/s "
        f"({achieved / HBM_PEAK_GBS:.1%} of HBM peak, {achieved / copy_gbs:.1%} of a {copy_gbs:.0f} GB/s device copy); "
        f"host wall {wall * 1e3 / args.steps:.1f} us/step")
    result = {
        "metric": METRIC, "value": round(gdof, 3), "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32^3 curved hexahedra (cyclic sine warp, amplitude 0.05) on the unit cube, "
                               "P=6 modified C0 basis, Q=8 GLL, FP64 local Helmholtz lambda=1, "
                               f"{ndof} local DOF per step",
                   "tile": nk.tile_config(2, 3, P, nk.F64)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "k_op3<double,7,8,EPB,OP_HELM>",
                     "bytes_per_launch": bpl,
                     "device_copy_GBs": round(copy_gbs, 1),
                     "frac_of_device_copy": round(achieved / copy_gbs, 4)},
    }
    sections = {}
    if "ops" in secs:
        log("section ops ...")
        sections["ops_32c_P6"] = section_ops(nk, W, torch, space, lat, P, Q, 40)
    if "deriv" in secs:
        log("section deriv ...")
        sections["deriv_32c_P6"] = section_deriv(nk, W, torch, space, lat, P, Q, 40)
    if "tri" in secs:
        log("section tri ...")
        sections["tri_131072"] = section_tri(nk, W, torch)
        log("section tri solve ...")
        sections["tri_solve_32768"] = section_tri_solve(nk, W, torch)
    if "tet" in secs:
        log("section tet ...")
        sections["tet"] = section_tet(nk, W, torch)
        log("section prism ...")
        sections["prism"] = section_tet(nk, W, torch, cases=((24, 4), (24, 6), (24, 8)), shape="prism")
        log("section pyramid ...")
        sections["pyramid"] = section_tet(nk, W, torch, cases=((20, 4), (20, 6), (20, 8)), shape="pyramid")
        log("section tet solve ...")
        sections["tet_solve_10368"] = section_tet_solve(nk, W, torch)
        log("section prism solve ...")
        sections["prism_solve_8192"] = section_prism_solve(nk, W, torch)
        log("section pyramid solve ...")
        sections["pyramid_solve_6000"] = section_pyr_solve(nk, W, torch)
    del space, x, y
    torch.cuda.empty_cache()
    if "cg" in secs:
        log("section cg ...")
        sections["cg_24c"] = section_cg(nk, W, torch, [int(p) for p in args.cg_orders.split(",") if p])
        torch.cuda.empty_cache()
        log("section cg (filter equation) ...")
        sections["filter_24c_P6"] = section_filter(nk, W, torch)
        torch.cuda.empty_cache()
    if "cg" in secs or "cond" in secs:
        log("section cg (static condensation) ...")
        sections["condensed_24c"] = section_condensed(nk, W, torch)
        torch.cuda.empty_cache()
    if "batch" in secs:
        log("section batch (mixed order) ...")
        sections["batch_varp_20000"] = section_varp(nk, W, torch)
        torch.cuda.empty_cache()
        log("section batch (mixed-order solve) ...")
        sections["varp_solve_12c"] = section_varp_solve(nk, W, torch)
        torch.cuda.empty_cache()
        log("section batch (mixed-order solve, orders 2..6, condensed) ...")
        sections["varp_solve_16c_P2_6"] = section_varp_solve(nk, W, torch, shape=(16, 16, 16), orders=(2, 6))
        torch.cuda.empty_cache()
        log("section batch (256 solves) ...")
        sections["batch_256_solves"] = section_many_solves(nk, W, torch)
        torch.cuda.empty_cache()
    if "grad" in secs:
        log("section grad ...")
        sections["grad_16c_P6"] = section_grad(nk, W, torch)
    result["sections"] = sections
    if "cpu" in secs:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(W)
        if "cpu_pcg" not in secs:
            # bounded sample of the oracle's PCG on the 24^3 P=4 problem
            ref = sections.get("cg_24c", {}).get("P4", {}).get("f64", {}).get("iters")
            log("cpu oracle PCG, 24^3 P=4 (setup and 30 iterations) ...")
            result["cpu_baseline"]["pcg_24c_P4"] = cpu_oracle_pcg(W, maxit=30, iters_ref=ref)
    if "cpu_pcg" in secs:
        log("cpu oracle PCG, 24^3 P=4 (minutes) ...")
        result.setdefault("cpu_baseline", {})["pcg_24c_P4"] = cpu_oracle_pcg(W)
    if "cpu_pcg6" in secs:
        # bounded sample at P=6: 13 824 dense 343 x 343 H_e (13 GB), setup and
        # 10 iterations, the time to solution extrapolated with the GPU's count
        ref = sections.get("cg_24c", {}).get("P6", {}).get("f64", {}).get("iters")
        log("cpu oracle PCG, 24^3 P=6 (setup and 10 iterations, minutes) ...")
        result.setdefault("cpu_baseline", {})["pcg_24c_P6"] = cpu_oracle_pcg(W, P=6, maxit=10, iters_ref=ref)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
