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


def make_space(nk, W, shape, P, amp, torch, kappa=None):
    Q = P + 2
    lat = W.lattice(shape)
    J = W.element_jacobians(nk.basis_tables(P, Q)[0], lat, amp)
    Jd = torch.from_numpy(J).cuda()
    del J
    sp = nk.Space.create(3, P, Q, Jd, kappa=kappa)
    del Jd
    return sp, lat


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
        del cs, fs, us, ys
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
        it_bytes64 = 8 * 7 * q3 * nel + 4 * n3 * nel + 8 * 12 * ng
        it_bytes32 = 4 * 7 * q3 * nel + 4 * n3 * nel + 4 * 12 * ng
        ms_it64 = t64 / max(i64[0]["iters"], 1)
        out[f"P{P}"] = {
            "nglobal": ng, "nelem": nel,
            "f64": {"ms": round(t64, 2), "iters": i64[0]["iters"], "rel_resid": i64[0]["rel_resid"],
                    "ms_per_iter": round(ms_it64, 4),
                    "GB_s_per_iter": round(it_bytes64 / (ms_it64 * 1e-3) / 1e9, 1)},
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


def cpu_baseline(W, budget_s=12.0):
    """The plain FP64 oracle (dense elemental matrices, build + apply) on a
    bounded sample of the 32^3, P=6 workload's elements."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    P, Q = 6, 8
    lat = W.lattice((32, 32, 32))
    rng = np.random.default_rng(W.seed(1, 6))
    idx = np.sort(rng.choice(lat.nelem, 4096, replace=False))
    x = W.uniform(W.seed(1, 0), (lat.nelem, (P + 1) ** 3))
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
    return {"value": round(done * (P + 1) ** 3 / dt / 1e9, 6), "unit": "GDOF/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{done} of 32768 elements of the 32^3 P=6 workload, dense H_e build + apply, "
                      f"{dt:.1f} s"}


# --------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sections", default="ops,cg,cpu",
                    help="comma list of ops,cg,batch,grad,cpu (or 'none')")
    ap.add_argument("--cg-orders", default="4,6,8")
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
    log(f"helmholtz f64: {ms * 1e3:.1f} us/launch, {gdof:.2f} GDOF/s, {achieved:.0f} GB/s "
        f"({achieved / HBM_PEAK_GBS:.1%} of HBM peak); host wall {wall * 1e3 / args.steps:.1f} us/step")
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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_op3<double,7,8,EPB,OP_HELM>",
                     "bytes_per_launch": bpl},
    }
    sections = {}
    if "ops" in secs:
        log("section ops ...")
        sections["ops_32c_P6"] = section_ops(nk, W, torch, space, lat, P, Q, 40)
    del space, x, y
    torch.cuda.empty_cache()
    if "cg" in secs:
        log("section cg ...")
        sections["cg_24c"] = section_cg(nk, W, torch, [int(p) for p in args.cg_orders.split(",") if p])
    if "batch" in secs:
        from bench_sections import section_batch
        log("section batch ...")
        sections["batch"] = section_batch(nk, W, torch)
    if "grad" in secs:
        from bench_sections import section_grad
        log("section grad ...")
        sections["grad_16c_P6"] = section_grad(nk, W, torch)
    result["sections"] = sections
    if "cpu" in secs:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
