"""Build the HIP library libnk.so for MI355X (gfx950) in-tree.

Each source compiles to its own object in parallel; the 3-D operator
instantiations are split by polynomial order (ops3d_inst.hip compiled once per
order set).  Usage:  python -m paper_1906_03489_amd.build  [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libnk.so")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wno-unused-command-line-argument"]
# packed FP32 VALU ops are disabled on the device pass
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [("api.cpp", []), ("basis.cpp", []), ("geom.hip", []), ("cg.hip", []),
           ("varp.hip", []), ("ops2d.hip", []), ("mfma.hip", []), ("deriv.hip", []), ("tri.hip", []),
           ("collapsed3d.hip", []), ("condense.hip", [])] + \
          [("ops3d_inst.hip", [f"-DNK_PSET={k}"]) for k in range(7)]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _obj(src: str, defs) -> str:
    tag = "".join(d.replace("-D", "_").replace("=", "") for d in defs)
    return os.path.join(BUILD, os.path.splitext(src)[0] + tag + ".o")


def _compile(src, defs):
    obj = _obj(src, defs)
    # hipcc compiles .cpp sources as HIP too (api.cpp holds a device array)
    flags = COMMON + DEVICE + list(defs)
    cmd = [hipcc()] + flags + ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj, time.time() - t


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, d) for s, d in SOURCES]
        for f in futs:
            obj, dt = f.result()
            objs.append(obj)
            if verbose:
                print(f"  {os.path.basename(obj)}  {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    args = ap.parse_args()
    t = time.time()
    print(build(args.j, verbose=True), f"({time.time() - t:.1f}s)")
    sys.exit(0)
