"""Build libipdg.so (the C-ABI library) for gfx950 with hipcc, in-tree.

Every source is compiled on each call (the per-degree element kernels once
per polynomial degree, in parallel) and linked into
paper_1801_00246_amd/libipdg.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libipdg.so")
ARCH = os.environ.get("IPDG_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]
HOST_SOURCES = ["refelem.cpp", "mesh_host.cpp", "ops_table.cpp", "mesh.cpp", "dispatch.cpp",
                "amg_host.cpp", "solver.cpp", "ins.cpp", "subcycle_host.cpp", "gradiv_host.cpp", "abi.cpp"]
DEVICE_SOURCES = ["blas.hip", "noalloc.hip", "probe.hip", "amg.hip", "gradiv.hip", "subcycle.hip"]
DEGREES = range(1, 9)


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(job):
    src, obj, extra = job
    cmd = [_hipcc(), "-x", "hip", *FLAGS, *extra, "-c", src, "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, time.time() - t


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    work = []
    for n in DEGREES:
        work.append((os.path.join(CSRC, "elem_inst.hip"), os.path.join(BUILD, f"elem_n{n}.o"),
                     [f"-DIPDG_N={n}"]))
    for s in DEVICE_SOURCES + HOST_SOURCES:
        p = os.path.join(CSRC, s)
        if os.path.exists(p):
            work.append((p, os.path.join(BUILD, os.path.splitext(s)[0] + ".o"), []))
    jobs = jobs or min(16, os.cpu_count() or 4)
    # the heaviest units first
    work.sort(key=lambda w: -int(w[2][0].split("=")[1]) if w[2] else 0)
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt in ex.map(_compile, work):
            objs.append(obj)
            if verbose:
                print(f"  built {os.path.basename(obj)} in {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"libipdg.so built in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else None)
