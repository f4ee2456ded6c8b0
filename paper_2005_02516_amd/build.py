"""Build the HIP library libesdg_swe.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2005_02516_amd.build   (or call build_library()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIBDIR = os.path.join(HERE, "_lib")
LIBNAME = "libesdg_swe.so"
# (source, extra defines): kernels.hip is compiled once per (precision, mass inverse) for its
# stage kernels and once for the rest, so that the objects build in parallel
SOURCES = [("host_setup.cpp", []), ("runtime.cpp", []), ("volume_bench.hip", []),
           ("kernels.hip", ["-DESDG_UNIT_HOST"]),
           ("kernels.hip", ["-DESDG_UNIT_REAL=float", "-DESDG_UNIT_WADG=0"]),
           ("kernels.hip", ["-DESDG_UNIT_REAL=float", "-DESDG_UNIT_WADG=1"]),
           ("kernels.hip", ["-DESDG_UNIT_REAL=double", "-DESDG_UNIT_WADG=0"]),
           ("kernels.hip", ["-DESDG_UNIT_REAL=double", "-DESDG_UNIT_WADG=1"])]

HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiplies and adds fuse into FMAs within one expression only, so that every build of
    # a kernel (per-stage, multi-stage, single-kind) rounds the same source the same way
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


def library_path() -> str:
    return os.path.join(LIBDIR, LIBNAME)


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(LIBDIR, exist_ok=True)
    cmds, objs = [], []
    for i, (src, defs) in enumerate(SOURCES):
        obj = os.path.join(LIBDIR, f"{os.path.splitext(src)[0]}_{i}.o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([hipcc, *HIPFLAGS, *defs, "-I" + INCLUDE, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(run, cmds))
    for cmd, r in zip(cmds, results):
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        if err.strip():
            print(err, file=sys.stderr, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
    out = library_path()
    tmp = out + ".tmp"
    cmd = [hipcc, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
