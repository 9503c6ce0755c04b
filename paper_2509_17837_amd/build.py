"""Build the HIP library libxzzx_sa.so in-tree for gfx950.

Usage: python -m paper_2509_17837_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxzzx_sa.so")
SOURCES = ["xzzx_planar.hip", "xzzx_ladder_planar.hip", "xzzx_ladder_rows_c.hip", "xzzx_ladder_rows_b.hip", "xzzx_ladder_rows.hip", "xzzx_ladder.hip", "xzzx_serve_29.hip", "xzzx_serve_31.hip", "xzzx_serve_25.hip", "xzzx_serve_21.hip", "xzzx_serve_15.hip", "xzzx_serve_9.hip",
           "xzzx_static_h.hip", "xzzx_static_g.hip", "xzzx_static_f.hip", "xzzx_static_e.hip", "xzzx_static_d.hip",
           "xzzx_static_c.hip", "xzzx_static_b.hip", "xzzx_static_a.hip",
           "xzzx_kernels.hip", "xzzx_probe.hip", "xzzx_host.cpp", "xzzx_server.cpp", "xzzx_tune.cpp"]   # longest first

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # packed FP32 instructions are never wanted in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # thresholds must be bit-identical to the plain double expression
    "-ffp-contract=off", "-fno-fast-math",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: cannot build the gfx950 library")
    return exe


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object in parallel (the specialised kernels
    are large), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor

    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    compile_flags = [f for f in FLAGS if f != "-shared"]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc(), *compile_flags, *inc, "-c", "-x", "hip", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    n = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 8)
    with ThreadPoolExecutor(n) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
