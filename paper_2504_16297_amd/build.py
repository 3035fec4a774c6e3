"""Build libptsbe.so (host planner + gfx950 kernels) in-tree with hipcc.

Usage: python -m paper_2504_16297_amd.build  [--jobs N]

Host sources are compiled as plain C++ (no floating-point contraction, so the
pre-trajectory sampler's arithmetic is bit-reproducible); the kernel source is
compiled for gfx950 with packed-FP32 instructions disabled.
"""

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libptsbe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HOST_SRCS = ["plan.cpp", "pts.cpp", "run.cpp", "abi.cpp", "adjoint.cpp", "jit.cpp"]
DEVICE_SRCS = ["kernels.hip", "unique.hip", "noalloc.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]
HOST_FLAGS = ["-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + "\n")
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return r.stdout


def build(jobs=8, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for s in HOST_SRCS:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([HIPCC] + COMMON + HOST_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEVICE_SRCS:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([HIPCC] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                sys.stdout.write(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs +
         ["-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.v))
