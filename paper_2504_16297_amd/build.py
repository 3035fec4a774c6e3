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


SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def build_sanitized(jobs=8):
    """A host-sanitized copy of the library for CPU test runs: the host sources
    (planner, PTS, executor, ABI, pass compiler) built with g++ under
    AddressSanitizer and UndefinedBehaviorSanitizer, the device sources built as
    usual (no GPU sanitizer), into _build/sanitize/libptsbe.so.  Run the CPU
    suite on it with

        LD_PRELOAD="$(g++ -print-file-name=libasan.so) $(g++ -print-file-name=libubsan.so)" \
        ASAN_OPTIONS=detect_leaks=0 PTSBE_LIB=_build/sanitize/libptsbe.so \
        python -m pytest tests -m "not gpu"
    """
    os.makedirs(SAN_DIR, exist_ok=True)
    cmds, objs = [], []
    for s in HOST_SRCS:
        o = os.path.join(SAN_DIR, s + ".o")
        cmds.append(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
                     "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")] +
                    SAN_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEVICE_SRCS:
        o = os.path.join(SAN_DIR, s + ".o")
        cmds.append([HIPCC] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(_run, cmds))
    lib = os.path.join(SAN_DIR, "libptsbe.so")
    _run(["g++", "-shared", "-o", lib] + objs + SAN_FLAGS[:1] +
         ["-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--sanitize", action="store_true", help="build the host-sanitized copy for CPU test runs")
    a = ap.parse_args()
    print(build_sanitized(a.jobs) if a.sanitize else build(a.jobs, a.v))
