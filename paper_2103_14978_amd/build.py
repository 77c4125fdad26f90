"""Build libgk.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgk.so")
CALIB_LIB = os.path.join(HERE, "libgk_calib.so")   # roofline calibration kernels
CALIB_SOURCES = ["gk_calib.hip"]
LOADGEN_LIB = os.path.join(HERE, "libgk_loadgen.so")  # served-bench load generator
LOADGEN_SOURCES = ["gk_loadgen.cpp"]                   # host-only, links libgk.so
SOURCES = ["gk_api.hip", "gk_encode.hip", "gk_filter.hip", "gk_fused.hip", "gk_host.hip",
           "gk_mixed.hip", "gk_reference.hip", "gk_server.hip", "gk_verify.hip"]
HOST_SOURCES = ["gk_host_encode.cpp"]     # host-only C++ (no device code)
ARCH = os.environ.get("GK_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"
CXX = os.environ.get("GK_HOST_CXX", "/opt/rocm/llvm/bin/clang++")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # never let the compiler form packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if src.endswith(".cpp"):
        cmd = [CXX, "-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + HOST_SOURCES + CALIB_SOURCES + LOADGEN_SOURCES
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    for lib, parts in ((LIB, SOURCES + HOST_SOURCES), (CALIB_LIB, CALIB_SOURCES)):
        tmp = lib + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread",
               *[objs[p] for p in parts], "-o", tmp]
        if lib == LIB:      # trace ranges (roctx)
            cmd += ["-L", ROCM_LIB, "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc link failed for {os.path.basename(lib)}")
        os.replace(tmp, lib)
        if verbose:
            print(f"built {lib}")
    tmp = LOADGEN_LIB + ".tmp"
    cmd = [CXX, "-shared", "-fPIC", "-pthread", objs[LOADGEN_SOURCES[0]], "-L", HERE, "-lgk",
           "-Wl,-rpath,$ORIGIN", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed for libgk_loadgen.so")
    os.replace(tmp, LOADGEN_LIB)
    if verbose:
        print(f"built {LOADGEN_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
