"""Build libslrng.so (the C-ABI library with the gfx950 kernels) in-tree.

hipcc cross-compiles for gfx950 without a GPU.  All HIP code is built with
packed FP32 instructions disabled (-Xclang -target-feature -Xclang
-packed-fp32-ops)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslrng.so")
HIP_SOURCES = ["kernels.hip", "kernels32.hip", "batch.hip", "lincomp.hip", "batch_static.hip", "xpow.hip"]  # device code: hipcc for gfx950
HOST_SOURCES = ["api.cpp", "f2poly.cpp", "batch.cpp", "server.cpp", "memory.cpp"]  # host C++ against the HIP runtime API
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]
HOST = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unknown-pragmas", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


def build(verbose: bool = False) -> str:
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    procs = []
    jobs = [([HIPCC, *COMMON, "-x", "hip"], s) for s in HIP_SOURCES] + \
        [(["g++", *HOST], s) for s in HOST_SOURCES]
    for pre, src in jobs:
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = [*pre, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
