"""Build liblbmcg.so (HIP kernels + C entry points) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbmcg.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_host.cpp")]
ARCH = os.environ.get("LBMCG_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-x", "hip",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


EXAMPLE_SRC = os.path.join(CSRC, "c_api_example.c")
EXAMPLE = os.path.join(PKG, "lbm_c_example")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_example(verbose)
    return LIB


def build_example(verbose: bool = False) -> str:
    """The C example of the interface (plain C99 with gcc, linked against liblbmcg.so found next
    to it and the HIP runtime)."""
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(os.path.dirname(ROCM_LIB), "include"), "-I", INCLUDE,
           "-o", EXAMPLE + ".tmp", EXAMPLE_SRC, "-L", PKG, "-llbmcg", "-L", ROCM_LIB, "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + ROCM_LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(EXAMPLE + ".tmp", EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
