"""Build the HIP library liblbcg.so for gfx950 (run on any host; hipcc cross-compiles)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbcg.so")
SOURCES = ["lbcg_capi.hip", "lbcg_mlp.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (binary32 code is emitted as scalar VALU ops)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_capi_demo(verbose: bool = False) -> str:
    """Compile tests/capi_demo.c, a C program that uses the library through include/lbcg.h only
    (gcc, linked against liblbcg.so and the HIP runtime for its own device allocation)."""
    root = os.path.dirname(HERE)
    src = os.path.join(root, "tests", "capi_demo.c")
    exe = os.path.join(root, "tests", "capi_demo")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", src, "-I", os.path.join(root, "include"),
           "-I", os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__", "-L", HERE, "-llbcg",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN/../paper_2206_02145_amd",
           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return exe


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
