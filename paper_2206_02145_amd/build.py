"""Build the HIP library liblbcg.so for gfx950 (run on any host; hipcc cross-compiles)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbcg.so")
SOURCES = ["lbcg_capi.hip", "batch_kits.hip", "lbcg_mlp.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (binary32 code is emitted as scalar VALU ops)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def source_hash() -> str:
    """SHA-256 over the library's sources (every file in csrc/ and include/lbcg.h) and the compiler
    flags. The build stores it in the library (lbcg_source_hash), and the binding refuses a library
    whose stored hash differs from the sources next to it: a stale build fails loudly."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    paths = [os.path.join(CSRC, f) for f in files] + [os.path.join(os.path.dirname(HERE), "include", "lbcg.h")]
    for path in paths:
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:32]


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (hipcc for gfx950), then link the library."""
    from concurrent.futures import ThreadPoolExecutor
    define = f"-DLBCG_SOURCE_HASH=\"{source_hash()}\""
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs = [os.path.join(CSRC, os.path.splitext(src)[0] + ".o") for src in SOURCES]

    def compile_one(k):
        cmd = ["hipcc", *compile_flags, define, "-c", os.path.join(CSRC, SOURCES[k]), "-o", objs[k] + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(objs[k] + ".tmp", objs[k])

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
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
