"""Build libdqmc.so (HIP, gfx950) in-tree with hipcc.

``python -m paper_2302_10083_amd.build`` or ``build()`` from Python.  Every
call compiles; loaders only build when no library exists yet.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdqmc.so")
SOURCES = ["api.hip", "server.hip", "k_low.hip", "k_col.hip", "k_col_chunk.hip", "k_list.hip", "k_batch.hip", "k_misc.hip", "tune.hip", "sparse.hip", "k_slice.hip"]
ARCH = os.environ.get("DQMC_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "--offload-arch=" + ARCH,
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def _compile(hipcc: str, src: str, obj: str, verbose: bool) -> None:
    cmd = [hipcc] + [f for f in HIPCC_FLAGS if f != "-shared"] + ["-I", os.path.join(ROOT, "include"), "-c", "-o",
                                                                  obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the library."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".%d.o" % os.getpid()) for s in SOURCES]
    workers = max(1, min(len(srcs), os.cpu_count() or 4, 16))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda so: _compile(hipcc, so[0], so[1], verbose), zip(srcs, objs)))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    try:
        subprocess.check_call(cmd)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    os.replace(tmp, LIB)
    build_example(verbose)
    return LIB


EXAMPLE_SRC = os.path.join(HERE, "examples", "c_primes.c")
EXAMPLE_BIN = os.path.join(HERE, "examples", "c_primes")


def build_example(verbose: bool = False) -> str:
    """The plain-C user of the ABI (host code only, linked against libdqmc.so
    and the system HIP runtime)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = EXAMPLE_BIN + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), "-o", tmp, EXAMPLE_SRC, "-L", HERE, "-ldqmc",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN/..",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, EXAMPLE_BIN)
    return EXAMPLE_BIN


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
