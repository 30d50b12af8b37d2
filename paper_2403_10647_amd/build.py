"""Compile the HIP library (libgridbuild.so) for gfx950, in-tree.

    python -m paper_2403_10647_amd.build

Every HIP source is built with contraction off (the cell map is an exact FP32
sequence) and packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgridbuild.so")
SOURCES = ["gridbuild.hip"]
HEADERS = ["common.hpp", "grid.hpp", "tiles.hpp", "kernels.hpp", "sort.hpp", "ranges.hpp", "scan.hpp", "cull.hpp",
           "compact.hpp", "raycast.hpp"]
ARCH = os.environ.get("GRIDBUILD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


C_CHECK_SRC = os.path.join(ROOT, "tests", "c_abi", "check_build.c")
C_CHECK_BIN = os.path.join(ROOT, "tests", "c_abi", "check_build")


def build_c_check(verbose: bool = False) -> str:
    """A plain C caller of the library (tests/c_abi): gridbuild.h and the HIP
    runtime API only, compiled by the host C compiler and linked to the built
    library, to show the boundary needs neither Python nor torch."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(rocm, 'include')}", f"-I{os.path.join(ROOT, 'include')}",
           C_CHECK_SRC, "-o", C_CHECK_BIN, f"-L{HERE}", "-lgridbuild", f"-L{os.path.join(rocm, 'lib')}",
           "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN/../../paper_2403_10647_amd",
           f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return C_CHECK_BIN


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_c_check(verbose="-v" in sys.argv)
    print(LIB)
