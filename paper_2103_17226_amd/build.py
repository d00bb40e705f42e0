"""Build the HIP library (libqkc.so) in-tree for gfx950 with hipcc.

Usage: python -m paper_2103_17226_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqkc.so")
SOURCES = [os.path.join(CSRC, "qkc_host.cpp"), os.path.join(CSRC, "qkc_kernels.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (plain scalar FP32 only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


# the plain CPU evaluator (a host-only baseline library, no HIP)
CPU_SOURCE = os.path.join(HERE, "cpu", "qkc_cpu.cpp")
CPU_LIB = os.path.join(HERE, "libqkc_cpu.so")
CXX = os.environ.get("CXX", "g++")
CPU_FLAGS = ["-O3", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", "-I", INCLUDE]


def build_cpu(verbose: bool = False) -> str:
    """Compile the CPU evaluator into paper_2103_17226_amd/libqkc_cpu.so."""
    tmp = CPU_LIB + ".tmp"
    cmd = [CXX] + CPU_FLAGS + [CPU_SOURCE, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False) -> str:
    """Compile every source into paper_2103_17226_amd/libqkc.so and the CPU
    evaluator into libqkc_cpu.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-x", "hip"] + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_cpu(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
