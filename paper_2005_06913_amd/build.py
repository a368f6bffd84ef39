"""Builds libmstx.so (HIP, gfx950 only) and libmstx_cpu.so (the paper's CPU
variants, host compiler) in the package directory.

    python -m paper_2005_06913_amd.build
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmstx.so")
SOURCES = ["mstx_kernels.hip", "mstx_batched.hip", "mstx_csr.hip", "mstx_host.hip"]
CPU_LIB = os.path.join(PKG, "libmstx_cpu.so")
CPU_SOURCES = ["mstx_cpu.cpp"]
CXX = os.environ.get("CXX", "g++")
CPU_FLAGS = ["-O3", "-std=c++20", "-fPIC", "-shared", "-pthread", "-Wall"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed fp32 instructions stay off for all HIP code built here
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into ``libmstx.so`` (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; anything else is shown
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (p.stdout + p.stderr).splitlines() if noise not in ln]
    if p.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


def build_cpu_library(verbose: bool = False, out: str = CPU_LIB, extra=()) -> str:
    """Compile the CPU variants into ``libmstx_cpu.so`` (always recompiles)."""
    tmp = out + ".tmp"
    cmd = [CXX, *CPU_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp,
           *[os.path.join(CSRC, s) for s in CPU_SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("g++ failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
    print(build_cpu_library(verbose="-v" in sys.argv))
