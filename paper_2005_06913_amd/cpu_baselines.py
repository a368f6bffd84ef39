"""ctypes binding of libmstx_cpu.so: the paper's CPU Boruvka variants
(sequential, sequential with covered edges, parallel with permission words,
parallel with compare-and-swap), same names as include/mstx_cpu.h.

These run on the host for context beside the GPU path; they are not used by
it.  Inputs are numpy arrays.
"""

from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmstx_cpu.so")

MSTX_CPU_SEQ_PLAIN = 0
MSTX_CPU_SEQ_COVERED = 1
MSTX_CPU_PAR_LOCK = 2
MSTX_CPU_PAR_CAS = 3
VARIANTS = (MSTX_CPU_SEQ_PLAIN, MSTX_CPU_SEQ_COVERED, MSTX_CPU_PAR_LOCK, MSTX_CPU_PAR_CAS)

_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built: python -m paper_2005_06913_amd.build")
    lib = ctypes.CDLL(path)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mst_cpu_solve.argtypes = [ctypes.c_int, i32, i32, i64, p, p, p, p, p, p]
    lib.mst_cpu_solve.restype = ctypes.c_int
    lib.mst_cpu_variant_name.argtypes = [ctypes.c_int]
    lib.mst_cpu_variant_name.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = lib
    return lib


class CpuResult(NamedTuple):
    status: int
    in_mst: np.ndarray  # uint8 [m]
    total: int
    rounds: int


def mst_cpu_variant_name(variant: int) -> str:
    return load_library().mst_cpu_variant_name(int(variant)).decode()


def mst_cpu_solve(variant: int, threads: int, n: int, src, dst, w, lib=None) -> CpuResult:
    lib = lib or load_library()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    w = np.ascontiguousarray(w, np.uint32)
    m = src.shape[0]
    if dst.shape[0] != m or w.shape[0] != m:
        raise ValueError("src, dst and w must have the same length")
    in_mst = np.zeros(max(m, 1), np.uint8)
    total = np.zeros(1, np.uint64)
    rounds = np.zeros(1, np.int64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    st = lib.mst_cpu_solve(int(variant), int(threads), int(n), int(m), ptr(src), ptr(dst), ptr(w), ptr(in_mst),
                           ptr(total), ptr(rounds))
    return CpuResult(int(st), in_mst[:m], int(total[0]), int(rounds[0]))
