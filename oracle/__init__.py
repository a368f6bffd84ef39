"""CPU oracle for the minimum spanning tree -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package.  The GPU library never calls it and it
shares no code with the GPU library.

The arithmetic lives in ``mst_oracle.c`` (plain C, built with gcc into
``liboracle.so``); this module only marshals numpy arrays through ctypes.

Routines (arXiv 2005.06913):
  * ``kruskal``   -- Kruskal's algorithm (Section 1 lists it among the classic
                     sequential MST algorithms);
  * ``boruvka``   -- the sequential Boruvka algorithm of Section 2.1 with the
                     "covered" optimisation, with per-round statistics;
  * ``check_mst`` -- certificate: forest, spanning, cycle property, total;
  * ``min_edge_keys`` -- the first round's edge loop alone: the lightest
                     edge key at every vertex.

Edges are ordered by ``(w[e], e)``; with the paper's distinct weights this is
the order by weight.  Pins (what the oracle is checked against) are in
``tests/test_oracle_pins.py``; none of them is derived from this code.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mst_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
DISCONNECTED = 1
ERR_ARG = -1
ERR_RANGE = -2
ERR_NOMEM = -4

CHECK_CODES = {
    0: "ok",
    -10: "in_mst holds a value other than 0/1",
    -11: "a self-loop is marked",
    -12: "marked edges contain a cycle",
    -13: "marked edges do not span every component",
    -14: "a non-tree edge precedes the maximum on its tree path (not minimum)",
    -15: "total differs from the sum of marked weights",
    -1: "invalid argument",
    -2: "vertex id out of range",
    -4: "out of memory",
}

_default = None


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no -march=native: the library also runs on other hosts)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                        "-o", tmp, src], check=True)
        os.replace(tmp, out)
    return out


def _bind(path: str):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_kruskal.argtypes = [i32, i64, p, p, p, p, p]
    lib.oracle_kruskal.restype = ctypes.c_int
    lib.oracle_boruvka.argtypes = [i32, i64, p, p, p, p, p, p, i32, p, p]
    lib.oracle_boruvka.restype = ctypes.c_int
    lib.oracle_check_mst.argtypes = [i32, i64, p, p, p, p, ctypes.c_uint64]
    lib.oracle_check_mst.restype = ctypes.c_int
    lib.oracle_min_edge_keys.argtypes = [i32, i64, p, p, p, p]
    lib.oracle_min_edge_keys.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _prep(src, dst, w):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    if not (src.shape == dst.shape == w.shape) or src.ndim != 1:
        raise ValueError("src, dst, w must be 1-D arrays of equal length")
    return src, dst, w


class MstResult(NamedTuple):
    in_mst: np.ndarray  # uint8 [m]
    total: int
    status: int


class BoruvkaResult(NamedTuple):
    in_mst: np.ndarray
    total: int
    status: int
    stats: np.ndarray  # int64 [rounds, 3]: components, live edges, edges added
    labels: np.ndarray | None  # int32 [n]: smallest vertex id of the final component


class Oracle:
    """ctypes handle on one build of the oracle library."""

    def __init__(self, path: str):
        self.path = path
        self.lib = _bind(path)

    def kruskal(self, n: int, src, dst, w) -> MstResult:
        src, dst, w = _prep(src, dst, w)
        m = src.shape[0]
        out = np.zeros(max(m, 1), np.uint8)
        total = ctypes.c_uint64(0)
        st = self.lib.oracle_kruskal(n, m, _ptr(src), _ptr(dst), _ptr(w), _ptr(out), ctypes.byref(total))
        return MstResult(out[:m], int(total.value), int(st))

    def boruvka(self, n: int, src, dst, w, max_rounds: int = 64, labels: bool = False) -> BoruvkaResult:
        src, dst, w = _prep(src, dst, w)
        m = src.shape[0]
        out = np.zeros(max(m, 1), np.uint8)
        total = ctypes.c_uint64(0)
        stats = np.zeros(3 * max_rounds, np.int64)
        rounds = ctypes.c_int32(0)
        lab = np.zeros(max(n, 1), np.int32) if labels else None
        st = self.lib.oracle_boruvka(n, m, _ptr(src), _ptr(dst), _ptr(w), _ptr(out), ctypes.byref(total),
                                    _ptr(stats), max_rounds, ctypes.byref(rounds),
                                    _ptr(lab) if lab is not None else None)
        r = min(int(rounds.value), max_rounds)
        return BoruvkaResult(out[:m], int(total.value), int(st), stats[:3 * r].reshape(r, 3),
                             lab[:n] if lab is not None else None)

    def check_mst(self, n: int, src, dst, w, in_mst, total: int) -> int:
        """0 if ``in_mst``/``total`` is the minimum spanning forest under (w, e); else a CHECK_CODES key."""
        src, dst, w = _prep(src, dst, w)
        in_mst = np.ascontiguousarray(in_mst, dtype=np.uint8)
        if in_mst.shape != src.shape:
            raise ValueError("in_mst must have one entry per edge")
        return int(self.lib.oracle_check_mst(n, src.shape[0], _ptr(src), _ptr(dst), _ptr(w),
                                            _ptr(in_mst), int(total)))

    def min_edge_keys(self, n: int, src, dst, w):
        """(status, uint64[n]): lightest key (w << 32 | e) of the non-loop edges at each vertex."""
        src, dst, w = _prep(src, dst, w)
        keys = np.zeros(max(n, 1), np.uint64)
        st = self.lib.oracle_min_edge_keys(n, src.shape[0], _ptr(src), _ptr(dst), _ptr(w), _ptr(keys))
        return int(st), keys[:max(n, 0)]


def default() -> Oracle:
    """The oracle built from ``mst_oracle.c`` (rebuilt when the source is newer)."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _default = Oracle(_LIB)
    return _default


def kruskal(n: int, src, dst, w) -> MstResult:
    return default().kruskal(n, src, dst, w)


def boruvka(n: int, src, dst, w, max_rounds: int = 64, labels: bool = False) -> BoruvkaResult:
    return default().boruvka(n, src, dst, w, max_rounds, labels)


def check_mst(n: int, src, dst, w, in_mst, total: int) -> int:
    return default().check_mst(n, src, dst, w, in_mst, total)


def min_edge_keys(n: int, src, dst, w):
    return default().min_edge_keys(n, src, dst, w)

