"""ctypes binding of the mstx C ABI (``include/mstx.h``).

The functions keep the C names and only marshal arguments: torch tensors on
the current HIP device become device pointers, the current torch stream
becomes the ``stream`` argument.  Every step of the solve runs in the HIP
kernels of ``libmstx.so``; if that library is missing or cannot be loaded the
call raises -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmstx.so")

MSTX_OK = 0
MSTX_DISCONNECTED = 1
MSTX_ERR_INVALID_ARG = -1
MSTX_ERR_VERTEX_RANGE = -2
MSTX_ERR_TOO_LARGE = -3
MSTX_ERR_OUT_OF_MEMORY = -4
MSTX_ERR_DEVICE = -5
MSTX_ERR_SCRATCH_LIMIT = -6

EXPORTS = ("mst_solve", "mst_solve_batched", "mst_batched_workspace_bytes", "mst_select_min_edges",
           "mst_last_round_stats", "mst_workspace_bytes", "mst_status_string", "mst_profile_enable",
           "mst_profile_read", "mst_profile_kernel_name", "mst_workspace_release", "mst_set_dense_limit", "mst_set_small_limit",
           "mst_set_tail_limit", "mst_set_mid_limit", "mst_set_bucket_limit", "mst_csr_to_edges",
           "mst_solve_noalloc", "mst_profile_read_rounds", "mst_set_scan_occupancy", "mst_solve_begin",
           "mst_solve_advance", "mst_solve_end", "mst_set_sparse_limit", "mst_solve_wait_round",
           "mst_batched_plan_create", "mst_batched_plan_run", "mst_batched_plan_destroy")

_lib = None


class MstxError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"mstx status {status}: {mst_status_string(status)}")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Load ``libmstx.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2005_06913_amd.build` "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.mst_solve.argtypes = [i32, i64, p, p, p, p, p, p]
    lib.mst_solve.restype = ctypes.c_int
    lib.mst_solve_begin.argtypes = [i32, i64, p, p, p, p, p, p, ctypes.POINTER(p)]
    lib.mst_solve_begin.restype = ctypes.c_int
    lib.mst_solve_advance.argtypes = [p, ctypes.POINTER(i32)]
    lib.mst_solve_advance.restype = ctypes.c_int
    lib.mst_solve_wait_round.argtypes = [p, ctypes.POINTER(i32)]
    lib.mst_solve_wait_round.restype = ctypes.c_int
    lib.mst_solve_end.argtypes = [p]
    lib.mst_solve_end.restype = ctypes.c_int
    lib.mst_solve_noalloc.argtypes = [i32, i64, p, p, p, p, p, p]
    lib.mst_solve_noalloc.restype = ctypes.c_int
    lib.mst_solve_batched.argtypes = [i32, p, p, p, p, p, p, p, p, p]
    lib.mst_solve_batched.restype = ctypes.c_int
    lib.mst_batched_plan_create.argtypes = [i32, p, p, p, p, p, p, p, p, p, ctypes.POINTER(p)]
    lib.mst_batched_plan_create.restype = ctypes.c_int
    lib.mst_batched_plan_run.argtypes = [p, p]
    lib.mst_batched_plan_run.restype = ctypes.c_int
    lib.mst_batched_plan_destroy.argtypes = [p]
    lib.mst_batched_plan_destroy.restype = ctypes.c_int
    lib.mst_batched_workspace_bytes.argtypes = [i32, p, p]
    lib.mst_batched_workspace_bytes.restype = ctypes.c_size_t
    lib.mst_select_min_edges.argtypes = [i32, i64, p, p, p, p, p]
    lib.mst_select_min_edges.restype = ctypes.c_int
    lib.mst_csr_to_edges.argtypes = [i32, i64, p, p, p, p, p, p, p, p]
    lib.mst_csr_to_edges.restype = ctypes.c_int
    lib.mst_last_round_stats.argtypes = [p, i32]
    lib.mst_last_round_stats.restype = ctypes.c_int
    lib.mst_workspace_bytes.argtypes = [i32, i64]
    lib.mst_workspace_bytes.restype = ctypes.c_size_t
    lib.mst_status_string.argtypes = [ctypes.c_int]
    lib.mst_status_string.restype = ctypes.c_char_p
    lib.mst_profile_enable.argtypes = [ctypes.c_int]
    lib.mst_profile_enable.restype = ctypes.c_int
    lib.mst_profile_read.argtypes = [p, p, p, i32]
    lib.mst_profile_read.restype = ctypes.c_int
    lib.mst_workspace_release.argtypes = [p]
    lib.mst_workspace_release.restype = ctypes.c_int
    lib.mst_set_dense_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_dense_limit.restype = ctypes.c_int32
    lib.mst_set_small_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_small_limit.restype = ctypes.c_int32
    lib.mst_set_tail_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_tail_limit.restype = ctypes.c_int32
    lib.mst_set_mid_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_mid_limit.restype = ctypes.c_int32
    lib.mst_set_scan_occupancy.argtypes = [ctypes.c_int32]
    lib.mst_set_scan_occupancy.restype = ctypes.c_int32
    lib.mst_set_bucket_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_bucket_limit.restype = ctypes.c_int32
    lib.mst_set_sparse_limit.argtypes = [ctypes.c_int32]
    lib.mst_set_sparse_limit.restype = ctypes.c_int32
    lib.mst_profile_read_rounds.argtypes = [p, p, p, i32]
    lib.mst_profile_read_rounds.restype = ctypes.c_int
    lib.mst_profile_kernel_name.argtypes = [ctypes.c_int]
    lib.mst_profile_kernel_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def mst_workspace_release(stream=None) -> int:
    """Free the library's workspace cached for (current device, stream)."""
    return int(load_library().mst_workspace_release(_stream_handle(stream)))


def mst_set_dense_limit(limit: int) -> int:
    """Set the component count at or below which a solve ends with the dense
    finish (0: off, clamped to 200; negative: query).  Returns the previous limit."""
    return int(load_library().mst_set_dense_limit(int(limit)))


def mst_set_small_limit(limit: int) -> int:
    """Set the vertex count up to which mst_solve uses the one-workgroup path
    (0: off, clamped to 8192; negative: query).  Returns the previous limit."""
    return int(load_library().mst_set_small_limit(int(limit)))


def mst_set_tail_limit(limit: int) -> int:
    """Set the component-count bound up to which a round's hook .. relabel run as
    one workgroup (0: off, clamped to 10240; negative: query).  Returns the
    previous limit."""
    return int(load_library().mst_set_tail_limit(int(limit)))


def mst_set_mid_limit(limit: int) -> int:
    """Set the vertex count up to which mst_solve_batched solves a graph above
    8192 vertices (and with at most 2^21 edges) with one workgroup; graphs with
    up to 65536 vertices are first contracted by one workgroup to at most that
    many components.  At most 8192: off (disjoint-union chunks instead);
    clamped to 16280; negative: query.  Returns the previous limit."""
    return int(load_library().mst_set_mid_limit(int(limit)))


def mst_set_bucket_limit(limit: int) -> int:
    """Set the component-count bound up to which a round above the LDS range
    takes its minima in bucket mode; above it the filtered global atomics
    (0: never bucket mode; clamped to 16760832; negative: query).  Returns the
    previous limit."""
    return int(load_library().mst_set_bucket_limit(int(limit)))


def mst_set_sparse_limit(live_edges: int) -> int:
    """Set the live-edge bound under which a late round tries the sparse finish
    (0: never; negative: query).  Returns the previous value."""
    return int(load_library().mst_set_sparse_limit(int(live_edges)))


class sparse_limit:
    """Context manager: ``with sparse_limit(0): ...`` never tries the sparse finish."""

    def __init__(self, limit: int):
        self.limit = limit

    def __enter__(self):
        self.prev = mst_set_sparse_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_sparse_limit(self.prev)
        return False


def mst_set_scan_occupancy(wg_per_cu: int) -> int:
    """Set how many LDS-mode scan workgroups share a compute unit (0: chosen from
    the LDS size; negative: query).  Returns the previous value."""
    return int(load_library().mst_set_scan_occupancy(int(wg_per_cu)))


class bucket_limit:
    """Context manager: ``with bucket_limit(0): ...`` takes every round above the
    LDS range with filtered global atomic minima."""

    def __init__(self, limit: int):
        self.limit = limit
        self.prev = None

    def __enter__(self):
        self.prev = mst_set_bucket_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_bucket_limit(self.prev)
        return False


class mid_limit:
    """Context manager: ``with mid_limit(0): ...`` solves every batched graph above
    8192 vertices in disjoint-union chunks."""

    def __init__(self, limit: int):
        self.limit = limit
        self.prev = None

    def __enter__(self):
        self.prev = mst_set_mid_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_mid_limit(self.prev)
        return False


class tail_limit:
    """Context manager: ``with tail_limit(0): ...`` runs every round's hook .. relabel
    as grid-wide kernels."""

    def __init__(self, limit: int):
        self.limit = limit
        self.prev = None

    def __enter__(self):
        self.prev = mst_set_tail_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_tail_limit(self.prev)
        return False


class small_limit:
    """Context manager: ``with small_limit(0): ...`` always takes the per-round kernel chain."""

    def __init__(self, limit: int):
        self.limit = limit
        self.prev = None

    def __enter__(self):
        self.prev = mst_set_small_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_small_limit(self.prev)
        return False


class dense_limit:
    """Context manager: ``with dense_limit(0): ...`` runs plain Boruvka rounds only."""

    def __init__(self, limit: int):
        self.limit = limit
        self.prev = None

    def __enter__(self):
        self.prev = mst_set_dense_limit(self.limit)
        return self

    def __exit__(self, *exc):
        mst_set_dense_limit(self.prev)
        return False


def mst_status_string(status: int) -> str:
    return load_library().mst_status_string(int(status)).decode()


def mst_workspace_bytes(n: int, m: int) -> int:
    return int(load_library().mst_workspace_bytes(int(n), int(m)))


def mst_solve(n, src, dst, w, out_in_mst, out_total_weight, stream=None) -> int:
    """C ``mst_solve`` on torch tensors: int32 src/dst, uint32 w, uint8 out_in_mst[m],
    uint64 out_total_weight[1] (all on the current GPU).  Returns the status."""
    import torch
    m = int(src.numel())
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_in_mst, torch.uint8, "out_in_mst", m),
            _dev_ptr(out_total_weight, torch.uint64, "out_total_weight", 1))
    return int(load_library().mst_solve(int(n), m, *args, _stream_handle(stream)))


def mst_solve_noalloc(n, src, dst, w, out_in_mst, out_total_weight, stream=None) -> int:
    """C ``mst_solve_noalloc`` (mst_solve on the library's fixed device scratch,
    allocating nothing); same tensors as ``mst_solve``.  Returns the status."""
    import torch
    m = int(src.numel())
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_in_mst, torch.uint8, "out_in_mst", m),
            _dev_ptr(out_total_weight, torch.uint64, "out_total_weight", 1))
    return int(load_library().mst_solve_noalloc(int(n), m, *args, _stream_handle(stream)))


def mst_solve_begin(n, src, dst, w, out_in_mst, out_total_weight, stream=None):
    """C ``mst_solve_begin`` (round-by-round solve): returns (status, handle);
    the handle is None on a negative status.  The tensors must stay alive
    until ``mst_solve_end``."""
    import torch
    m = int(src.numel())
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_in_mst, torch.uint8, "out_in_mst", m),
            _dev_ptr(out_total_weight, torch.uint64, "out_total_weight", 1))
    h = ctypes.c_void_p(0)
    st = int(load_library().mst_solve_begin(int(n), m, *args, _stream_handle(stream), ctypes.byref(h)))
    return st, (h if st >= 0 and h.value else None)


def mst_solve_advance(handle) -> bool:
    """C ``mst_solve_advance``: enqueues the next round if the last has finished;
    True once the solve has ended."""
    done = ctypes.c_int32(0)
    rc = load_library().mst_solve_advance(handle, ctypes.byref(done))
    if rc < 0:
        raise MstxError(rc)
    return bool(done.value)


def mst_solve_wait_round(handle) -> bool:
    """C ``mst_solve_wait_round``: waits for the next round's record, takes it and
    enqueues what follows; True once the solve has ended."""
    done = ctypes.c_int32(0)
    rc = load_library().mst_solve_wait_round(handle, ctypes.byref(done))
    if rc < 0:
        raise MstxError(rc)
    return bool(done.value)


def mst_solve_end(handle) -> int:
    """C ``mst_solve_end``: completes the solve, frees the handle, returns the status."""
    return int(load_library().mst_solve_end(handle))


def _host_offsets(a, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int64)
    if a.ndim != 1 or a.shape[0] < 1:
        raise ValueError(f"{name} must be a 1-D array of G+1 offsets")
    return a


def mst_solve_batched(vertex_offsets, edge_offsets, src, dst, w, out_in_mst, out_total_weight, out_status,
                      stream=None) -> int:
    """C ``mst_solve_batched``: offsets are host int64 arrays [G+1] (numpy); src/dst (local ids),
    w, out_in_mst [sum m] and out_total_weight (uint64 [G]), out_status (int32 [G]) are GPU tensors."""
    import torch
    vo = _host_offsets(vertex_offsets, "vertex_offsets")
    eo = _host_offsets(edge_offsets, "edge_offsets")
    G = vo.shape[0] - 1
    if eo.shape[0] != G + 1:
        raise ValueError("vertex_offsets and edge_offsets must have the same length")
    m = int(eo[-1])
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_in_mst, torch.uint8, "out_in_mst", m),
            _dev_ptr(out_total_weight, torch.uint64, "out_total_weight", G),
            _dev_ptr(out_status, torch.int32, "out_status", G))
    return int(load_library().mst_solve_batched(G, vo.ctypes.data_as(ctypes.c_void_p),
                                                 eo.ctypes.data_as(ctypes.c_void_p), *args,
                                                 _stream_handle(stream)))


def mst_batched_plan_create(vertex_offsets, edge_offsets, src, dst, w, out_in_mst, out_total_weight, out_status,
                            stream=None):
    """C ``mst_batched_plan_create``: plans and captures the batched solve of this
    shape on these tensors; returns (status, plan) with plan None on a negative
    status.  The tensors must stay alive until ``mst_batched_plan_destroy``."""
    import torch
    vo = _host_offsets(vertex_offsets, "vertex_offsets")
    eo = _host_offsets(edge_offsets, "edge_offsets")
    G = vo.shape[0] - 1
    if eo.shape[0] != G + 1:
        raise ValueError("vertex_offsets and edge_offsets must have the same length")
    m = int(eo[-1])
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_in_mst, torch.uint8, "out_in_mst", m),
            _dev_ptr(out_total_weight, torch.uint64, "out_total_weight", G),
            _dev_ptr(out_status, torch.int32, "out_status", G))
    h = ctypes.c_void_p(0)
    st = int(load_library().mst_batched_plan_create(G, vo.ctypes.data_as(ctypes.c_void_p),
                                                     eo.ctypes.data_as(ctypes.c_void_p), *args,
                                                     _stream_handle(stream), ctypes.byref(h)))
    return st, (h if st >= 0 and h.value else None)


def mst_batched_plan_run(plan, stream=None) -> int:
    """C ``mst_batched_plan_run``: replays the captured solve on the stream (asynchronous)."""
    return int(load_library().mst_batched_plan_run(plan, _stream_handle(stream)))


def mst_batched_plan_destroy(plan) -> int:
    """C ``mst_batched_plan_destroy``: frees the plan (no run may be in flight)."""
    return int(load_library().mst_batched_plan_destroy(plan))


def mst_batched_workspace_bytes(vertex_offsets, edge_offsets) -> int:
    vo = _host_offsets(vertex_offsets, "vertex_offsets")
    eo = _host_offsets(edge_offsets, "edge_offsets")
    return int(load_library().mst_batched_workspace_bytes(vo.shape[0] - 1, vo.ctypes.data_as(ctypes.c_void_p),
                                                          eo.ctypes.data_as(ctypes.c_void_p)))


def mst_select_min_edges(n, src, dst, w, out_best, stream=None) -> int:
    """C ``mst_select_min_edges``: out_best uint64[n] <- lightest key per vertex."""
    import torch
    m = int(src.numel())
    args = (_dev_ptr(src, torch.int32, "src", m), _dev_ptr(dst, torch.int32, "dst", m),
            _dev_ptr(w, torch.uint32, "w", m), _dev_ptr(out_best, torch.uint64, "out_best", int(n)))
    return int(load_library().mst_select_min_edges(int(n), m, *args, _stream_handle(stream)))


def mst_csr_to_edges(n, row_ptr, col, w, stream=None):
    """C ``mst_csr_to_edges``: the edge list of a symmetric CSR adjacency (every
    arc u -> v with u < v, in row-major arc order) as new device tensors
    ``(src int32, dst int32, w uint32)``.  Raises MstxError on an error status."""
    import torch
    nnz = int(col.numel())
    dev = row_ptr.device
    src = torch.empty(nnz, dtype=torch.int32, device=dev)
    dst = torch.empty(nnz, dtype=torch.int32, device=dev)
    ww = torch.empty(nnz, dtype=torch.uint32, device=dev)
    m = ctypes.c_int64(0)
    rc = load_library().mst_csr_to_edges(
        int(n), nnz, _dev_ptr(row_ptr, torch.int64, "row_ptr", int(n) + 1), _dev_ptr(col, torch.int32, "col", nnz),
        _dev_ptr(w, torch.uint32, "w", nnz), _dev_ptr(src, torch.int32, "out_src"),
        _dev_ptr(dst, torch.int32, "out_dst"), _dev_ptr(ww, torch.uint32, "out_w"), ctypes.byref(m),
        _stream_handle(stream))
    if rc < 0:
        raise MstxError(rc)
    k = int(m.value)
    return src[:k], dst[:k], ww[:k]


def mst_last_round_stats(max_rounds: int = 40):
    """Per-round (components, live edges, edges added) of this thread's last mst_solve."""
    import numpy as np
    buf = np.zeros(3 * max_rounds, np.int64)
    k = load_library().mst_last_round_stats(buf.ctypes.data_as(ctypes.c_void_p), max_rounds)
    if k < 0:
        raise MstxError(k)
    return buf[:3 * k].reshape(k, 3)


def mst_profile_enable(enable: bool) -> bool:
    """Start (and zero) or stop per-kernel event timing; returns the previous state."""
    return bool(load_library().mst_profile_enable(1 if enable else 0))


def mst_profile_read() -> dict:
    """{kernel kind: (total ms, launches, algorithmic bytes)} accumulated while enabled."""
    import numpy as np
    lib = load_library()
    cap = 64
    ms = np.zeros(cap, np.float64)
    n = np.zeros(cap, np.int64)
    b = np.zeros(cap, np.float64)
    k = lib.mst_profile_read(ms.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
                             b.ctypes.data_as(ctypes.c_void_p), cap)
    if k < 0:
        raise MstxError(k)
    k = min(k, cap)
    return {lib.mst_profile_kernel_name(i).decode(): (float(ms[i]), int(n[i]), float(b[i])) for i in range(k)}


def mst_profile_read_rounds(max_rounds: int = 41) -> dict:
    """{round: {kernel: (total ms, launches, algorithmic bytes)}} accumulated while
    profiling is enabled (kernels with no launch in a round are left out)."""
    import numpy as np
    lib = load_library()
    K = lib.mst_profile_read_rounds(None, None, None, 0)
    if K < 0:
        raise MstxError(K)
    ms = np.zeros(max_rounds * K, np.float64)
    n = np.zeros(max_rounds * K, np.int64)
    b = np.zeros(max_rounds * K, np.float64)
    rc = lib.mst_profile_read_rounds(ms.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
                                     b.ctypes.data_as(ctypes.c_void_p), max_rounds)
    if rc < 0:
        raise MstxError(rc)
    names = [lib.mst_profile_kernel_name(i).decode() for i in range(K)]
    out = {}
    for r in range(max_rounds):
        row = {names[i]: (float(ms[r * K + i]), int(n[r * K + i]), float(b[r * K + i]))
               for i in range(K) if n[r * K + i]}
        if row:
            out[r] = row
    return out


class Solution(NamedTuple):
    in_mst: object  # torch.uint8 [m] on the GPU
    total: int
    status: int


def solve(n, src, dst, w, stream=None) -> Solution:
    """Allocate outputs and run ``mst_solve``; raises ``MstxError`` on a negative status."""
    import torch
    m = int(src.numel())
    in_mst = torch.empty(m, dtype=torch.uint8, device=src.device)
    total = torch.empty(1, dtype=torch.uint64, device=src.device)
    st = mst_solve(n, src, dst, w, in_mst, total, stream)
    if st < 0:
        raise MstxError(st)
    return Solution(in_mst, int(total.view(torch.int64).item()), st)
