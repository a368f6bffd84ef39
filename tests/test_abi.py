"""The C ABI without a GPU: the library loads, exports every function that
include/mstx.h declares, and its host-only paths (argument checks that run
before any HIP call, status strings, options, workspace sizing) behave as the
header states.  Also the host-side helper that compares round statistics.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import gpu_cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mstx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(mst_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2005_06913_amd import binding, build
    if not os.path.exists(build.LIB):
        build.build_library()
    return binding.load_library()


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("mst_solve", "mst_solve_batched", "mst_select_min_edges", "mst_workspace_bytes",
                 "mst_set_dense_limit", "mst_set_small_limit", "mst_set_tail_limit", "mst_set_mid_limit",
                 "mst_set_bucket_limit",
                 "mst_csr_to_edges", "mst_status_string"):
        assert must in names, names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    from paper_2005_06913_amd import binding as B
    codes = [B.MSTX_OK, B.MSTX_DISCONNECTED, B.MSTX_ERR_INVALID_ARG, B.MSTX_ERR_VERTEX_RANGE,
             B.MSTX_ERR_TOO_LARGE, B.MSTX_ERR_OUT_OF_MEMORY, B.MSTX_ERR_DEVICE, B.MSTX_ERR_SCRATCH_LIMIT]
    texts = [B.mst_status_string(c) for c in codes]
    assert len(set(texts)) == len(codes)
    assert B.mst_status_string(12345) == "unknown status"


def test_host_argument_checks(lib):
    """Errors the header says are decided on the host return before any device call."""
    c = ctypes
    null = c.c_void_p(0)
    dummy = c.c_void_p(16)  # never dereferenced: the checks fail first
    B = __import__("paper_2005_06913_amd.binding", fromlist=["x"])
    assert lib.mst_solve(-1, 0, null, null, null, null, null, null) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve(4, -1, null, null, null, null, null, null) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve(4, 1 << 32, dummy, dummy, dummy, dummy, dummy, null) == B.MSTX_ERR_TOO_LARGE
    assert lib.mst_solve(4, 3, null, dummy, dummy, dummy, dummy, null) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_select_min_edges(-5, 0, null, null, null, null, null) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_batched(-1, None, None, null, null, null, null, null, null, null) == \
        B.MSTX_ERR_INVALID_ARG
    vo = np.array([0, 3, 2], np.int64)  # decreasing offsets
    eo = np.array([0, 1, 2], np.int64)
    ptr = lambda a: a.ctypes.data_as(c.c_void_p)
    assert lib.mst_solve_batched(2, ptr(vo), ptr(eo), dummy, dummy, dummy, dummy, dummy, dummy, null) == \
        B.MSTX_ERR_INVALID_ARG
    assert lib.mst_last_round_stats(None, 4) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_last_round_stats(None, -1) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_workspace_bytes(-1, 5) == 0 and lib.mst_workspace_bytes(5, 1 << 32) == 0


def test_dense_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_dense_limit(-1)
    assert prev == gpu_cases.DENSE_MAX  # default
    try:
        assert B.mst_set_dense_limit(1000) == prev
        assert B.mst_set_dense_limit(-1) == gpu_cases.DENSE_MAX  # clamped
        assert B.mst_set_dense_limit(0) == gpu_cases.DENSE_MAX
        assert B.mst_set_dense_limit(-7) == 0
        with B.dense_limit(17):
            assert B.mst_set_dense_limit(-1) == 17
        assert B.mst_set_dense_limit(-1) == 0
    finally:
        B.mst_set_dense_limit(prev)


def test_small_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_small_limit(-1)
    assert prev == gpu_cases.SMALL_MAX
    try:
        assert B.mst_set_small_limit(100000) == prev
        assert B.mst_set_small_limit(-1) == gpu_cases.SMALL_MAX  # clamped
        with B.small_limit(0):
            assert B.mst_set_small_limit(-1) == 0
        assert B.mst_set_small_limit(-1) == gpu_cases.SMALL_MAX
    finally:
        B.mst_set_small_limit(prev)


def test_bucket_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_bucket_limit(-1)
    assert prev == gpu_cases.BUCKET_MAX
    try:
        assert B.mst_set_bucket_limit(2 ** 31 - 1) == prev
        assert B.mst_set_bucket_limit(-1) == gpu_cases.BUCKET_MAX  # clamped
        with B.bucket_limit(0):
            assert B.mst_set_bucket_limit(-1) == 0
        assert B.mst_set_bucket_limit(-1) == gpu_cases.BUCKET_MAX
    finally:
        B.mst_set_bucket_limit(prev)


def test_tail_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_tail_limit(-1)
    assert prev == gpu_cases.TAIL_MAX
    try:
        assert B.mst_set_tail_limit(10 ** 6) == prev
        assert B.mst_set_tail_limit(-1) == gpu_cases.TAIL_MAX  # clamped
        with B.tail_limit(0):
            assert B.mst_set_tail_limit(-1) == 0
        assert B.mst_set_tail_limit(-1) == gpu_cases.TAIL_MAX
    finally:
        B.mst_set_tail_limit(prev)


def test_csr_to_edges_host_checks(lib):
    """Argument errors are reported on the host, before any HIP call."""
    import ctypes
    from paper_2005_06913_amd import binding as B
    m = ctypes.c_int64(-7)
    one = ctypes.c_void_p(1)  # never dereferenced: the checks fail first
    assert lib.mst_csr_to_edges(-1, 0, one, None, None, None, None, None, ctypes.byref(m), None) == \
        B.MSTX_ERR_INVALID_ARG
    assert lib.mst_csr_to_edges(3, -1, one, None, None, None, None, None, ctypes.byref(m), None) == \
        B.MSTX_ERR_INVALID_ARG
    assert lib.mst_csr_to_edges(3, 4, None, one, one, one, one, one, ctypes.byref(m), None) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_csr_to_edges(3, 4, one, None, one, one, one, one, ctypes.byref(m), None) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_csr_to_edges(3, 4, one, one, one, one, one, one, None, None) == B.MSTX_ERR_INVALID_ARG
    assert m.value == -7


def test_mid_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_mid_limit(-1)
    assert prev == gpu_cases.MID_MAX
    vo = np.array([0, 100, 12100], np.int64)
    eo = np.array([0, 400, 100400], np.int64)
    try:
        with_mid = B.mst_batched_workspace_bytes(vo, eo)
        assert B.mst_set_mid_limit(10 ** 6) == prev
        assert B.mst_set_mid_limit(-1) == gpu_cases.MID_MAX  # clamped
        with B.mid_limit(0):
            assert B.mst_set_mid_limit(-1) == 0
            # the union path needs the round kernels' workspace: records per edge
            assert B.mst_batched_workspace_bytes(vo, eo) > with_mid
        assert B.mst_set_mid_limit(-1) == gpu_cases.MID_MAX
    finally:
        B.mst_set_mid_limit(prev)


def test_workspace_bytes(lib):
    from paper_2005_06913_amd import binding as B
    a = B.mst_workspace_bytes(1000, 8000)
    b = B.mst_workspace_bytes(1 << 20, 1 << 23)
    assert 0 < a < b
    # the edge stream dominates: at least 16 B of records per edge
    assert b >= 16 * (1 << 23)
    vo = np.array([0, 100, 20000], np.int64)
    eo = np.array([0, 400, 90000], np.int64)
    assert B.mst_batched_workspace_bytes(vo, eo) > 0


def test_kernel_names(lib):
    from paper_2005_06913_amd import binding as B
    names = [lib.mst_profile_kernel_name(i).decode() for i in range(64)]
    names = [x for x in names if x]
    assert "k_dense_finish" in names and "k_hook" in names and "k_round_tail" in names
    for mode in range(4):
        for stage in range(4):
            assert f"k_scan<{mode}, {stage}>" in names
    assert len(names) == len(set(names))
    prof = B.mst_profile_read()  # host counters only: no device call
    assert set(prof) == set(names)


# ------------------------------------------------- round statistics helper

def test_stats_consistent_rules():
    o = [(1000, 8000, 700), (300, 7000, 250), (50, 6500, 40), (10, 3000, 8), (2, 400, 1)]
    assert gpu_cases.stats_consistent(o, o)
    # dense finish at round 2 (50 components): adds 40 + 8 + 1
    assert gpu_cases.stats_consistent(o[:2] + [(50, 6500, 49)], o)
    # wrong sum, wrong live count, a count above the limit, a changed prefix
    assert not gpu_cases.stats_consistent(o[:2] + [(50, 6500, 48)], o)
    assert not gpu_cases.stats_consistent(o[:2] + [(50, 6400, 49)], o)
    assert not gpu_cases.stats_consistent(o[:2] + [(50, 6500, 49)], o, limit=49)
    assert not gpu_cases.stats_consistent([(1000, 8000, 701)] + o[1:2] + [(50, 6500, 49)], o)
    assert not gpu_cases.stats_consistent(o + [(1, 0, 0)], o)
    assert not gpu_cases.stats_consistent([], o)


def test_noalloc_scratch_limit_on_host(lib):
    """mst_solve_noalloc rejects a graph whose workspace exceeds its fixed
    device scratch before any HIP call (the pointers are never dereferenced)."""
    from paper_2005_06913_amd import binding as B
    dummy = ctypes.c_void_p(16)
    assert lib.mst_solve_noalloc(1 << 20, 1 << 23, dummy, dummy, dummy, dummy, dummy, None) == \
        B.MSTX_ERR_SCRATCH_LIMIT
    assert lib.mst_solve_noalloc(-1, 0, None, None, None, None, None, None) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_noalloc(4, 1 << 32, dummy, dummy, dummy, dummy, dummy, None) == B.MSTX_ERR_TOO_LARGE
    # the documented examples fit: workspace plus 2 KB of records within 256 MiB
    for n, m in ((1 << 20, 1 << 22), (1 << 18, 5 << 20)):
        assert B.mst_workspace_bytes(n, m) + 2048 <= 256 << 20
    assert "256 MiB" in B.mst_status_string(B.MSTX_ERR_SCRATCH_LIMIT)


def test_profile_read_rounds_host(lib):
    """Per-round profile counters: host arrays only, no device call."""
    from paper_2005_06913_amd import binding as B
    K = lib.mst_profile_read_rounds(None, None, None, 0)
    names = [lib.mst_profile_kernel_name(i).decode() for i in range(K)]
    assert K > 0 and all(names)
    assert lib.mst_profile_read_rounds(None, None, None, 3) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_profile_read_rounds(None, None, None, -1) == B.MSTX_ERR_INVALID_ARG
    was = B.mst_profile_enable(True)  # zeroes the counters
    try:
        assert B.mst_profile_read_rounds() == {}
    finally:
        B.mst_profile_enable(was)


def test_stepwise_host_checks(lib):
    """mst_solve_begin / advance / end refuse bad arguments before any device
    call and leave no handle behind."""
    from paper_2005_06913_amd import binding as B
    c = ctypes
    dummy = c.c_void_p(16)
    h = c.c_void_p(0)
    assert lib.mst_solve_begin(-1, 0, None, None, None, None, None, None, c.byref(h)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_begin(4, 1 << 32, dummy, dummy, dummy, dummy, dummy, None, c.byref(h)) == \
        B.MSTX_ERR_TOO_LARGE
    assert lib.mst_solve_begin(4, 3, dummy, dummy, dummy, None, dummy, None, c.byref(h)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_begin(4, 3, dummy, dummy, dummy, dummy, dummy, None, None) == B.MSTX_ERR_INVALID_ARG
    assert h.value is None
    done = c.c_int32(0)
    assert lib.mst_solve_advance(None, c.byref(done)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_wait_round(None, c.byref(done)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_solve_end(None) == B.MSTX_ERR_INVALID_ARG


def test_sparse_limit_option(lib):
    from paper_2005_06913_amd import binding as B
    prev = B.mst_set_sparse_limit(-1)
    try:
        assert prev == gpu_cases.SPARSE_DEFAULT
        assert B.mst_set_sparse_limit(0) == prev
        with B.sparse_limit(123):
            assert B.mst_set_sparse_limit(-1) == 123
        assert B.mst_set_sparse_limit(-1) == 0
    finally:
        B.mst_set_sparse_limit(prev)


def test_batched_plan_host_checks(lib):
    """mst_batched_plan_create / run / destroy refuse bad arguments on the host."""
    from paper_2005_06913_amd import binding as B
    c = ctypes
    h = c.c_void_p(0)
    dummy = c.c_void_p(16)
    vo = np.array([0, 3, 2], np.int64)  # decreasing offsets
    eo = np.array([0, 1, 2], np.int64)
    ptr = lambda a: a.ctypes.data_as(c.c_void_p)
    assert lib.mst_batched_plan_create(2, ptr(vo), ptr(eo), dummy, dummy, dummy, dummy, dummy, dummy, None,
                                       c.byref(h)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_batched_plan_create(0, None, None, None, None, None, None, None, None, None,
                                       c.byref(h)) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_batched_plan_create(1, ptr(vo), ptr(eo), dummy, dummy, dummy, dummy, dummy, dummy, None,
                                       None) == B.MSTX_ERR_INVALID_ARG
    assert h.value is None
    assert lib.mst_batched_plan_run(None, None) == B.MSTX_ERR_INVALID_ARG
    assert lib.mst_batched_plan_destroy(None) == B.MSTX_ERR_INVALID_ARG
