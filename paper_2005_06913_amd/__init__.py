"""MI355X (gfx950) parallel Boruvka minimum spanning tree.

The product is the HIP library ``libmstx.so`` behind the C ABI of
``include/mstx.h``; this package holds its sources (``csrc/``), its build
script and a thin ctypes binding with the same function names.  PyTorch is
used only for device memory and streams.

``graphgen`` holds the seeded synthetic input generators.
"""

from .binding import (  # noqa: F401
    EXPORTS,
    MSTX_DISCONNECTED,
    MSTX_ERR_DEVICE,
    MSTX_ERR_INVALID_ARG,
    MSTX_ERR_OUT_OF_MEMORY,
    MSTX_ERR_SCRATCH_LIMIT,
    MSTX_ERR_TOO_LARGE,
    MSTX_ERR_VERTEX_RANGE,
    MSTX_OK,
    MstxError,
    Solution,
    bucket_limit,
    dense_limit,
    load_library,
    mid_limit,
    small_limit,
    tail_limit,
    mst_batched_workspace_bytes,
    mst_csr_to_edges,
    mst_last_round_stats,
    mst_profile_enable,
    mst_profile_read,
    mst_profile_read_rounds,
    mst_select_min_edges,
    mst_set_bucket_limit,
    mst_set_dense_limit,
    mst_set_mid_limit,
    mst_set_scan_occupancy,
    mst_set_sparse_limit,
    mst_solve_wait_round,
    mst_batched_plan_create,
    mst_batched_plan_run,
    mst_batched_plan_destroy,
    sparse_limit,
    mst_set_small_limit,
    mst_set_tail_limit,
    mst_solve,
    mst_solve_advance,
    mst_solve_batched,
    mst_solve_begin,
    mst_solve_end,
    mst_solve_noalloc,
    mst_status_string,
    mst_workspace_bytes,
    mst_workspace_release,
    solve,
)
