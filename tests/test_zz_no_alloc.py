"""The allocation-free entry point (mst_solve_noalloc) through the C ABI: on
the same inputs it gives the same bytes, total, status and round statistics
as mst_solve, and the oracle's tree.  Calls come in a row on the one device
scratch, each later call smaller than the one before it (stale contents of a
larger solve must not leak into a smaller one), through both of its paths
(the per-round kernels and the one-workgroup solve), and on a disconnected
graph.
"""

import numpy as np
import pytest

import gpu_cases
import oracle
from paper_2005_06913_amd import graphgen as G

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_06913_amd as P
    P.load_library()
    return torch.device("cuda:0")


def run(dev, fn, g):
    import paper_2005_06913_amd as P
    s = torch.from_numpy(g.src).to(dev)
    d = torch.from_numpy(g.dst).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    in_mst = torch.full((g.m,), 7, dtype=torch.uint8, device=dev)  # garbage: must be overwritten
    total = torch.full((1,), 12345, dtype=torch.int64, device=dev).view(torch.uint64)
    st = fn(g.n, s, d, w, in_mst, total)
    torch.cuda.synchronize()
    return st, in_mst.cpu().numpy(), int(total.view(torch.int64).cpu().item()), P.mst_last_round_stats()


def sequence():
    """Graphs in decreasing size: round kernels (bucket, then LDS rounds), the
    one-workgroup path, a disconnected graph."""
    return [
        G.tree_plus_extra(1 << 18, 1 << 21, seed=41, name="random_n262144_m2M"),
        G.tree_plus_extra(60_000, 420_001, seed=42, name="random_n60000_ragged"),
        G.workload("random_n1k_m8k"),
        gpu_cases.small_cases()[-1],  # three parts plus isolated vertices
        G.tree_plus_extra(300, 900, seed=43, name="random_n300"),
    ]


def test_noalloc_equals_solve_in_a_row(dev):
    import paper_2005_06913_amd as P
    gs = sequence()
    assert all(gs[i].m > gs[i + 1].m for i in range(len(gs) - 1))
    for rep in range(2):  # the second pass reuses scratch left by the smaller graphs
        for g in gs:
            print(f"[case] noalloc rep={rep} {g.name} n={g.n} m={g.m}", flush=True)
            want = run(dev, P.mst_solve, g)
            got = run(dev, P.mst_solve_noalloc, g)
            k = oracle.kruskal(g.n, g.src, g.dst, g.w)
            assert got[0] == want[0] == k.status, (g.name, got[0], want[0], k.status)
            assert got[2] == want[2] == k.total, (g.name, got[2], want[2], k.total)
            assert np.array_equal(got[1], want[1]), f"{g.name}: edge flags differ from mst_solve"
            assert np.array_equal(got[1], k.in_mst), f"{g.name}: edge flags differ from the oracle"
            assert np.array_equal(got[3], want[3]), f"{g.name}: round statistics differ\n{got[3]}\n{want[3]}"


def test_noalloc_second_call_smaller(dev):
    """Two calls in a row on the round-kernel path, the second with a smaller input."""
    import paper_2005_06913_amd as P
    big = G.tree_plus_extra(200_000, 1_600_000, seed=44, name="big")
    small = G.tree_plus_extra(30_000, 150_003, seed=45, name="smaller")
    with P.small_limit(0):
        for g in (big, small):
            print(f"[case] noalloc pair {g.name} n={g.n} m={g.m}", flush=True)
            want = run(dev, P.mst_solve, g)
            got = run(dev, P.mst_solve_noalloc, g)
            assert got[0] == want[0] == 0
            assert got[2] == want[2]
            assert np.array_equal(got[1], want[1])
            assert np.array_equal(got[3], want[3])


def test_noalloc_edge_cases_and_limit(dev):
    import paper_2005_06913_amd as P
    for name, n, s, d, w in gpu_cases.edge_cases():
        g = G.Graph(n, s, d, w, name)
        print(f"[case] noalloc edge {name}", flush=True)
        want = run(dev, P.mst_solve, g)
        got = run(dev, P.mst_solve_noalloc, g)
        assert got[0] == want[0], name
        assert got[2] == want[2], name
        assert np.array_equal(got[1], want[1]), name
    # out of range id: detected on the device, as mst_solve does
    g = G.Graph(5, np.array([0, 1, 7], np.int32), np.array([1, 2, 3], np.int32), np.array([1, 2, 3], np.uint32))
    with P.small_limit(0):
        assert run(dev, P.mst_solve_noalloc, g)[0] == P.MSTX_ERR_VERTEX_RANGE
    assert run(dev, P.mst_solve_noalloc, g)[0] == P.MSTX_ERR_VERTEX_RANGE
    # over the scratch: rejected before any device work, then a good call still works
    s = torch.zeros(1, dtype=torch.int32, device=dev)
    lib = P.load_library()
    import ctypes
    one = ctypes.c_void_p(s.data_ptr())
    assert lib.mst_solve_noalloc(1 << 20, 1 << 23, one, one, one, one, one, None) == P.MSTX_ERR_SCRATCH_LIMIT
    k = G.workload("random_n1k_m8k")
    with P.small_limit(0):
        got = run(dev, P.mst_solve_noalloc, k)
    assert got[0] == 0 and got[2] == oracle.kruskal(k.n, k.src, k.dst, k.w).total
