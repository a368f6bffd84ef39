"""GPU parity of the batched solve: every graph of a batch against the oracle.

A batch mixes graphs solved by one workgroup each (n <= 8192) with larger
graphs solved as chunks of a disjoint union; ties, self-loops, parallel
edges, isolated vertices, empty graphs and out-of-range ids are included.
Every graph's edge flags, total and status must equal the oracle's on that
graph alone.
"""

import numpy as np
import pytest

import gpu_cases
import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_06913_amd as P
    P.load_library()
    return torch.device("cuda:0")


def concat(graphs):
    """Batch arrays from a list of (n, src, dst, w)."""
    vo = np.zeros(len(graphs) + 1, np.int64)
    eo = np.zeros(len(graphs) + 1, np.int64)
    for i, (n, s, d, w) in enumerate(graphs):
        vo[i + 1] = vo[i] + n
        eo[i + 1] = eo[i] + len(s)
    cat = lambda k, dt: (np.concatenate([g[k] for g in graphs]).astype(dt) if eo[-1] else np.zeros(0, dt))
    return vo, eo, cat(1, np.int32), cat(2, np.int32), cat(3, np.uint32)


def run_batched(dev, vo, eo, src, dst, w):
    import paper_2005_06913_amd as P
    G = len(vo) - 1
    m = int(eo[-1])
    s = torch.from_numpy(src).to(dev)
    d = torch.from_numpy(dst).to(dev)
    ww = torch.from_numpy(w).to(dev)
    in_mst = torch.full((m,), 9, dtype=torch.uint8, device=dev)
    total = torch.full((G,), 77, dtype=torch.int64, device=dev).view(torch.uint64)
    status = torch.full((G,), 99, dtype=torch.int32, device=dev)
    rc = P.mst_solve_batched(vo, eo, s, d, ww, in_mst, total, status)
    torch.cuda.synchronize()
    return rc, in_mst.cpu().numpy(), total.view(torch.int64).cpu().numpy(), status.cpu().numpy()


def check_batch(dev, graphs, name):
    print(f"[case] batched {name}: {len(graphs)} graphs", flush=True)
    vo, eo, src, dst, w = concat(graphs)
    rc, in_mst, total, status = run_batched(dev, vo, eo, src, dst, w)
    assert rc == 0
    for i, (n, s, d, ww) in enumerate(graphs):
        k = oracle.kruskal(n, s, d, ww)
        a, b = eo[i], eo[i + 1]
        assert status[i] == k.status, f"{name} graph {i}: status {status[i]} != {k.status}"
        if k.status < 0:
            continue
        assert int(total[i]) == k.total, f"{name} graph {i}: total"
        assert np.array_equal(in_mst[a:b], k.in_mst), f"{name} graph {i}: edge set"


def test_batched_small_and_large(dev):
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(40, seed=7, n_lo=64, n_hi=40_000)
    graphs = [(int(b.vertex_offsets[g + 1] - b.vertex_offsets[g]),) + tuple(
        arr[b.edge_offsets[g]:b.edge_offsets[g + 1]] for arr in (b.src, b.dst, b.w)) for g in range(b.num_graphs)]
    assert any(x[0] > 8192 for x in graphs) and any(x[0] <= 8192 for x in graphs)
    check_batch(dev, graphs, "mixed_40")


def test_batched_degenerate_members(dev):
    graphs = []
    for name, n, s, d, w in gpu_cases.edge_cases():
        graphs.append((n, s, d, w))
    for g in gpu_cases.small_cases()[:6]:
        graphs.append((g.n, g.src, g.dst, g.w))
    t = gpu_cases.ties_multigraph(9000, 40_000, seed=3)  # above the one-workgroup size, ties
    graphs.append((t.n, t.src, t.dst, t.w))
    # an out-of-range id in one small and one large graph: only those graphs fail
    graphs.append((5, np.array([0, 7], np.int32), np.array([1, 2], np.int32), np.array([1, 2], np.uint32)))
    big = gpu_cases.ties_multigraph(10_000, 30_000, seed=4)
    bs = big.src.copy()
    bs[17] = 10_000
    graphs.append((big.n, bs, big.dst, big.w))
    check_batch(dev, graphs, "degenerate")


def test_batched_equals_single(dev):
    """Batched flags equal mst_solve on each graph alone (the per-graph path)."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(12, seed=11, n_lo=1000, n_hi=30_000)
    vo, eo = b.vertex_offsets, b.edge_offsets
    rc, in_mst, total, status = run_batched(dev, vo, eo, b.src, b.dst, b.w)
    assert rc == 0
    for g in range(b.num_graphs):
        one = b.graph(g)
        r = P.solve(one.n, torch.from_numpy(one.src).to(dev), torch.from_numpy(one.dst).to(dev),
                    torch.from_numpy(one.w).to(dev))
        assert r.status == status[g] and r.total == total[g]
        assert np.array_equal(r.in_mst.cpu().numpy(), in_mst[eo[g]:eo[g + 1]])


def test_batched_empty_and_args(dev):
    import paper_2005_06913_amd as P
    rc, _, _, _ = run_batched(dev, np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(0, np.int32),
                              np.zeros(0, np.int32), np.zeros(0, np.uint32))
    assert rc == 0
    lib = P.load_library()
    bad = np.array([0, 5, 3], np.int64)  # decreasing
    ok = np.array([0, 1, 2], np.int64)
    import ctypes
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.mst_solve_batched(2, ptr(bad), ptr(ok), None, None, None, None, None, None, None) == P.MSTX_ERR_INVALID_ARG
