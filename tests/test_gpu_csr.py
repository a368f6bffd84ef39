"""GPU: the edge list of a symmetric CSR adjacency (mst_csr_to_edges).

The expected edge list is written out with numpy from the same CSR arrays (each
arc u -> v with u < v, row-major arc order); the conversion must equal it
exactly, and the solve of the converted graph must equal the oracle on it.
Invalid adjacencies (a column out of range, an inconsistent row_ptr) must be
reported, not read.
"""

import numpy as np
import pytest

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


def symmetric_csr(n, src, dst, w, seed, extra_loops=0):
    """Both arcs of every edge, rows in vertex order, arcs shuffled inside each row."""
    rng = np.random.default_rng(seed)
    u = np.concatenate([src, dst]).astype(np.int64)
    v = np.concatenate([dst, src]).astype(np.int64)
    ww = np.concatenate([w, w]).astype(np.uint32)
    if extra_loops:
        loops = rng.integers(0, n, extra_loops)
        u = np.concatenate([u, loops])
        v = np.concatenate([v, loops])
        ww = np.concatenate([ww, rng.integers(1, 1000, extra_loops).astype(np.uint32)])
    order = np.lexsort((rng.random(len(u)), u))
    u, v, ww = u[order], v[order], ww[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, u + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, v.astype(np.int32), ww


def expected_edges(n, row_ptr, col):
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    keep = col.astype(np.int64) > rows
    return rows[keep].astype(np.int32), col[keep], keep


def convert(dev, n, row_ptr, col, w):
    import paper_2005_06913_amd as P
    return P.mst_csr_to_edges(n, torch.from_numpy(row_ptr).to(dev), torch.from_numpy(col).to(dev),
                              torch.from_numpy(w).to(dev))


@pytest.mark.parametrize("n,m,loops,seed", [(5000, 40_000, 0, 1), (1 << 18, 1 << 21, 777, 2), (3, 2, 5, 3)])
def test_csr_conversion_and_solve(dev, n, m, loops, seed):
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    print(f"[case] csr n={n} m={m} loops={loops}", flush=True)
    g = G.tree_plus_extra(n, m, seed=seed)
    row_ptr, col, w = symmetric_csr(n, g.src, g.dst, g.w, seed, extra_loops=loops)
    s, d, ww = convert(dev, n, row_ptr, col, w)
    es, ed, keep = expected_edges(n, row_ptr, col)
    assert np.array_equal(s.cpu().numpy(), es)
    assert np.array_equal(d.cpu().numpy(), ed)
    assert np.array_equal(ww.cpu().numpy(), w[keep])
    # the converted graph is the original one, edges in another order
    r = P.solve(n, s, d, ww)
    k = oracle.kruskal(n, es, ed, w[keep])
    assert r.status == k.status and r.total == k.total
    assert np.array_equal(r.in_mst.cpu().numpy(), k.in_mst)
    assert r.total == oracle.kruskal(g.n, g.src, g.dst, g.w).total


def test_csr_empty_rows_and_one_sided(dev):
    """Isolated vertices (empty rows), and an adjacency holding only the arcs
    u -> v with u < v (nothing mirrored): all of them are kept."""
    n = 9
    row_ptr = np.array([0, 2, 2, 3, 3, 3, 5, 5, 5, 5], np.int64)
    col = np.array([4, 1, 8, 7, 8], np.int32)
    w = np.array([5, 3, 9, 1, 2], np.uint32)
    s, d, ww = convert(dev, n, row_ptr, col, w)
    assert s.cpu().tolist() == [0, 0, 2, 5, 5]
    assert d.cpu().tolist() == [4, 1, 8, 7, 8]
    assert ww.cpu().tolist() == [5, 3, 9, 1, 2]


def test_csr_degenerate_and_errors(dev):
    import paper_2005_06913_amd as P
    s, d, ww = convert(dev, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint32))
    assert s.numel() == 0
    s, d, ww = convert(dev, 4, np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint32))
    assert s.numel() == 0
    rp = np.array([0, 1, 2], np.int64)
    with pytest.raises(P.MstxError) as e:  # a column outside [0, n)
        convert(dev, 2, rp, np.array([1, 2], np.int32), np.array([1, 1], np.uint32))
    assert e.value.status == P.MSTX_ERR_VERTEX_RANGE
    with pytest.raises(P.MstxError) as e:  # decreasing row_ptr
        convert(dev, 2, np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32), np.array([1, 1], np.uint32))
    assert e.value.status == P.MSTX_ERR_INVALID_ARG
    with pytest.raises(P.MstxError) as e:  # row_ptr[n] != nnz
        convert(dev, 2, np.array([0, 1, 1], np.int64), np.array([1, 0], np.int32), np.array([1, 1], np.uint32))
    assert e.value.status == P.MSTX_ERR_INVALID_ARG
