"""The device-side input generator's claim, checked on the host with the
oracle: built with torch on the CPU at small sizes, the planted tree is the
minimum spanning tree (the last n - 1 edges, weight n(n - 1)/2)."""

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,m_extra,seed", [(2, 0, 1), (2, 5, 2), (1000, 20_000, 3), (4097, 100_000, 4)])
def test_planted_on_device_is_its_own_mst(n, m_extra, seed):
    from paper_2005_06913_amd import graphgen as G
    src, dst, w = G.planted_on_device(n, m_extra, seed=seed, device="cpu", chunk=7_000)
    s, d, ww = src.numpy(), dst.numpy(), w.numpy().view(np.uint32)
    assert s.shape[0] == m_extra + n - 1
    assert np.all(s != d) and s.min() >= 0 and max(s.max(), d.max()) < n
    assert np.array_equal(np.sort(ww[m_extra:]), np.arange(1, n, dtype=np.uint32))
    k = oracle.kruskal(n, s, d, ww)
    assert k.status == 0 and k.total == n * (n - 1) // 2
    assert not k.in_mst[:m_extra].any() and k.in_mst[m_extra:].all()
