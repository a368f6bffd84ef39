"""The CPU oracle against what the paper and mathematics fix (no GPU).

Each pin is described in ``tests/mst_pins.py``.  These tests establish that
the oracle can be trusted before the GPU path is compared with it.
"""

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import mst_pins
import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("pin", sorted(mst_pins.PINS))
def test_pin(orc, pin):
    mst_pins.PINS[pin](orc)


def test_matrix_tree_pins_brute_force():
    mst_pins.pin_matrix_tree()


def test_golden_fixtures_present():
    names = {f.name for f in mst_pins.all_fixtures()}
    assert "paper_fig_4comp.txt" in names
    assert len(names) >= 5


@st.composite
def small_multigraph(draw):
    n = draw(st.integers(1, 7))
    m = draw(st.integers(0, 11))
    src = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    dst = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    w = draw(st.lists(st.integers(0, 2**32 - 1) | st.integers(1, 3), min_size=m, max_size=m))
    return n, np.array(src, np.int32), np.array(dst, np.int32), np.array(w, np.uint32)


@settings(max_examples=300, deadline=None)
@given(small_multigraph())
def test_hypothesis_brute_force(g):
    n, src, dst, w = g
    orc = oracle.default()
    flags, total, _ = mst_pins.brute_force_msf(n, src, dst, w)
    k = orc.kruskal(n, src, dst, w)
    b = orc.boruvka(n, src, dst, w)
    assert np.array_equal(k.in_mst, flags)
    assert np.array_equal(b.in_mst, flags)
    assert k.total == total == b.total
    assert orc.check_mst(n, src, dst, w, flags, total) == 0


def test_boruvka_labels_are_min_ids(orc):
    """Final labels: the smallest vertex id of each connected component (BFS)."""
    from paper_2005_06913_amd import graphgen as G
    a = G.tree_plus_extra(50, 120, seed=1)
    b = G.tree_plus_extra(30, 60, seed=2)
    src = np.concatenate([a.src + 30, b.src]).astype(np.int32)  # second part holds ids 0..29
    dst = np.concatenate([a.dst + 30, b.dst]).astype(np.int32)
    w = np.concatenate([a.w, b.w + 1000]).astype(np.uint32)
    r = orc.boruvka(80, src, dst, w, labels=True)
    assert r.status == 0 or r.status == 1
    _, comp = mst_pins._components(80, src, dst)
    want = np.array([min(v for v in range(80) if comp[v] == comp[u]) for u in range(80)], np.int32)
    assert np.array_equal(r.labels, want)


@pytest.mark.slow
def test_planted_tree_full_size(orc):
    """n = 2^20, average degree 16: the MST is the planted tree, weight n(n-1)/2."""
    from paper_2005_06913_amd import graphgen as G
    g = G.planted_weights(G.workload("random_n1M_d16"))
    k = orc.kruskal(g.n, g.src, g.dst, g.w)
    assert k.status == 0
    assert k.total == g.n * (g.n - 1) // 2 == 549_755_289_600
    assert np.array_equal(k.in_mst, g.tree_mask.astype(np.uint8))
