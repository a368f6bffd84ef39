"""The autotuner on the GPU: tuning a single graph and a batch stores settings
under their classes, every candidate setting gives byte-identical results
(the tuner raises otherwise), and the tuned settings applied through the
cache solve the graph exactly as the oracle does."""

import numpy as np
import pytest

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


def test_tune_single_and_apply(dev, tmp_path):
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import autotune as A
    path = str(tmp_path / "tuning.json")
    g = G.tree_plus_extra(40_000, 320_001, seed=51, name="tune_single")
    s, d, w = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.w))
    before = A.defaults(list(A.SINGLE_KNOBS))
    print(f"[case] autotune single n={g.n} m={g.m}", flush=True)
    entry = A.tune_single(g.n, s, d, w, reps=2, passes=1, path=path)
    assert A.defaults(list(A.SINGLE_KNOBS)) == before  # knobs restored
    assert entry["candidates"] >= 2 and entry["ms"] > 0
    assert A.lookup(A.single_class(g.n, g.m), path) == entry["knobs"]
    k = oracle.kruskal(g.n, g.src, g.dst, g.w)
    with A.tuned_single(g.n, g.m, path) as applied:
        assert applied == entry["knobs"]
        res = P.solve(g.n, s, d, w)
    torch.cuda.synchronize()
    assert res.status == k.status and res.total == k.total
    assert np.array_equal(res.in_mst.cpu().numpy(), k.in_mst)


def test_tune_batched(dev, tmp_path):
    from paper_2005_06913_amd import autotune as A
    path = str(tmp_path / "tuning.json")
    b = G.batch(48, seed=52, n_lo=64, n_hi=40_000)
    s, d, w = (torch.from_numpy(a).to(dev) for a in (b.src, b.dst, b.w))
    print(f"[case] autotune batched graphs={b.num_graphs} m={int(b.edge_offsets[-1])}", flush=True)
    entry = A.tune_batched(b.vertex_offsets, b.edge_offsets, s, d, w, reps=2, passes=1, path=path)
    assert A.lookup(A.batch_class(b.num_graphs, int(b.edge_offsets[-1])), path) == entry["knobs"]
