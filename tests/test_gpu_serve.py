"""GPU serving: every result in the mix equals the oracle on that graph alone
and the GPU solve of it alone, bit-exact.

Three slots on three streams solve overlapping batches of requests of
uneven sizes (one-workgroup graphs and larger union-chunk graphs) that
arrive by a Poisson process.
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


def test_served_equals_alone(dev):
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    from paper_2005_06913_amd import serve
    b = G.batch(48, seed=21, n_lo=100, n_hi=60_000)
    reqs = [serve.Request(i, *(lambda g: (g.n, g.src, g.dst, g.w))(b.graph(i))) for i in range(b.num_graphs)]
    ex = serve.GpuExecutor(slots=3, device=dev)
    srv = serve.MstServer(ex, slots=3, hbm_budget_bytes=6 << 30).start()
    print("[case] served 48 requests, 3 slots", flush=True)
    serve.poisson_replay(srv, reqs, qps=3000.0, seed=22)
    srv.close()
    assert max(len(ids) for _, ids in srv.batches) > 1  # requests were batched
    for r in reqs:
        # in the mix == the oracle on that graph alone == the GPU on it alone
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status == 0, (r.rid, r.status, k.status)
        assert r.total == k.total, r.rid
        assert np.array_equal(r.in_mst, k.in_mst), r.rid
        alone = P.solve(r.n, torch.from_numpy(r.src).to(dev), torch.from_numpy(r.dst).to(dev),
                        torch.from_numpy(r.w).to(dev))
        assert alone.status == 0 and alone.total == k.total, r.rid
        assert np.array_equal(alone.in_mst.cpu().numpy(), k.in_mst), r.rid
    ex.release()


def test_plain_server(dev):
    from paper_2005_06913_amd import graphgen as G
    from paper_2005_06913_amd import serve
    b = G.batch(10, seed=23, n_lo=100, n_hi=20_000)
    reqs = [serve.Request(i, *(lambda g: (g.n, g.src, g.dst, g.w))(b.graph(i))) for i in range(b.num_graphs)]
    srv = serve.PlainServer(device=dev).start()
    serve.poisson_replay(srv, reqs, qps=1000.0, seed=24)
    srv.close()
    for r in reqs:
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status and r.total == k.total
        assert np.array_equal(r.in_mst, k.in_mst)
