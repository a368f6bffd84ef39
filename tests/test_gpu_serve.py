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


def test_stepwise_solve_with_work_between_rounds(dev):
    """mst_solve_begin / advance / end: the same bytes, total and round
    statistics as mst_solve, with a batched call run on the same stream
    between two rounds (its results exact too); a second stepwise solve on the
    same stream is refused while one is open."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    g = G.tree_plus_extra(300_000, 2_400_001, seed=25, name="stepwise")
    s, d, w = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.w))
    stream = torch.cuda.current_stream()
    want = P.solve(g.n, s, d, w)
    want_stats = P.mst_last_round_stats()
    in_mst = torch.full((g.m,), 9, dtype=torch.uint8, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    print(f"[case] stepwise n={g.n} m={g.m}", flush=True)
    st, h = P.mst_solve_begin(g.n, s, d, w, in_mst, total, stream)
    assert st == 0 and h is not None
    st2, h2 = P.mst_solve_begin(g.n, s, d, w, in_mst, total, stream)
    assert st2 == P.MSTX_ERR_INVALID_ARG and h2 is None
    b = G.batch(6, seed=26, n_lo=100, n_hi=5000)
    bs, bd, bw = (torch.from_numpy(a).to(dev) for a in (b.src, b.dst, b.w))
    bm = torch.empty(int(b.edge_offsets[-1]), dtype=torch.uint8, device=dev)
    bt = torch.empty(b.num_graphs, dtype=torch.uint64, device=dev)
    bst = torch.empty(b.num_graphs, dtype=torch.int32, device=dev)
    steps, batched = 0, False
    while not P.mst_solve_advance(h):
        steps += 1
        if not batched:
            assert P.mst_solve_batched(b.vertex_offsets, b.edge_offsets, bs, bd, bw, bm, bt, bst, stream) == 0
            batched = True
        elif steps % 2 == 0 and P.mst_solve_wait_round(h):  # one round at a time, waiting
            break
    assert P.mst_solve_end(h) == want.status == 0
    torch.cuda.synchronize()
    assert int(total.view(torch.int64).item()) == want.total
    assert torch.equal(in_mst, want.in_mst)
    assert np.array_equal(P.mst_last_round_stats(), want_stats)
    flags, tots = bm.cpu().numpy(), bt.view(torch.int64).cpu().numpy()
    for i in range(b.num_graphs):
        x = b.graph(i)
        k = oracle.kruskal(x.n, x.src, x.dst, x.w)
        assert int(bst[i]) == k.status and int(tots[i]) == k.total
        assert np.array_equal(flags[b.edge_offsets[i]:b.edge_offsets[i + 1]], k.in_mst)


def test_round_granular_admission_gpu(dev):
    """One slot: small requests that arrive while a large one is solved round by
    round run between its rounds and finish before it; every result equals the
    oracle's."""
    import time

    from paper_2005_06913_amd import graphgen as G
    from paper_2005_06913_amd import serve
    big_g = G.tree_plus_extra(1 << 20, 1 << 23, seed=27)
    big = serve.Request(1000, big_g.n, big_g.src, big_g.dst, big_g.w)
    b = G.batch(24, seed=28, n_lo=100, n_hi=4000)
    small = [serve.Request(i, *(lambda x: (x.n, x.src, x.dst, x.w))(b.graph(i))) for i in range(b.num_graphs)]
    ex = serve.GpuExecutor(slots=1, device=dev)
    srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=8 << 30, solo_edges=1 << 19).start()
    print("[case] round-granular admission, 1 slot", flush=True)
    srv.submit(big)
    time.sleep(0.0005)
    for r in small:
        srv.submit(r)
    for r in small + [big]:
        r.done.wait()
    srv.close()
    for r in small + [big]:
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status == 0, (r.rid, r.status)
        assert r.total == k.total and np.array_equal(r.in_mst, k.in_mst), r.rid
    if srv.interleaved:  # the large solve was still running when the small ones came
        assert all(big_id == 1000 for _, big_id, _ in srv.interleaved)
        ran = {rid for _, _, ids in srv.interleaved for rid in ids}
        assert all(next(x for x in small if x.rid == rid).done_at < big.done_at for rid in ran)
    ex.release()


def test_resident_requests(dev):
    """Requests whose graphs are already device tensors: small ones batched by
    one concatenation inside HBM, a large one solved round by round; flags stay
    on the device; every result equals the oracle's, and the plain server's."""
    from paper_2005_06913_amd import graphgen as G
    from paper_2005_06913_amd import serve
    b = G.batch(20, seed=29, n_lo=100, n_hi=8000)
    graphs = [b.graph(i) for i in range(b.num_graphs)] + [G.tree_plus_extra(200_000, 1_200_000, seed=30)]

    def requests():
        return [serve.Request(i, g.n, *(torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.w)))
                for i, g in enumerate(graphs)]

    reqs = requests()
    assert all(r.resident for r in reqs)
    ex = serve.GpuExecutor(slots=2, device=dev)
    srv = serve.MstServer(ex, slots=2, hbm_budget_bytes=4 << 30, solo_edges=1 << 19).start()
    print("[case] resident requests, 2 slots", flush=True)
    serve.poisson_replay(srv, reqs, qps=5000.0, seed=31)
    srv.close()
    plain = requests()
    psrv = serve.PlainServer(device=dev).start()
    serve.poisson_replay(psrv, plain, qps=5000.0, seed=32)
    psrv.close()
    for r, p, g in zip(reqs, plain, graphs):
        assert hasattr(r.in_mst, "is_cuda") and r.in_mst.is_cuda
        k = oracle.kruskal(g.n, g.src, g.dst, g.w)
        assert r.status == p.status == k.status == 0, r.rid
        assert r.total == p.total == k.total, r.rid
        assert np.array_equal(r.flags(), k.in_mst) and np.array_equal(p.flags(), k.in_mst), r.rid
    assert any(len(ids) > 1 for _, ids in srv.batches)
    ex.release()


@pytest.mark.parametrize("server", ["batched", "solo", "plain"])
def test_resident_request_waits_for_its_producer(dev, server):
    """A resident request whose arrays are still being written on the
    submitting thread's stream (behind a 20-ms spin) is solved only after
    them: its result equals the oracle's.  Small requests go through the
    batched call, large ones through the round-by-round solve."""
    from paper_2005_06913_amd import graphgen as G
    from paper_2005_06913_amd import serve
    n, m = (20_000, 120_000) if server != "solo" else (300_000, 2_400_000)
    g = G.tree_plus_extra(n, m, seed=34)
    staged = [torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.w)]
    arrays = [torch.zeros_like(t) for t in staged]
    torch.cuda.synchronize()
    if server == "plain":
        srv = serve.PlainServer(device=dev).start()
        ex = None
    else:
        ex = serve.GpuExecutor(slots=1, device=dev)
        srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=4 << 30, solo_edges=1 << 19).start()
    producer = torch.cuda.Stream(device=dev)
    print(f"[case] resident request behind its producer, {server}", flush=True)
    with torch.cuda.stream(producer):
        torch.cuda._sleep(50_000_000)  # a bounded spin, then the arrays are written
        for a, t in zip(arrays, staged):
            a.copy_(t)
        r = srv.submit(serve.Request(0, g.n, *arrays))
    r.done.wait()
    srv.close()
    k = oracle.kruskal(g.n, g.src, g.dst, g.w)
    assert r.status == k.status == 0, r.status
    assert r.total == k.total
    assert np.array_equal(r.flags(), k.in_mst)
    if ex is not None:
        ex.release()
