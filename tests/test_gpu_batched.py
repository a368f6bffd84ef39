"""GPU parity of the batched solve: every graph of a batch against the oracle.

A batch mixes graphs solved by one workgroup each with everything in LDS
(n <= 8192 and the edges fit there too), graphs solved by one workgroup each
with the edges streamed every round (the other graphs of up to 16280 vertices
and 2^21 edges), graphs contracted round by round
by one workgroup to at most 16280 components and then finished like those (up
to 65536 vertices) and larger graphs solved as chunks of a disjoint union; the
middle classes are also forced onto the union path (``mid_limit(0)``) so both
stay covered.  Ties, self-loops, parallel edges,
isolated vertices, empty graphs and out-of-range ids are included.  Every
graph's edge flags, total and status must equal the oracle's on that graph
alone.
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


# the mid-size class on its own path, and forced onto the union path
MID_PATHS = {"mid": gpu_cases.MID_MAX, "union": 0}


def batch_graphs(b):
    return [(int(b.vertex_offsets[g + 1] - b.vertex_offsets[g]),) + tuple(
        arr[b.edge_offsets[g]:b.edge_offsets[g + 1]] for arr in (b.src, b.dst, b.w)) for g in range(b.num_graphs)]


@pytest.mark.parametrize("path", list(MID_PATHS))
def test_batched_small_and_large(dev, path):
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(40, seed=7, n_lo=64, n_hi=40_000)
    graphs = batch_graphs(b)
    assert any(x[0] > gpu_cases.SMALL_MAX for x in graphs) and any(x[0] <= gpu_cases.SMALL_MAX for x in graphs)
    with P.mid_limit(MID_PATHS[path]):
        check_batch(dev, graphs, f"mixed_40_{path}")


@pytest.mark.parametrize("path", list(MID_PATHS))
def test_batched_mid_boundaries(dev, path):
    """Graphs at the edges of every class: a small graph whose edges just fit in
    LDS and one with one edge more, 8193 and 16280 vertices (mid),
    16281, 32560, 32561 and 65536 (contracted by one to three rounds, one to
    four LDS windows of minima), 65537 (union), 2^21 edges exactly (mid,
    contracted) and 2^21 + 1 (union), path graphs whose first round joins
    everything (increasing weights) or only halves the components
    (alternating weights)."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    E = gpu_cases.MID_MAX_EDGES
    M = gpu_cases.MID_MAX
    n_alt = 2 * M - 7
    alt = np.where(np.arange(n_alt - 1) % 2 == 0, 1000, 1).astype(np.uint32) + np.arange(n_alt - 1, dtype=np.uint32)
    parts = [
        G.tree_plus_extra(gpu_cases.SMALL_MAX + 1, 6 * gpu_cases.SMALL_MAX, seed=41),
        G.tree_plus_extra(M, 8 * M, seed=42),
        G.tree_plus_extra(M + 1, 3 * M, seed=43),
        G.tree_plus_extra(2 * M, 4 * M, seed=46),
        G.tree_plus_extra(2 * M + 1, 5 * M, seed=47),
        G.tree_plus_extra(gpu_cases.PRE_MAX, 6 * M, seed=48),
        G.tree_plus_extra(gpu_cases.PRE_MAX + 1, 6 * M, seed=49),
        G.tree_plus_extra(12_000, E, seed=44),
        G.tree_plus_extra(40_000, E, seed=50),
        G.tree_plus_extra(12_000, E + 1, seed=45),
        G.path_graph(M - 5),
        G.path_graph(3 * M),
        G.path_graph(n_alt, alt),
        # n = 4096: 16 B per vertex and 12 B per edge fill the 162816 B of LDS
        # at 8106 edges (the small solve keeps them) and overflow at 8107
        # (the mid-size solve streams them)
        G.tree_plus_extra(4096, 8106, seed=51),
        G.tree_plus_extra(4096, 8107, seed=52),
    ]
    graphs = [(g.n, g.src, g.dst, g.w) for g in parts]
    with P.mid_limit(MID_PATHS[path]):
        check_batch(dev, graphs, f"mid_boundaries_{path}")


def test_batched_many_contracted(dev):
    """Many graphs of the contracted class (more workgroups than the chip holds
    at a time; also more vertices than one union chunk holds, for the union
    path), several average degrees, against the oracle."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(140, seed=23, n_lo=gpu_cases.MID_MAX + 1, n_hi=gpu_cases.PRE_MAX, d_lo=2.0, d_hi=12.0)
    assert sum(int(b.vertex_offsets[g + 1] - b.vertex_offsets[g]) for g in range(b.num_graphs)) > 1 << 22
    check_batch(dev, batch_graphs(b), "many_contracted_140")
    with P.mid_limit(0):
        check_batch(dev, batch_graphs(b), "many_contracted_140_union")


def test_batched_many_mid(dev):
    """Many mid-size graphs at once (more workgroups than the chip holds at a
    time), several average degrees, against the oracle."""
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(600, seed=19, n_lo=gpu_cases.SMALL_MAX + 1, n_hi=gpu_cases.MID_MAX, d_lo=2.0, d_hi=24.0)
    check_batch(dev, batch_graphs(b), "many_mid_600")


@pytest.mark.parametrize("path", list(MID_PATHS))
def test_batched_degenerate_members(dev, path):
    import paper_2005_06913_amd as P
    with P.mid_limit(MID_PATHS[path]):
        degenerate_members(dev, path)


def degenerate_members(dev, path):
    from paper_2005_06913_amd import graphgen as G
    graphs = []
    for name, n, s, d, w in gpu_cases.edge_cases():
        graphs.append((n, s, d, w))
    for g in gpu_cases.small_cases()[:6]:
        graphs.append((g.n, g.src, g.dst, g.w))
    t = gpu_cases.ties_multigraph(9000, 40_000, seed=3)  # above the all-LDS one-workgroup size, ties
    graphs.append((t.n, t.src, t.dst, t.w))
    # an out-of-range id in one small and one large graph: only those graphs fail
    graphs.append((5, np.array([0, 7], np.int32), np.array([1, 2], np.int32), np.array([1, 2], np.uint32)))
    big = gpu_cases.ties_multigraph(10_000, 30_000, seed=4)
    bs = big.src.copy()
    bs[17] = 10_000
    graphs.append((big.n, bs, big.dst, big.w))
    # the contracted classes: ties and an out-of-range id; isolated vertices
    # (half the graph has no edge); a star, joined by its first round
    for n, m, seed in ((25_000, 90_000, 5), (50_000, 150_000, 6)):
        t = gpu_cases.ties_multigraph(n, m, seed=seed)
        graphs.append((t.n, t.src, t.dst, t.w))
        ts = t.src.copy()
        ts[m // 2] = -3
        graphs.append((t.n, ts, t.dst, t.w))
    # few vertices but more edges than one workgroup streams (the union path)
    dense = gpu_cases.ties_multigraph(2000, gpu_cases.MID_MAX_EDGES, seed=9)
    graphs.append((dense.n, dense.src, dense.dst, dense.w))
    half = G.tree_plus_extra(20_000, 70_000, seed=7)
    graphs.append((40_000, half.src, half.dst, half.w))
    star = G.star_graph(30_000, seed=8)
    graphs.append((star.n, star.src, star.dst, star.w))
    # no edges at all, in every class: small, mid-size, contracted, union
    z32, zw = np.zeros(0, np.int32), np.zeros(0, np.uint32)
    for n in (4000, 12_000, 20_000, gpu_cases.PRE_MAX, gpu_cases.PRE_MAX + 1):
        graphs.append((n, z32, z32, zw))
    check_batch(dev, graphs, f"degenerate_{path}")


@pytest.mark.timeout(600)
def test_batched_4096_full_vs_oracle(dev):
    """The full batched workload (4096 graphs, n log-uniform in [64, 65536],
    average degree uniform in [4, 32], seed 5; about 3.3e8 edges): every
    graph's edge flags, total and status against Kruskal on that graph alone
    (host threads share the oracle calls)."""
    import concurrent.futures as cf
    import os

    from paper_2005_06913_amd import graphgen as G
    print("[case] batched_4096 seed 5, full size", flush=True)
    b = G.batch(4096, seed=5)
    vo, eo = b.vertex_offsets, b.edge_offsets
    rc, in_mst, total, status = run_batched(dev, vo, eo, b.src, b.dst, b.w)
    assert rc == 0
    print("[case] batched_4096: GPU done, oracle per graph", flush=True)

    def check(g):
        x = b.graph(g)
        k = oracle.kruskal(x.n, x.src, x.dst, x.w)
        a, c = eo[g], eo[g + 1]
        return (int(status[g]) == k.status and int(total[g]) == k.total
                and bool(np.array_equal(in_mst[a:c], k.in_mst)))

    oracle.default()  # built and loaded once, before the threads share it
    workers = min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        ok = list(ex.map(check, range(b.num_graphs)))
    bad = [g for g, x in enumerate(ok) if not x]
    assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:8]}"


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


def test_batched_plan_replays(dev):
    """A batch planned once and captured as a HIP graph (mst_batched_plan_*):
    three replays, with the weights rewritten and other solves run on the
    stream between them; every replay equals mst_solve_batched on the same
    inputs, and the oracle on every graph."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    b = G.batch(40, seed=61, n_lo=64, n_hi=60_000)
    vo, eo = b.vertex_offsets, b.edge_offsets
    m, Gn = int(eo[-1]), b.num_graphs
    src, dst = torch.from_numpy(b.src).to(dev), torch.from_numpy(b.dst).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    flags = torch.full((m,), 7, dtype=torch.uint8, device=dev)
    tot = torch.full((Gn,), 5, dtype=torch.int64, device=dev).view(torch.uint64)
    st = torch.full((Gn,), 9, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    print("[case] batched plan: 40 graphs, capture", flush=True)
    rc, plan = P.mst_batched_plan_create(vo, eo, src, dst, w, flags, tot, st, stream)
    assert rc == 0 and plan is not None
    other = G.tree_plus_extra(50_000, 300_000, seed=63)
    os_, od, ow = (torch.from_numpy(a).to(dev) for a in (other.src, other.dst, other.w))
    rng = np.random.default_rng(64)
    try:
        for rep in range(3):
            wn = b.w if rep == 0 else rng.permutation(b.w).astype(np.uint32)
            w.copy_(torch.from_numpy(wn))
            assert P.solve(other.n, os_, od, ow).status == 0  # eager work between replays
            print(f"[case] batched plan: replay {rep}", flush=True)
            assert P.mst_batched_plan_run(plan, stream) == 0
            torch.cuda.synchronize()
            got_f, got_t = flags.cpu().numpy(), tot.view(torch.int64).cpu().numpy()
            got_s = st.cpu().numpy()
            rc2, ref_f, ref_t, ref_s = run_batched(dev, vo, eo, b.src, b.dst, wn)
            assert rc2 == 0
            assert np.array_equal(got_f, ref_f) and np.array_equal(got_t, ref_t) and np.array_equal(got_s, ref_s)
            for g in range(Gn):
                a, c = int(eo[g]), int(eo[g + 1])
                k = oracle.kruskal(int(vo[g + 1] - vo[g]), b.src[a:c], b.dst[a:c], wn[a:c])
                assert got_s[g] == k.status and int(got_t[g]) == k.total, (rep, g)
                assert np.array_equal(got_f[a:c], k.in_mst), (rep, g)
    finally:
        torch.cuda.synchronize()
        assert P.mst_batched_plan_destroy(plan) == 0


def test_batched_plan_refuses_union_graphs(dev):
    """A batch with a graph that needs the union rounds cannot be captured."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    big = G.tree_plus_extra(70_000, 200_000, seed=65)
    small = G.tree_plus_extra(1000, 5000, seed=66)
    vo, eo, s, d, w = concat([(big.n, big.src, big.dst, big.w), (small.n, small.src, small.dst, small.w)])
    m = int(eo[-1])
    args = [torch.from_numpy(a).to(dev) for a in (s, d, w)]
    flags = torch.empty(m, dtype=torch.uint8, device=dev)
    tot = torch.empty(2, dtype=torch.uint64, device=dev)
    st = torch.empty(2, dtype=torch.int32, device=dev)
    rc, plan = P.mst_batched_plan_create(vo, eo, *args, flags, tot, st)
    assert rc == P.MSTX_ERR_INVALID_ARG and plan is None
