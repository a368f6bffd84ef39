"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer graph work, so the bar is bit-exact: the in_mst byte array, the
uint64 total weight, the status, and the per-round statistics (components,
live edges, edges added) must equal the oracle's.  Where the graph is
connected the oracle's sequential Boruvka round counts are comparable one to
one: both remove exactly the internal edges and add one tree edge per
distinct selected minimum.  A solve that ends with the dense finish stops its
rows at that round, whose added edges are those of the oracle's remaining
rounds together (gpu_cases.stats_consistent); so does a solve that ends with
the sparse finish (the lightest edge of every component pair, finished in
one workgroup).  The small cases run with the dense finish off, at its
default limit and at limits that make it start in earlier or later rounds,
with the sparse finish at its default and off.
"""

import functools

import numpy as np
import pytest

import gpu_cases
import mst_pins
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


def to_dev(dev, src, dst, w):
    return (torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(dst, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(w, np.uint32)).to(dev))


def gpu_solve(dev, n, src, dst, w, limit=gpu_cases.DENSE_MAX, small=gpu_cases.SMALL_MAX, tail=gpu_cases.TAIL_MAX,
              bucket=gpu_cases.BUCKET_MAX, sparse=gpu_cases.SPARSE_DEFAULT):
    import paper_2005_06913_amd as P
    s, d, ww = to_dev(dev, src, dst, w)
    m = len(src)
    in_mst = torch.full((m,), 7, dtype=torch.uint8, device=dev)  # garbage: must be overwritten
    total = torch.full((1,), 12345, dtype=torch.int64, device=dev).view(torch.uint64)
    with P.dense_limit(limit), P.small_limit(small), P.tail_limit(tail), P.bucket_limit(bucket), \
            P.sparse_limit(sparse):
        st = P.mst_solve(n, s, d, ww, in_mst, total)
    torch.cuda.synchronize()
    stats = P.mst_last_round_stats()
    return st, in_mst.cpu().numpy(), int(total.view(torch.int64).cpu().item()), stats


def finish_limit(limit, sparse):
    """Largest component count at which a finish may end the solve."""
    return max(limit, gpu_cases.SPARSE_MAX) if sparse else limit


def check_against_oracle(dev, name, n, src, dst, w, stats=True, limit=gpu_cases.DENSE_MAX,
                         small=gpu_cases.SMALL_MAX, tail=gpu_cases.TAIL_MAX, bucket=gpu_cases.BUCKET_MAX,
                         sparse=gpu_cases.SPARSE_DEFAULT):
    print(f"[case] {name} n={n} m={len(src)} dense_limit={limit} small_limit={small} tail_limit={tail} "
          f"bucket_limit={bucket} sparse_limit={sparse}", flush=True)
    st, in_mst, total, gstats = gpu_solve(dev, n, src, dst, w, limit, small, tail, bucket, sparse)
    k = oracle.kruskal(n, src, dst, w)
    assert st == k.status, f"{name}: status {st} != oracle {k.status}"
    assert total == k.total, f"{name}: total {total} != oracle {k.total}"
    diff = np.flatnonzero(in_mst != k.in_mst)
    assert diff.size == 0, f"{name}: {diff.size} edges differ, first {diff[:8]}"
    if stats and k.status == 0 and n > 1:
        b = oracle.boruvka(n, src, dst, w)
        assert gpu_cases.stats_consistent(gstats, b.stats, finish_limit(limit, sparse)), \
            f"{name}: round stats\n{gstats}\n!~\n{b.stats}"
        if limit == 0 and sparse == 0:
            assert np.array_equal(gstats, b.stats)
    return gstats


# -------------------------------------------------------- first kernel (S1)

@pytest.mark.parametrize("idx", range(len(gpu_cases.small_cases())))
def test_min_edge_keys(dev, idx):
    import paper_2005_06913_amd as P
    g = gpu_cases.small_cases()[idx]
    print(f"[case] min-edge {g.name}", flush=True)
    s, d, w = to_dev(dev, g.src, g.dst, g.w)
    out = torch.zeros(g.n, dtype=torch.int64, device=dev).view(torch.uint64)
    assert P.mst_select_min_edges(g.n, s, d, w, out) == 0
    st, want = oracle.min_edge_keys(g.n, g.src, g.dst, g.w)
    assert st == 0
    got = out.view(torch.int64).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("idx", [i for i, g in enumerate(gpu_cases.small_cases()) if g.n > gpu_cases.LDS_SLOTS])
def test_min_edge_keys_global_mode(dev, idx):
    """Round-0 minima by filtered global atomics (bucket mode off) on every case
    above the LDS range."""
    import paper_2005_06913_amd as P
    g = gpu_cases.small_cases()[idx]
    print(f"[case] min-edge global {g.name}", flush=True)
    s, d, w = to_dev(dev, g.src, g.dst, g.w)
    out = torch.zeros(g.n, dtype=torch.int64, device=dev).view(torch.uint64)
    with P.bucket_limit(0):
        assert P.mst_select_min_edges(g.n, s, d, w, out) == 0
    st, want = oracle.min_edge_keys(g.n, g.src, g.dst, g.w)
    assert st == 0
    assert np.array_equal(out.view(torch.int64).cpu().numpy().view(np.uint64), want)


def test_min_edge_keys_golden(dev):
    import paper_2005_06913_amd as P
    for fx in mst_pins.all_fixtures():
        if not fx.minedge:
            continue
        s, d, w = to_dev(dev, fx.src, fx.dst, fx.w)
        out = torch.zeros(fx.n, dtype=torch.int64, device=dev).view(torch.uint64)
        assert P.mst_select_min_edges(fx.n, s, d, w, out) == 0
        got = out.view(torch.int64).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, mst_pins.expected_min_keys(fx)), fx.name


# ------------------------------------------------------------- full solve

# (dense-finish limit, small-graph limit, round-tail limit, sparse-finish
# limit): the defaults (graphs of at most 8192 vertices take the
# one-workgroup path), and the per-round kernel chain with the dense finish at
# its default, off, and starting earlier or later, with late rounds closed in
# one workgroup or by the grid-wide hook .. relabel kernels, with the sparse
# finish tried (the default) or not, and tried whatever the live edges
D, S, T, SP = gpu_cases.DENSE_MAX, gpu_cases.SMALL_MAX, gpu_cases.TAIL_MAX, gpu_cases.SPARSE_DEFAULT
ANY = (1 << 31) - 1
PATHS = [(D, S, T, SP), (D, 0, T, SP), (D, 0, 0, SP), (0, 0, T, SP), (0, 0, 0, SP), (0, 0, T, 0), (0, 0, 0, 0),
         (D, 0, T, 0), (2, 0, T, SP), (9, 0, 0, SP), (64, 0, T, SP), (64, 0, 0, SP), (0, 0, T, ANY), (D, 0, 0, ANY)]
PATH_IDS = [f"dense{a}-small{b}-tail{c}-sparse{d}" for a, b, c, d in PATHS]
FEW_PATHS = [(D, S, T, SP), (D, 0, T, SP), (0, 0, T, 0), (0, 0, 0, SP), (D, 0, T, ANY)]
FEW_IDS = [f"dense{a}-small{b}-tail{c}-sparse{d}" for a, b, c, d in FEW_PATHS]


@pytest.mark.parametrize("limit,small,tail,sparse", PATHS, ids=PATH_IDS)
@pytest.mark.parametrize("idx", range(len(gpu_cases.small_cases())))
def test_solve_small(dev, idx, limit, small, tail, sparse):
    g = gpu_cases.small_cases()[idx]
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, limit=limit, small=small, tail=tail, sparse=sparse)


# GLOBAL minima mode (bucket mode off): every round above the LDS range takes
# filtered 64-bit atomic minima in device memory
GLOBAL_CASES = [i for i, g in enumerate(gpu_cases.small_cases()) if g.n > gpu_cases.LDS_SLOTS]


@pytest.mark.parametrize("limit,small,tail,sparse", FEW_PATHS[1:], ids=FEW_IDS[1:])
@pytest.mark.parametrize("idx", GLOBAL_CASES)
def test_solve_global_mode(dev, idx, limit, small, tail, sparse):
    g = gpu_cases.small_cases()[idx]
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, limit=limit, small=small, tail=tail, bucket=0,
                         sparse=sparse)


def test_dense_finish_ends_early(dev):
    """The dense finish replaces the oracle's last rounds (n=1000, m=8000: a
    few hundred components after round 0, a few dozen after round 1)."""
    g = gpu_cases.small_cases()[0]
    gstats = check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, small=0)
    b = oracle.boruvka(g.n, g.src, g.dst, g.w)
    assert len(gstats) < len(b.stats), (gstats, b.stats)
    # a graph of at most 200 vertices is solved by the dense finish in round 0
    k64 = gpu_cases.small_cases()[7]
    assert k64.n == 64
    gstats = check_against_oracle(dev, k64.name, k64.n, k64.src, k64.dst, k64.w, small=0)
    assert len(gstats) == 1 and gstats[0][2] == 63


def test_sparse_finish_ends_early(dev):
    """A grid's late rounds join few component pairs: the sparse finish ends the
    solve before the oracle's last round (dense finish off), with the rows
    consistent; with it off the rows equal the oracle's."""
    g = next(x for x in gpu_cases.small_cases() if x.name == "grid_256x256")
    b = oracle.boruvka(g.n, g.src, g.dst, g.w)
    on = check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, limit=0, small=0, tail=0)
    assert len(on) < len(b.stats), (on, b.stats)
    assert int(on[-1][0]) <= gpu_cases.SPARSE_MAX and len(on) >= 2
    off = check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, limit=0, small=0, tail=0, sparse=0)
    assert np.array_equal(off, b.stats)


def test_small_path_matches_chain(dev):
    """The one-workgroup path and the per-round chain give the same bytes and the
    oracle's round statistics exactly (the small path has no dense finish)."""
    for g in gpu_cases.small_cases():
        if g.n > gpu_cases.SMALL_MAX or len(g.src) > (1 << 17):
            continue
        a = gpu_solve(dev, g.n, g.src, g.dst, g.w, small=gpu_cases.SMALL_MAX)
        c = gpu_solve(dev, g.n, g.src, g.dst, g.w, limit=0, small=0, tail=0, sparse=0)
        t = gpu_solve(dev, g.n, g.src, g.dst, g.w, limit=0, small=0, sparse=0)
        for x in (a, t):
            assert x[0] == c[0] and x[2] == c[2] and np.array_equal(x[1], c[1]), g.name
            assert np.array_equal(x[3], c[3]), g.name
        if a[0] == 0:
            assert np.array_equal(a[3], oracle.boruvka(g.n, g.src, g.dst, g.w).stats), g.name


@pytest.mark.parametrize("limit,small,tail,sparse", FEW_PATHS, ids=FEW_IDS)
def test_solve_golden(dev, limit, small, tail, sparse):
    for fx in mst_pins.all_fixtures():
        st, in_mst, total, stats = gpu_solve(dev, fx.n, fx.src, fx.dst, fx.w, limit, small, tail, sparse=sparse)
        assert st == fx.status, fx.name
        assert total == fx.total, fx.name
        assert np.array_equal(in_mst, fx.in_mst), fx.name
        if fx.status == 0:
            assert gpu_cases.stats_consistent(stats, fx.rounds, finish_limit(limit, sparse)), fx.name
            if limit == 0 and sparse == 0:
                assert [tuple(r) for r in stats.tolist()] == fx.rounds, fx.name


@pytest.mark.parametrize("limit,small,tail,sparse", FEW_PATHS, ids=FEW_IDS)
@pytest.mark.parametrize("case", gpu_cases.edge_cases(), ids=[c[0] for c in gpu_cases.edge_cases()])
def test_solve_edge_cases(dev, case, limit, small, tail, sparse):
    name, n, src, dst, w = case
    check_against_oracle(dev, name, n, src, dst, w, stats=False, limit=limit, small=small, tail=tail, sparse=sparse)


def test_vertex_range_error(dev):
    import paper_2005_06913_amd as P
    for bad_src in (5, -1, 1 << 30):
        src = np.array([0, 1, bad_src], np.int32)
        dst = np.array([1, 2, 0], np.int32)
        w = np.array([1, 2, 3], np.uint32)
        for small in (gpu_cases.SMALL_MAX, 0):
            st, _, _, _ = gpu_solve(dev, 5, src, dst, w, small=small)
            assert st == P.MSTX_ERR_VERTEX_RANGE
        s, d, ww = to_dev(dev, src, dst, w)
        out = torch.zeros(5, dtype=torch.int64, device=dev).view(torch.uint64)
        assert P.mst_select_min_edges(5, s, d, ww, out) == P.MSTX_ERR_VERTEX_RANGE
    # edges but no vertices
    st, _, _, _ = gpu_solve(dev, 0, np.array([0], np.int32), np.array([0], np.int32), np.array([1], np.uint32))
    assert st == P.MSTX_ERR_VERTEX_RANGE


def test_determinism_and_reuse(dev):
    """Repeated solves give identical bytes; a smaller graph after a larger one reuses the workspace."""
    g = gpu_cases.small_cases()[3]
    first = gpu_solve(dev, g.n, g.src, g.dst, g.w)
    for _ in range(4):
        again = gpu_solve(dev, g.n, g.src, g.dst, g.w)
        assert again[0] == first[0] and again[2] == first[2]
        assert np.array_equal(again[1], first[1])
        assert np.array_equal(again[3], first[3])
    small = gpu_cases.small_cases()[0]
    check_against_oracle(dev, small.name + "_after_larger", small.n, small.src, small.dst, small.w)


# ----------------------------------------------- full-size configurations

@pytest.mark.parametrize("name,tail", [("random_n1M_d16", gpu_cases.TAIL_MAX), ("grid_1024x1024", gpu_cases.TAIL_MAX),
                                       ("grid_1024x1024", 0)])
def test_solve_full_size(dev, name, tail):
    from paper_2005_06913_amd import graphgen as G
    g = G.workload(name)
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, stats=(name == "grid_1024x1024"), tail=tail)


def test_solve_full_size_planted(dev):
    """n = 2^20, degree 16, planted tree: the MST is the planted tree, weight n(n-1)/2."""
    from paper_2005_06913_amd import graphgen as G
    g = G.planted_weights(G.workload("random_n1M_d16"))
    print(f"[case] {g.name}", flush=True)
    st, in_mst, total, _ = gpu_solve(dev, g.n, g.src, g.dst, g.w)
    assert st == 0
    assert total == g.n * (g.n - 1) // 2
    assert np.array_equal(in_mst, g.tree_mask.astype(np.uint8))


@pytest.mark.timeout(400)
def test_solve_full_size_rmat(dev):
    """R-MAT scale 22, 2^26 samples (skewed degrees, hubs): bit-exact against Kruskal."""
    from paper_2005_06913_amd import graphgen as G
    g = G.workload("rmat_s22_e26")
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, stats=False)


@pytest.mark.parametrize("n,d", [(10_000, 3), (10_000, 9), (100_000, 3), (100_000, 6), (100_000, 9),
                                 (1_000_000, 3), (1_000_000, 6), (1_000_000, 9)])
def test_solve_paper_shapes(dev, n, d):
    """Table 1 shapes (n vertices, average degree d): edge set, total and round statistics."""
    from paper_2005_06913_amd import graphgen as G
    g = G.paper_shape(n, d, seed=100 + d)
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, stats=True)


@pytest.mark.parametrize("tail", [gpu_cases.TAIL_MAX, 0])
def test_solve_increasing_path_2_20(dev, tail):
    """A path of n = 2^20 vertices with increasing weights: every vertex's
    lightest edge goes to its predecessor, so round 0 adds all n - 1 edges as one
    parent chain of depth n - 1 (the deepest forest the hooking builds and the
    pointer jumping flattens)."""
    from paper_2005_06913_amd import graphgen as G
    g = G.path_graph(1 << 20)
    gstats = check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, tail=tail)
    assert len(gstats) == 1 and int(gstats[0][2]) == g.n - 1


# ------------------------------------------- more than 256 offer buckets

@functools.lru_cache(maxsize=1)
def _five_million():
    """n = 5,000,000 > 256 * 16384: round 0's bucket minima take 306 buckets of
    the widest size, whose offer runs are not padded (the headline sizes use
    at most 256 padded buckets)."""
    from paper_2005_06913_amd import graphgen as G
    return G.tree_plus_extra(5_000_000, 20_000_000, seed=41, name="tree_plus_extra_n5M_m20M")


@pytest.mark.timeout(300)
def test_min_edge_keys_more_than_256_buckets(dev):
    import paper_2005_06913_amd as P
    g = _five_million()
    print(f"[case] min-edge {g.name}", flush=True)
    s, d, w = to_dev(dev, g.src, g.dst, g.w)
    out = torch.zeros(g.n, dtype=torch.int64, device=dev).view(torch.uint64)
    assert P.mst_select_min_edges(g.n, s, d, w, out) == 0
    st, want = oracle.min_edge_keys(g.n, g.src, g.dst, g.w)
    assert st == 0
    assert np.array_equal(out.view(torch.int64).cpu().numpy().view(np.uint64), want)


@pytest.mark.timeout(300)
def test_solve_more_than_256_buckets(dev):
    g = _five_million()
    check_against_oracle(dev, g.name, g.n, g.src, g.dst, g.w, stats=True)


@pytest.mark.timeout(600)
def test_solve_edge_positions_beyond_2_31(dev):
    """m = 2^31 + 2^23 - 1 edges (about 117 GB of device memory with the
    workspace), built on the device: 2^31 uniform extra edges first, weighing
    n .. n + 2^31 - 1, then a random recursive tree on n = 2^23 vertices whose
    edges weigh a permutation of 1 .. n - 1, at positions beyond 2^31.  Every
    extra edge is the heaviest on the cycle it closes with the tree, so the
    MST is the tree (closed form: total n(n - 1)/2, exactly the last n - 1
    flags set)."""
    import paper_2005_06913_amd as P
    from paper_2005_06913_amd import graphgen as G
    n, m_extra = 1 << 23, 1 << 31
    m = m_extra + n - 1
    src, dst, w = G.planted_on_device(n, m_extra, seed=51, device=dev)
    in_mst = torch.full((m,), 7, dtype=torch.uint8, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    print(f"[case] edge positions beyond 2^31: n={n} m={m}", flush=True)
    st = P.mst_solve(n, src, dst, w.view(torch.uint32), in_mst, total, stream)
    torch.cuda.synchronize()
    try:
        assert st == 0, st
        assert int(total.view(torch.int64).item()) == n * (n - 1) // 2
        assert not bool(torch.any(in_mst[:m_extra] != 0))
        assert bool(torch.all(in_mst[m_extra:] == 1))
    finally:
        del src, dst, w, in_mst
        P.mst_workspace_release(stream)
        torch.cuda.empty_cache()
