"""Graph cases for the GPU parity tests (inputs only; no method arithmetic).

Small and mid-size cases run the full oracle (Kruskal for the tree, Boruvka
for the round statistics); sizes are chosen to span several workgroup tiles
(1024 records) and segments with ragged tails.
"""

from __future__ import annotations

import numpy as np

from paper_2005_06913_amd import graphgen as G


def _concat(parts, name):
    n = 0
    src, dst, w = [], [], []
    for g, wshift in parts:
        src.append(g.src + n)
        dst.append(g.dst + n)
        w.append(g.w + np.uint32(wshift))
        n += g.n
    return G.Graph(n, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32),
                   np.concatenate(w).astype(np.uint32), name)


DENSE_MAX = 200  # largest component count the library's dense finish takes
SMALL_MAX = 8192  # largest vertex count of the library's one-workgroup path
LDS_SLOTS = 20352  # largest component count whose minima the scan keeps in LDS
TAIL_MAX = 10240  # largest round bound whose hook .. relabel run in one workgroup
MID_MAX = 16280  # largest vertex count of a batched graph solved by one workgroup, edges streamed
MID_MAX_EDGES = 1 << 21  # ... and its largest edge count
PRE_MAX = 65536  # largest vertex count of a batched graph contracted by one workgroup first
BUCKET_MAX = 1023 << 14  # largest component count whose minima bucket mode takes
SPARSE_MAX = 8192  # largest component count at which the sparse finish may end the solve
SPARSE_DEFAULT = 1 << 20  # the library's default live-edge bound for trying it


def stats_consistent(gpu_stats, oracle_stats, limit=DENSE_MAX):
    """Whether per-round statistics (components, live edges, edges added) of a
    solve that may end with the dense or the sparse finish agree with the
    oracle's Boruvka rounds.

    Without a finish the rows are equal.  A finish at round r ends the rows at
    r: rows before r are equal, row r has the oracle's component and live-edge
    counts (at most `limit` components), and its edges added are the oracle's
    added edges of round r and every later round together.
    """
    g = [tuple(int(x) for x in r) for r in gpu_stats]
    o = [tuple(int(x) for x in r) for r in oracle_stats]
    if g == o:
        return True
    r = len(g) - 1
    if r < 0 or r >= len(o) or g[:r] != o[:r]:
        return False
    return (g[r][0] == o[r][0] <= limit and g[r][1] == o[r][1]
            and g[r][2] == sum(row[2] for row in o[r:]))


def ties_multigraph(n, m, seed, wmax=4):
    """Random multigraph with self-loops, parallel edges and heavily tied weights."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    w = rng.integers(1, wmax + 1, m).astype(np.uint32)
    # make it connected: a path through a random permutation with heavy weights
    perm = rng.permutation(n).astype(np.int32)
    src = np.concatenate([src, perm[:-1]])
    dst = np.concatenate([dst, perm[1:]])
    w = np.concatenate([w, np.full(n - 1, wmax + 1, np.uint32)])
    order = rng.permutation(len(src))
    return G.Graph(n, src[order], dst[order], w[order], f"ties_n{n}_m{m}_s{seed}")


def halving_path(k, extra, seed):
    """A path 0 - 1 - ... - (n - 1), n = 2^k, whose edge (i, i + 1) weighs the
    position of the lowest set bit of i + 1 (ties broken by i), plus `extra`
    uniform random extra edges per vertex, all heavier than every path edge.
    Every round pairs neighbouring components of the path, so the component
    count halves round by round while almost every edge stays live: rounds
    that read 16-bit records while bucket, LDS and dense minima follow one
    another."""
    rng = np.random.default_rng(seed)
    n = 1 << k
    i = np.arange(n - 1, dtype=np.int64)
    low = i + 1
    ctz = np.zeros(n - 1, np.int64)
    while np.any(low % 2 == 0):
        even = low % 2 == 0
        ctz[even] += 1
        low[even] //= 2
    wp = ctz * n + i + 1
    me = extra * n
    a = rng.integers(0, n, me)
    b = rng.integers(0, n - 1, me)
    b = b + (b >= a)  # no loops
    we = (k + 1) * n + 1 + rng.permutation(me)
    src = np.concatenate([i, a]).astype(np.int32)
    dst = np.concatenate([i + 1, b]).astype(np.int32)
    w = np.concatenate([wp, we]).astype(np.uint32)
    order = rng.permutation(len(src))
    return G.Graph(n, src[order], dst[order], w[order], f"halving_path_2^{k}_x{extra}")


def small_cases():
    """(graph, expect_connected) pairs that the oracle finishes in well under a second."""
    cases = [
        G.workload("random_n1k_m8k"),
        G.tree_plus_extra(1000, 4097, seed=21, name="ragged_n1000_m4097"),
        G.tree_plus_extra(3000, 3000 * 4 + 77, seed=22, name="ragged_n3000"),
        G.paper_shape(10_000, 3, seed=100),
        G.paper_shape(10_000, 6, seed=101),
        G.paper_shape(10_000, 9, seed=102),
        G.grid2d(64, 96, seed=23, name="grid_64x96"),
        G.complete_graph(64, seed=24),
        G.star_graph(20_000, seed=25),
        G.cycle_graph(10_001, seed=26),
        G.path_graph(30_000),  # increasing weights: one round, a hook chain of depth n-1
        G.path_graph(30_000, np.arange(29_999, 0, -1, dtype=np.uint32)).with_weights(
            np.arange(29_999, 0, -1, dtype=np.uint32), "path_decreasing_30000"),
        ties_multigraph(2000, 12_000, seed=27),
        ties_multigraph(5000, 9000, seed=28, wmax=1),  # every weight equal but the path
        G.rmat(14, 120_000, seed=29),
        G.planted_weights(G.tree_plus_extra(50_000, 400_000, seed=30)),
        # either side of the LDS-table limit: round 0 in LDS mode at it, bucket mode above
        G.tree_plus_extra(LDS_SLOTS, 5 * LDS_SLOTS + 3, seed=35, name="lds_limit_n20352"),
        G.tree_plus_extra(LDS_SLOTS + 1, 5 * LDS_SLOTS + 5, seed=36, name="lds_limit_n20353"),
        # more than 20352 vertices: offers sorted into buckets.  Skewed degrees put
        # most offers into a few buckets (extra workgroups for them); a grid's
        # row-major edge order gives long runs (cut into items)
        G.rmat(16, 400_000, seed=33),
        G.grid2d(256, 256, seed=34, name="grid_256x256"),
        # component counts halving round by round with few edges dying:
        # 16-bit records kept in place from round 2 on, read through composed
        # label maps in bucket (2^17), LDS and dense rounds
        halving_path(17, 8, seed=37),
        halving_path(15, 6, seed=38),
        _concat([(G.tree_plus_extra(700, 3000, seed=31), 0), (G.tree_plus_extra(500, 900, seed=32), 10_000),
                 (G.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint32)), 0)],
                "disconnected_3parts_plus_isolated"),
    ]
    return cases


def edge_cases():
    """Degenerate inputs: (name, n, src, dst, w)."""
    z32 = np.zeros(0, np.int32)
    zw = np.zeros(0, np.uint32)
    return [
        ("n0_m0", 0, z32, z32, zw),
        ("n1_m0", 1, z32, z32, zw),
        ("n2_m0", 2, z32, z32, zw),
        ("n1_loops", 1, np.zeros(3, np.int32), np.zeros(3, np.int32), np.array([5, 1, 9], np.uint32)),
        ("n2_one_edge", 2, np.array([1], np.int32), np.array([0], np.int32), np.array([7], np.uint32)),
        ("n2_parallel_ties", 2, np.array([0, 1, 0], np.int32), np.array([1, 0, 1], np.int32),
         np.array([3, 3, 3], np.uint32)),
        ("max_weight", 3, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32),
         np.array([0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFE], np.uint32)),
        ("zero_weight", 3, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32),
         np.array([0, 0, 0], np.uint32)),
        ("isolated_many", 100, np.array([5, 70], np.int32), np.array([6, 71], np.int32),
         np.array([2, 1], np.uint32)),
    ]
