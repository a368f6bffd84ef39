"""Pins for the CPU oracle: facts fixed by the paper and by mathematics.

None of these is derived from the oracle's code:

* golden fixtures (``tests/golden/*.txt``): the paper's four-component proof
  figure (Section 2.2.1) with weights satisfying its stated inequalities, and
  hand traces of the Section 2.1 pseudocode;
* brute force: the minimum spanning forest is, by definition, the spanning
  forest of least total weight.  Equal weights are ordered by input index,
  which (as an infinitesimal perturbation ``w[e] + eps*e``) makes the minimum
  unique: it is the forest minimising ``(sum w, sum e)`` lexicographically;
* Kirchhoff's matrix-tree theorem pins the brute-force enumerator itself;
* closed forms (planted tree, tree input, cycle, star, monotone path);
* library routines (scipy, networkx) on simple distinct-weight graphs;
* Boruvka round invariants: every component picks an edge, every distinct
  picked edge joins two components, so ``added_r = n_r - n_{r+1}``, the
  component count at least halves, and the number of rounds is at most
  ``ceil(log2 n)`` (the O(m log n) bound stated after Section 2.1's code).

``pin_suite(orc)`` runs every pin against an oracle build and returns the
names of the pins that fail; the mutation test uses it to show that planted
mistakes in the oracle are caught.
"""

from __future__ import annotations

import itertools
import math
import os
from dataclasses import dataclass

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------- fixtures

@dataclass
class Fixture:
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray
    in_mst: np.ndarray
    total: int
    status: int
    rounds: list  # [(components, live, added)]
    minedge: dict  # vertex -> edge index (or None) of its lightest edge in round 0


def load_fixture(path: str) -> Fixture:
    n = None
    src, dst, w, flag, rounds = [], [], [], [], []
    names, minedge = {}, {}
    total = status = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "edge":
                names[tok[1]] = len(src)
                src.append(int(tok[2]))
                dst.append(int(tok[3]))
                w.append(int(tok[4]))
                flag.append(int(tok[5]))
            elif tok[0] == "total":
                total = int(tok[1])
            elif tok[0] == "status":
                status = int(tok[1])
            elif tok[0] == "round":
                rounds.append(tuple(int(t) for t in tok[1:4]))
            elif tok[0] == "minedge":
                minedge[int(tok[1])] = None if tok[2] == "none" else names[tok[2]]
            else:
                raise ValueError(f"{path}: unknown line {line!r}")
    return Fixture(os.path.basename(path), n, np.array(src, np.int32), np.array(dst, np.int32),
                   np.array(w, np.uint32), np.array(flag, np.uint8), total, status, rounds, minedge)


def all_fixtures() -> list[Fixture]:
    return [load_fixture(os.path.join(GOLDEN, f)) for f in sorted(os.listdir(GOLDEN))
            if f.endswith(".txt")]


# -------------------------------------------------------------- brute force

def _components(n, src, dst):
    """Connected components by BFS (independent of any union-find)."""
    adj = [[] for _ in range(n)]
    for a, b in zip(src.tolist(), dst.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    comp = [-1] * n
    c = 0
    for s in range(n):
        if comp[s] != -1:
            continue
        comp[s] = c
        stack = [s]
        while stack:
            v = stack.pop()
            for u in adj[v]:
                if comp[u] == -1:
                    comp[u] = c
                    stack.append(u)
        c += 1
    return c, comp


def _is_forest(n, edges):
    """True if the edge list has no cycle (checked by repeated leaf removal)."""
    deg = [0] * n
    adj = [[] for _ in range(n)]
    for i, (a, b) in enumerate(edges):
        if a == b:
            return False
        deg[a] += 1
        deg[b] += 1
        adj[a].append((b, i))
        adj[b].append((a, i))
    removed = [False] * len(edges)
    leaves = [v for v in range(n) if deg[v] == 1]
    left = len(edges)
    while leaves:
        v = leaves.pop()
        for u, i in adj[v]:
            if not removed[i]:
                removed[i] = True
                left -= 1
                deg[v] -= 1
                deg[u] -= 1
                if deg[u] == 1:
                    leaves.append(u)
    return left == 0


def brute_force_msf(n, src, dst, w):
    """Enumerate every spanning forest; return (in_mst, total, count).

    A spanning forest has ``n - c`` edges and no cycle (c = connected
    components).  The minimum is taken over ``(sum w, sum index)``.  ``count``
    is the number of spanning forests (spanning trees when connected).
    """
    m = len(src)
    c, _ = _components(n, src, dst)
    k = n - c
    best = None
    count = 0
    pairs = list(zip(src.tolist(), dst.tolist()))
    for sub in itertools.combinations(range(m), k):
        if not _is_forest(n, [pairs[i] for i in sub]):
            continue
        count += 1
        key = (sum(int(w[i]) for i in sub), sum(sub))
        if best is None or key < best[0]:
            best = (key, sub)
    flags = np.zeros(m, np.uint8)
    if best is not None:
        flags[list(best[1])] = 1
        return flags, best[0][0], count
    return flags, 0, count


def matrix_tree_count(n, src, dst):
    """Number of spanning trees of a connected multigraph (Kirchhoff)."""
    if n <= 1:
        return 1
    L = np.zeros((n, n), dtype=np.float64)
    for a, b in zip(src.tolist(), dst.tolist()):
        if a == b:
            continue
        L[a, a] += 1
        L[b, b] += 1
        L[a, b] -= 1
        L[b, a] -= 1
    return int(round(np.linalg.det(L[1:, 1:])))


def random_small_graph(rng, n_max=7, m_max=11, wmax=None, loops=True):
    n = int(rng.integers(1, n_max + 1))
    m = int(rng.integers(0, m_max + 1))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if not loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
        m = len(src)
    hi = wmax if wmax is not None else 4
    w = rng.integers(1, hi + 1, m).astype(np.uint32)
    return n, src, dst, w


# ---------------------------------------------------------------- the pins

def _eq(a, b, what):
    if isinstance(a, np.ndarray):
        if not np.array_equal(a, b):
            raise AssertionError(f"{what}: arrays differ")
    elif a != b:
        raise AssertionError(f"{what}: {a!r} != {b!r}")


def pin_golden(orc):
    for fx in all_fixtures():
        for name, res in (("kruskal", orc.kruskal(fx.n, fx.src, fx.dst, fx.w)),
                          ("boruvka", orc.boruvka(fx.n, fx.src, fx.dst, fx.w))):
            _eq(res.in_mst, fx.in_mst, f"{fx.name} {name} edge set")
            _eq(res.total, fx.total, f"{fx.name} {name} total")
            _eq(res.status, fx.status, f"{fx.name} {name} status")
        b = orc.boruvka(fx.n, fx.src, fx.dst, fx.w)
        _eq([tuple(r) for r in b.stats.tolist()], fx.rounds, f"{fx.name} boruvka rounds")
        _eq(orc.check_mst(fx.n, fx.src, fx.dst, fx.w, fx.in_mst, fx.total), 0, f"{fx.name} certificate")


def expected_min_keys(fx: Fixture) -> np.ndarray:
    """Round-0 keys (w << 32 | e) spelled out from a fixture's ``minedge`` lines."""
    keys = np.full(fx.n, np.iinfo(np.uint64).max, np.uint64)
    for v, e in fx.minedge.items():
        if e is not None:
            keys[v] = (np.uint64(fx.w[e]) << np.uint64(32)) | np.uint64(e)
    return keys


def numpy_min_keys(n, src, dst, w) -> np.ndarray:
    """Round-0 minima with numpy's unbuffered ``minimum.at`` (a library reduction)."""
    keys = np.full(n, np.iinfo(np.uint64).max, np.uint64)
    e = np.arange(len(src), dtype=np.uint64)
    k = (w.astype(np.uint64) << np.uint64(32)) | e
    keep = src != dst
    np.minimum.at(keys, src[keep], k[keep])
    np.minimum.at(keys, dst[keep], k[keep])
    return keys


def pin_min_edges(orc, seed=17):
    for fx in all_fixtures():
        if not fx.minedge:
            continue
        st, keys = orc.min_edge_keys(fx.n, fx.src, fx.dst, fx.w)
        _eq(st, 0, f"{fx.name} min-edge status")
        _eq(keys, expected_min_keys(fx), f"{fx.name} round-0 minima")
    rng = np.random.default_rng(seed)
    for t in range(60):
        n, src, dst, w = random_small_graph(rng, n_max=40, m_max=200, wmax=3 if t % 2 else 10**9)
        st, keys = orc.min_edge_keys(n, src, dst, w)
        _eq(keys, numpy_min_keys(n, src, dst, w), f"case {t} round-0 minima vs numpy")


def pin_brute_force(orc, cases=250, seed=11):
    rng = np.random.default_rng(seed)
    for t in range(cases):
        # alternate tie-heavy and distinct weights
        n, src, dst, w = random_small_graph(rng, wmax=3 if t % 2 else 1000)
        flags, total, _ = brute_force_msf(n, src, dst, w)
        c, _ = _components(n, src, dst)
        want_status = 0 if c <= 1 else 1
        for name, res in (("kruskal", orc.kruskal(n, src, dst, w)),
                          ("boruvka", orc.boruvka(n, src, dst, w))):
            _eq(res.in_mst, flags, f"case {t} {name} edge set")
            _eq(res.total, total, f"case {t} {name} total")
            _eq(res.status, want_status, f"case {t} {name} status")
        _eq(orc.check_mst(n, src, dst, w, flags, total), 0, f"case {t} certificate accepts brute force")


def pin_closed_forms(orc, seed=5):
    from paper_2005_06913_amd import graphgen as G
    rng = np.random.default_rng(seed)
    # tree input: every edge, total = sum of weights
    n = 300
    tu, tv = G.random_tree_edges(n, rng)
    w = (rng.permutation(n - 1) + 1).astype(np.uint32)
    for name, res in (("kruskal", orc.kruskal(n, tu, tv, w)), ("boruvka", orc.boruvka(n, tu, tv, w))):
        _eq(res.in_mst, np.ones(n - 1, np.uint8), f"tree input {name}")
        _eq(res.total, int(w.sum()), f"tree input {name} total")
    # cycle: every edge but the heaviest
    g = G.cycle_graph(257, seed=seed)
    want = np.ones(g.m, np.uint8)
    want[int(np.argmax(g.w))] = 0
    for name, res in (("kruskal", orc.kruskal(g.n, g.src, g.dst, g.w)),
                      ("boruvka", orc.boruvka(g.n, g.src, g.dst, g.w))):
        _eq(res.in_mst, want, f"cycle {name}")
        _eq(res.total, int(g.w.sum()) - int(g.w.max()), f"cycle {name} total")
    # star: every edge, one round
    g = G.star_graph(500, seed=seed)
    b = orc.boruvka(g.n, g.src, g.dst, g.w)
    _eq(b.in_mst, np.ones(g.m, np.uint8), "star edge set")
    _eq(len(b.stats), 1, "star rounds")
    # monotone paths: every edge, one round (each vertex's lightest edge is distinct per pair)
    for wts in (np.arange(1, 1000, dtype=np.uint32), np.arange(999, 0, -1, dtype=np.uint32)):
        g = G.path_graph(1000, wts)
        for name, res in (("kruskal", orc.kruskal(g.n, g.src, g.dst, g.w)),
                          ("boruvka", orc.boruvka(g.n, g.src, g.dst, g.w))):
            _eq(res.in_mst, np.ones(g.m, np.uint8), f"path {name}")
            _eq(res.total, 999 * 1000 // 2, f"path {name} total")
        _eq(len(orc.boruvka(g.n, g.src, g.dst, g.w).stats), 1, "monotone path rounds")
    # planted tree: tree edges weigh 1..n-1, extras heavier -> MST is the tree, total n(n-1)/2
    g = G.planted_weights(G.tree_plus_extra(2048, 2048 * 6, seed=seed))
    for name, res in (("kruskal", orc.kruskal(g.n, g.src, g.dst, g.w)),
                      ("boruvka", orc.boruvka(g.n, g.src, g.dst, g.w))):
        _eq(res.in_mst, g.tree_mask.astype(np.uint8), f"planted {name}")
        _eq(res.total, g.n * (g.n - 1) // 2, f"planted {name} total")


def pin_libraries(orc, seed=7):
    """scipy and networkx on simple graphs with distinct weights >= 1."""
    import networkx as nx
    import scipy.sparse as sp
    from scipy.sparse.csgraph import minimum_spanning_tree

    from paper_2005_06913_amd import graphgen as G
    graphs = [G.tree_plus_extra(2000, 9000, seed=seed), G.grid2d(40, 50, seed=seed),
              G.complete_graph(60, seed=seed)]
    # a disconnected one: two random graphs side by side
    a = G.tree_plus_extra(300, 900, seed=seed + 1)
    b = G.tree_plus_extra(200, 500, seed=seed + 2)
    graphs.append(G.Graph(500, np.concatenate([a.src, b.src + 300]).astype(np.int32),
                          np.concatenate([a.dst, b.dst + 300]).astype(np.int32),
                          np.concatenate([a.w, b.w + 10_000]).astype(np.uint32), "two_parts"))
    for g in graphs:
        k = orc.kruskal(g.n, g.src, g.dst, g.w)
        bo = orc.boruvka(g.n, g.src, g.dst, g.w)
        M = sp.coo_matrix((g.w.astype(np.float64), (g.src, g.dst)), shape=(g.n, g.n)).tocsr()
        T = minimum_spanning_tree(M).tocoo()
        _eq(k.total, int(T.data.sum()), f"{g.name} scipy total")
        _eq(bo.total, int(T.data.sum()), f"{g.name} scipy total (boruvka)")
        H = nx.Graph()
        H.add_nodes_from(range(g.n))
        for i, (u, v, wt) in enumerate(zip(g.src.tolist(), g.dst.tolist(), g.w.tolist())):
            H.add_edge(u, v, weight=wt, idx=i)
        want = np.zeros(g.m, np.uint8)
        for _, _, d in nx.minimum_spanning_edges(H, algorithm="kruskal", data=True):
            want[d["idx"]] = 1
        _eq(k.in_mst, want, f"{g.name} networkx edge set")
        _eq(bo.in_mst, want, f"{g.name} networkx edge set (boruvka)")


def pin_round_invariants(orc, seed=3):
    from paper_2005_06913_amd import graphgen as G
    graphs = [G.tree_plus_extra(5000, 40000, seed=seed), G.grid2d(64, 64, seed=seed),
              G.tree_plus_extra(1024, 8192, seed=1), G.rmat(12, 30000, seed=seed)]
    for g in graphs:
        b = orc.boruvka(g.n, g.src, g.dst, g.w)
        st = b.stats
        c, _ = _components(g.n, g.src, g.dst)
        _eq(int(st[0, 0]), g.n, f"{g.name} first round components")
        _eq(int(st[0, 1]), int((g.src != g.dst).sum()), f"{g.name} first round live edges")
        for r in range(len(st) - 1):
            _eq(int(st[r, 2]), int(st[r, 0] - st[r + 1, 0]), f"{g.name} added == n_r - n_(r+1)")
            if not st[r + 1, 0] * 2 <= st[r, 0]:
                raise AssertionError(f"{g.name}: components did not halve in round {r}")
            if not st[r + 1, 1] <= st[r, 1]:
                raise AssertionError(f"{g.name}: live edges grew in round {r}")
        _eq(int(st[:, 2].sum()), g.n - c, f"{g.name} tree edges == n - c")
        if not len(st) <= math.ceil(math.log2(g.n)):
            raise AssertionError(f"{g.name}: {len(st)} rounds > ceil(log2 n)")
        _eq(int(b.in_mst.sum()), g.n - c, f"{g.name} marked edges")


def pin_certificate_rejects(orc, seed=9):
    """The checker must reject every kind of wrong answer."""
    from paper_2005_06913_amd import graphgen as G
    g = G.tree_plus_extra(400, 2400, seed=seed)
    k = orc.kruskal(g.n, g.src, g.dst, g.w)
    _eq(orc.check_mst(g.n, g.src, g.dst, g.w, k.in_mst, k.total), 0, "accepts the MST")
    rng = np.random.default_rng(seed)
    tree = np.flatnonzero(k.in_mst)
    non = np.flatnonzero(k.in_mst == 0)
    adj = {}
    for t in tree.tolist():
        adj.setdefault(int(g.src[t]), []).append((int(g.dst[t]), t))
        adj.setdefault(int(g.dst[t]), []).append((int(g.src[t]), t))

    def tree_path(a, b):
        prev = {a: None}
        stack = [a]
        while stack:
            v = stack.pop()
            for u, t in adj.get(v, []):
                if u not in prev:
                    prev[u] = (v, t)
                    stack.append(u)
        path = []
        v = b
        while prev[v] is not None:
            v, t = prev[v]
            path.append(t)
        return path

    # swap: add a non-tree edge e, drop an edge of the tree path it closes -> still a
    # spanning tree, but heavier, so the cycle property must fail
    for e in rng.choice(non, size=40, replace=False).tolist():
        path = tree_path(int(g.src[e]), int(g.dst[e]))
        for drop in {path[int(rng.integers(len(path)))], min(path, key=lambda t: (int(g.w[t]), t))}:
            bad = k.in_mst.copy()
            bad[e] = 1
            bad[drop] = 0
            tot = k.total + int(g.w[e]) - int(g.w[drop])
            _eq(orc.check_mst(g.n, g.src, g.dst, g.w, bad, tot), -14, "rejects a heavier spanning tree")
    # the heavier edge sits right below the lowest common ancestor: star 0-{1,2}
    s3 = np.array([0, 0, 1], np.int32)
    d3 = np.array([1, 2, 2], np.int32)
    w3 = np.array([10, 1, 5], np.uint32)
    _eq(orc.check_mst(3, s3, d3, w3, np.array([1, 1, 0], np.uint8), 11), -14, "rejects the heavier star")
    _eq(orc.check_mst(3, s3, d3, w3, np.array([0, 1, 1], np.uint8), 6), 0, "accepts the lighter tree")
    e = int(non[0])
    bad = k.in_mst.copy()
    bad[int(tree[0])] = 0
    _eq(orc.check_mst(g.n, g.src, g.dst, g.w, bad, k.total - int(g.w[tree[0]])), -13, "rejects a dropped edge")
    bad = k.in_mst.copy()
    bad[e] = 1
    _eq(orc.check_mst(g.n, g.src, g.dst, g.w, bad, k.total + int(g.w[e])), -12, "rejects a cycle")
    _eq(orc.check_mst(g.n, g.src, g.dst, g.w, k.in_mst, k.total + 1), -15, "rejects a wrong total")
    bad = k.in_mst.copy()
    bad[int(tree[1])] = 2
    _eq(orc.check_mst(g.n, g.src, g.dst, g.w, bad, k.total), -10, "rejects a non-0/1 flag")
    loop_src = np.append(g.src, np.int32(5))
    loop_dst = np.append(g.dst, np.int32(5))
    loop_w = np.append(g.w, np.uint32(1))
    flags = np.append(k.in_mst, np.uint8(1))
    _eq(orc.check_mst(g.n, loop_src, loop_dst, loop_w, flags, k.total + 1), -11, "rejects a marked loop")


def pin_args(orc):
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    w = np.array([1, 2], np.uint32)
    _eq(orc.kruskal(2, src, dst, w).status, -2, "vertex id >= n")
    for bad_src, bad_dst in ((2, 0), (0, 2), (-1, 0), (0, -1)):
        s1, d1 = np.array([bad_src], np.int32), np.array([bad_dst], np.int32)
        _eq(orc.kruskal(2, s1, d1, w[:1]).status, -2, f"vertex ({bad_src},{bad_dst}) out of range")
        _eq(orc.boruvka(2, s1, d1, w[:1]).status, -2, f"vertex ({bad_src},{bad_dst}) out of range")
    _eq(orc.boruvka(2, src, dst, w).status, -2, "vertex id >= n (boruvka)")
    _eq(orc.kruskal(-1, src[:0], dst[:0], w[:0]).status, -1, "negative n")
    for n in (0, 1):
        r = orc.kruskal(n, src[:0], dst[:0], w[:0])
        _eq((r.status, r.total), (0, 0), f"n={n} no edges")
        _eq(orc.boruvka(n, src[:0], dst[:0], w[:0]).status, 0, f"n={n} no edges (boruvka)")
    _eq(orc.kruskal(2, src[:0], dst[:0], w[:0]).status, 1, "two isolated vertices")


def pin_matrix_tree(orc=None, cases=120, seed=13):
    """The brute-force enumerator counts exactly Kirchhoff's number of spanning trees."""
    rng = np.random.default_rng(seed)
    done = 0
    while done < cases:
        n, src, dst, w = random_small_graph(rng)
        c, _ = _components(n, src, dst)
        if c != 1:
            continue
        _, _, count = brute_force_msf(n, src, dst, w)
        _eq(count, matrix_tree_count(n, src, dst), f"spanning tree count n={n} m={len(src)}")
        done += 1


PINS = {
    "golden": pin_golden,
    "brute_force": pin_brute_force,
    "min_edges": pin_min_edges,
    "closed_forms": pin_closed_forms,
    "libraries": pin_libraries,
    "round_invariants": pin_round_invariants,
    "certificate_rejects": pin_certificate_rejects,
    "args": pin_args,
}


def pin_suite(orc) -> list[str]:
    """Names of the pins that fail on ``orc`` (a crash counts as a failure)."""
    failed = []
    for name, fn in PINS.items():
        try:
            fn(orc)
        except Exception:  # noqa: BLE001 - any exception is a caught mistake
            failed.append(name)
    return failed
