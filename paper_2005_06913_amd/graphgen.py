"""Seeded synthetic graph generators.

This module builds input graphs only: it holds none of the MST method's
arithmetic and is the one piece of code shared by the GPU path's tests and
the CPU oracle's tests.  The paper evaluates on its own generated graphs,
described only by vertex count and average degree (Section 3, Table 1), with
the requirement that the graph is connected and the edge weights distinct
(Section 2.1, inputs).  The constructions here stand in for those graphs:

* ``tree_plus_extra`` -- a random recursive spanning tree over a random
  vertex permutation plus uniform random extra pairs (no self-loops, no
  duplicate pairs), which makes the graph connected by construction;
* ``grid2d`` -- an R x C 4-neighbour grid, vertex id ``r*C + c``;
* ``rmat`` -- an R-MAT graph, loops and duplicate pairs removed, made
  connected by adding the edges of a random spanning tree it lacks;
* ``paper_shape`` -- ``tree_plus_extra`` at the paper's Table 1 sizes.

Every graph is undirected; each edge is stored once, as ``(min, max)`` before
a seeded orientation shuffle, in a seeded random order.  Weights are a random
permutation of ``1..m`` (distinct, uint32).  Vertex ids are int32.  All
randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph",
    "tree_plus_extra",
    "grid2d",
    "rmat",
    "paper_shape",
    "planted_weights",
    "random_tree_edges",
    "path_graph",
    "star_graph",
    "cycle_graph",
    "complete_graph",
    "workload",
    "WORKLOADS",
    "Batch",
    "batch",
    "planted_on_device",
]


@dataclass
class Graph:
    """An undirected edge list: ``src[e] -- dst[e]`` with weight ``w[e]``.

    ``tree_mask`` (optional) flags the edges of the spanning tree the
    generator planted to guarantee connectivity.
    """

    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    w: np.ndarray  # uint32 [m]
    name: str = ""
    tree_mask: np.ndarray | None = None  # bool [m]

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def with_weights(self, w: np.ndarray, name: str | None = None) -> "Graph":
        return Graph(self.n, self.src, self.dst, np.ascontiguousarray(w, dtype=np.uint32),
                     name if name is not None else self.name, self.tree_mask)


def random_tree_edges(n: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Random recursive tree over a random permutation of the vertices.

    Vertex ``perm[i]`` (i >= 1) attaches to ``perm[j]`` with ``j`` uniform in
    ``[0, i)``.  Returns ``n - 1`` pairs.
    """
    if n <= 1:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    perm = rng.permutation(n).astype(np.int64)
    i = np.arange(1, n, dtype=np.int64)
    j = np.floor(rng.random(n - 1) * i).astype(np.int64)
    j = np.minimum(j, i - 1)
    return perm[i], perm[j]


def _pair_codes(u: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    lo = np.minimum(u, v).astype(np.int64)
    hi = np.maximum(u, v).astype(np.int64)
    return lo * np.int64(n) + hi


def _unique_keep_first(codes: np.ndarray) -> np.ndarray:
    """Distinct values of ``codes`` in order of first occurrence."""
    _, first = np.unique(codes, return_index=True)
    first.sort()
    return codes[first]


def _finish(n: int, codes: np.ndarray, rng: np.random.Generator, name: str,
            tree_count: int = 0, shuffle: bool = True) -> Graph:
    """Decode pair codes, shuffle order and orientation, draw weights.

    The first ``tree_count`` codes are the planted tree's edges.
    """
    m = int(codes.shape[0])
    lo = (codes // n).astype(np.int32)
    hi = (codes % n).astype(np.int32)
    tree = np.zeros(m, dtype=bool)
    tree[:tree_count] = True
    if shuffle:
        order = rng.permutation(m)
        lo, hi, tree = lo[order], hi[order], tree[order]
        flip = rng.random(m) < 0.5
        src = np.where(flip, hi, lo).astype(np.int32)
        dst = np.where(flip, lo, hi).astype(np.int32)
    else:
        src, dst = lo, hi
    w = (rng.permutation(m) + 1).astype(np.uint32)
    return Graph(n, np.ascontiguousarray(src), np.ascontiguousarray(dst), w, name, tree)


def tree_plus_extra(n: int, m: int, seed: int, name: str | None = None) -> Graph:
    """Connected random graph: random spanning tree + ``m - (n-1)`` uniform extra pairs.

    No self-loops and no duplicate pairs; requires ``n - 1 <= m <= n(n-1)/2``.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    max_pairs = n * (n - 1) // 2
    if m < n - 1 or m > max_pairs:
        raise ValueError(f"m={m} outside [n-1, n(n-1)/2] for n={n}")
    rng = np.random.default_rng(seed)
    tu, tv = random_tree_edges(n, rng)
    tree_codes = _pair_codes(tu, tv, n)
    need = m - (n - 1)
    extra = np.zeros(0, np.int64)
    dense = n < 4096 and max_pairs < 4 * m
    if need > 0 and dense:
        # Dense small case: sample without replacement from the pair universe.
        all_lo, all_hi = np.triu_indices(n, k=1)
        universe = all_lo.astype(np.int64) * n + all_hi
        universe = np.setdiff1d(universe, tree_codes, assume_unique=False)
        pick = rng.choice(universe.shape[0], size=need, replace=False)
        extra = universe[pick]
    elif need > 0:
        pool = tree_codes
        while True:
            k = int((need - extra.shape[0]) * 1.15) + 1024
            u = rng.integers(0, n, size=k, dtype=np.int64)
            v = rng.integers(0, n, size=k, dtype=np.int64)
            keep = u != v
            cand = _pair_codes(u[keep], v[keep], n)
            allc = _unique_keep_first(np.concatenate([pool, extra, cand]))
            extra = allc[tree_codes.shape[0]:]
            if extra.shape[0] >= need:
                extra = extra[:need]
                break
    codes = np.concatenate([tree_codes, extra])
    return _finish(n, codes, rng, name or f"tree_plus_extra_n{n}_m{m}_s{seed}", tree_count=n - 1)


def grid2d(rows: int, cols: int, seed: int, name: str | None = None) -> Graph:
    """``rows x cols`` 4-neighbour grid, vertex ``r*cols + c``, row-major edge order.

    Horizontal edges of a row come first, then the vertical edges below it.
    Weights are a random permutation of ``1..m``.
    """
    rng = np.random.default_rng(seed)
    n = rows * cols
    r = np.arange(rows, dtype=np.int64)[:, None]
    c = np.arange(cols, dtype=np.int64)[None, :]
    vid = r * cols + c
    hs = vid[:, :-1].ravel()
    hd = vid[:, 1:].ravel()
    vs = vid[:-1, :].ravel()
    vd = vid[1:, :].ravel()
    # interleave per row: row i horizontals then row i verticals
    h = np.stack([hs, hd], 1).reshape(rows, cols - 1, 2)
    v = np.stack([vs, vd], 1).reshape(rows - 1, cols, 2) if rows > 1 else np.zeros((0, cols, 2), np.int64)
    parts = []
    for i in range(rows):
        parts.append(h[i])
        if i < rows - 1:
            parts.append(v[i])
    e = np.concatenate(parts, 0) if parts else np.zeros((0, 2), np.int64)
    m = e.shape[0]
    w = (rng.permutation(m) + 1).astype(np.uint32)
    return Graph(n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), w,
                 name or f"grid_{rows}x{cols}_s{seed}")


def rmat(scale: int, samples: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, name: str | None = None, chunk: int = 1 << 22) -> Graph:
    """R-MAT graph on ``2**scale`` vertices from ``samples`` draws.

    Each draw picks one quadrant per bit level with probabilities
    ``(a, b, c, 1-a-b-c)`` (no noise, no label permutation).  Self-loops and
    duplicate pairs are removed, then the edges of a random spanning tree that
    the graph lacks are added so the result is connected.
    """
    n = 1 << scale
    rng = np.random.default_rng(seed)
    pieces = []
    left = samples
    ab = a + b
    abc = a + b + c
    while left > 0:
        k = min(chunk, left)
        u = np.zeros(k, np.int64)
        v = np.zeros(k, np.int64)
        for bit in range(scale - 1, -1, -1):
            x = rng.random(k, dtype=np.float32)
            # quadrant: a -> (0,0), b -> (0,1), c -> (1,0), d -> (1,1)
            ubit = (x >= ab).astype(np.int64)
            vbit = ((x >= a) & (x < ab)) | (x >= abc)
            u |= ubit << bit
            v |= vbit.astype(np.int64) << bit
        keep = u != v
        pieces.append(_pair_codes(u[keep], v[keep], n))
        left -= k
    codes = np.unique(np.concatenate(pieces))
    tu, tv = random_tree_edges(n, rng)
    tree_codes = _pair_codes(tu, tv, n)
    missing = np.setdiff1d(tree_codes, codes, assume_unique=False)
    codes = np.concatenate([codes, missing])
    g = _finish(n, codes, rng, name or f"rmat_s{scale}_e{samples}_s{seed}")
    g.tree_mask = None
    return g


def planted_weights(g: Graph, seed: int = 0) -> Graph:
    """Twin of ``g`` whose planted tree edges weigh ``1..n-1`` and extras ``n..m``.

    Every extra edge is heavier than every tree edge, so the minimum spanning
    tree is exactly the planted tree and its weight is ``n(n-1)/2``.
    """
    if g.tree_mask is None:
        raise ValueError("graph has no planted tree")
    rng = np.random.default_rng(seed)
    t = np.flatnonzero(g.tree_mask)
    x = np.flatnonzero(~g.tree_mask)
    w = np.empty(g.m, np.uint32)
    w[t] = (rng.permutation(t.shape[0]) + 1).astype(np.uint32)
    w[x] = (rng.permutation(x.shape[0]) + 1 + t.shape[0]).astype(np.uint32)
    return g.with_weights(w, g.name + "_planted")


def paper_shape(n: int, degree: int, seed: int) -> Graph:
    """Table 1 shape: ``n`` vertices, average degree ``degree`` (m = n*degree/2)."""
    m = max(n - 1, int(round(n * degree / 2)))
    return tree_plus_extra(n, m, seed, name=f"paper_n{n}_d{degree}")


def path_graph(n: int, weights: np.ndarray | None = None) -> Graph:
    """Path ``0-1-...-(n-1)``; edge ``i`` joins ``i`` and ``i+1``."""
    i = np.arange(max(n - 1, 0), dtype=np.int32)
    w = np.arange(1, n, dtype=np.uint32) if weights is None else np.asarray(weights, np.uint32)
    return Graph(n, i, i + 1, w, f"path_{n}")


def star_graph(n: int, seed: int = 0) -> Graph:
    """Star centred at vertex 0 with random distinct weights."""
    rng = np.random.default_rng(seed)
    leaves = np.arange(1, n, dtype=np.int32)
    w = (rng.permutation(n - 1) + 1).astype(np.uint32)
    return Graph(n, np.zeros(n - 1, np.int32), leaves, w, f"star_{n}")


def cycle_graph(n: int, seed: int = 0) -> Graph:
    """Cycle ``0-1-...-(n-1)-0`` with random distinct weights."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int32)
    w = (rng.permutation(n) + 1).astype(np.uint32)
    return Graph(n, i, ((i + 1) % n).astype(np.int32), w, f"cycle_{n}")


def complete_graph(n: int, seed: int = 0) -> Graph:
    """Complete graph K_n, edges in (i<j) lexicographic order, random distinct weights."""
    rng = np.random.default_rng(seed)
    lo, hi = np.triu_indices(n, k=1)
    m = lo.shape[0]
    w = (rng.permutation(m) + 1).astype(np.uint32)
    return Graph(n, lo.astype(np.int32), hi.astype(np.int32), w, f"complete_{n}")


# Named workloads: the single-graph evaluation configurations.
WORKLOADS = {
    # small: n=1024, m=8192, tree + extra pairs
    "random_n1k_m8k": lambda: tree_plus_extra(1024, 8192, seed=1, name="random_n1k_m8k"),
    # paper scale: n=2^20, average degree 16
    "random_n1M_d16": lambda: tree_plus_extra(1 << 20, 8 * (1 << 20), seed=2, name="random_n1M_d16"),
    # 1024 x 1024 4-neighbour grid
    "grid_1024x1024": lambda: grid2d(1024, 1024, seed=3, name="grid_1024x1024"),
    # skewed: R-MAT scale 22, 2^26 samples
    "rmat_s22_e26": lambda: rmat(22, 1 << 26, seed=4, name="rmat_s22_e26"),
}


def workload(name: str) -> Graph:
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}")
    return WORKLOADS[name]()


def planted_on_device(n: int, m_extra: int, seed: int, device, chunk: int = 1 << 28):
    """A graph too large to build on the host, built on `device` (torch tensors
    int32 src, dst and weights as int32 bits of uint32): m_extra uniform extra
    pairs (u != v) first, weighing n .. n + m_extra - 1 in order, then a random
    recursive tree on n vertices (vertex i joins a uniform earlier vertex)
    whose edges weigh a random permutation of 1 .. n - 1.  Every extra edge is
    heavier than every tree edge, so the minimum spanning tree is the tree:
    its flags are exactly the last n - 1 and its weight n(n - 1)/2."""
    import torch

    if not (2 <= n <= 1 << 30 and 0 <= m_extra and n + m_extra <= 1 << 32):
        raise ValueError(f"planted_on_device: n = {n}, m_extra = {m_extra} out of range")
    m = m_extra + n - 1
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    src = torch.empty(m, dtype=torch.int32, device=device)
    dst = torch.empty(m, dtype=torch.int32, device=device)
    w = torch.empty(m, dtype=torch.int32, device=device)
    for off in range(0, m_extra, chunk):
        k = min(chunk, m_extra - off)
        u = torch.randint(0, n, (k,), generator=gen, device=device, dtype=torch.int64)
        v = (u + 1 + torch.randint(0, n - 1, (k,), generator=gen, device=device, dtype=torch.int64)) % n
        src[off:off + k] = u.to(torch.int32)
        dst[off:off + k] = v.to(torch.int32)
        w[off:off + k] = (n + off + torch.arange(k, device=device, dtype=torch.int64)).to(torch.int32)
        del u, v
    i = torch.arange(1, n, device=device, dtype=torch.int64)
    parent = (torch.rand(n - 1, generator=gen, device=device, dtype=torch.float64) * i).floor().to(torch.int64)
    src[m_extra:] = i.to(torch.int32)
    dst[m_extra:] = parent.to(torch.int32)
    w[m_extra:] = (torch.randperm(n - 1, generator=gen, device=device) + 1).to(torch.int32)
    return src, dst, w



@dataclass
class Batch:
    """Independent graphs concatenated: graph g owns vertices [0, n_g) (local ids) and
    edges [edge_offsets[g], edge_offsets[g+1]) of src/dst/w."""

    vertex_offsets: np.ndarray  # int64 [G+1]
    edge_offsets: np.ndarray  # int64 [G+1]
    src: np.ndarray  # int32 [sum m], local ids
    dst: np.ndarray
    w: np.ndarray  # uint32
    name: str = ""

    @property
    def num_graphs(self) -> int:
        return int(self.vertex_offsets.shape[0] - 1)

    def graph(self, g: int) -> Graph:
        a, b = int(self.edge_offsets[g]), int(self.edge_offsets[g + 1])
        n = int(self.vertex_offsets[g + 1] - self.vertex_offsets[g])
        return Graph(n, self.src[a:b], self.dst[a:b], self.w[a:b], f"{self.name}[{g}]")


def batch(num_graphs: int, seed: int, n_lo: int = 64, n_hi: int = 65536, d_lo: float = 4.0,
          d_hi: float = 32.0, name: str | None = None) -> Batch:
    """Independent connected graphs: n log-uniform in [n_lo, n_hi], average degree uniform in
    [d_lo, d_hi], a random recursive spanning tree plus uniform random extra pairs (no
    self-loops; parallel edges possible), weights a random permutation of 1..m per graph,
    random edge order and orientation.  Each graph draws from its own spawned seed."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(num_graphs + 1)
    top = np.random.default_rng(kids[-1])
    ns = np.round(np.exp(top.uniform(np.log(n_lo), np.log(n_hi), num_graphs))).astype(np.int64)
    ds = top.uniform(d_lo, d_hi, num_graphs)
    ms = np.round(ns * ds / 2).astype(np.int64)
    ms = np.clip(ms, ns - 1, ns * (ns - 1) // 2)
    voff = np.zeros(num_graphs + 1, np.int64)
    eoff = np.zeros(num_graphs + 1, np.int64)
    voff[1:] = np.cumsum(ns)
    eoff[1:] = np.cumsum(ms)
    total = int(eoff[-1])
    src = np.empty(total, np.int32)
    dst = np.empty(total, np.int32)
    w = np.empty(total, np.uint32)
    for g in range(num_graphs):
        rng = np.random.default_rng(kids[g])
        n, m = int(ns[g]), int(ms[g])
        tu, tv = random_tree_edges(n, rng)
        k = m - (n - 1)
        u = rng.integers(0, n, k, dtype=np.int64)
        v = (u + 1 + rng.integers(0, n - 1, k, dtype=np.int64)) % n if n > 1 else u
        a = np.concatenate([tu, u])
        b = np.concatenate([tv, v])
        order = rng.permutation(m)
        a, b = a[order], b[order]
        flip = rng.random(m) < 0.5
        lo, hi = int(eoff[g]), int(eoff[g + 1])
        src[lo:hi] = np.where(flip, b, a)
        dst[lo:hi] = np.where(flip, a, b)
        w[lo:hi] = rng.permutation(m) + 1
    return Batch(voff, eoff, src, dst, w, name or f"batch_G{num_graphs}_s{seed}")
