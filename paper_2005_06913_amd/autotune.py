"""Autotuner for the library's launch knobs.

The solve is exact whatever the knobs say (every knob only chooses between
kernels or launch shapes that compute the same thing), so tuning is a pure
timing search: for a workload class it times the solve under candidate knob
settings, checks that every candidate produced the same bytes (edge flags,
total, status) as the library defaults, and keeps the fastest.  Results are
cached in a JSON file keyed by (device, workload class), where a class is a
bucket of graph shapes:

* single graphs (``mst_solve``): ceil(log2 n) and round(log2 of the average
  degree 2m/n);
* batches (``mst_solve_batched``): ceil(log2 of the graph count) and
  ceil(log2 of the total edge count).

Knobs (the C ABI setters of ``include/mstx.h``): the dense-finish limit, the
round-tail limit, the one-workgroup limit for small single graphs, the
bucket-mode limit, the LDS-mode scan occupancy, the sparse-finish limit, and
for batches the mid-size limit.  The search is coordinate descent from the defaults: each knob in
turn takes the candidate value that is fastest with the others fixed, two
passes.

    from paper_2005_06913_amd import autotune
    best = autotune.tune_single(n, src, dst, w)        # device tensors
    with autotune.tuned_single(n, m):                  # knobs from the cache
        res = paper_2005_06913_amd.solve(n, src, dst, w)

The cache file is ``$MSTX_TUNING_FILE`` if set, else
``~/.cache/mstx/tuning.json``; lookups fall back to ``tuning.json`` beside
this module, the settings tuned on an MI355X for the benchmark classes
(``python -m paper_2005_06913_amd.autotune --ship`` rewrites it).
"""

from __future__ import annotations

import contextlib
import json
import math
import os
import statistics
from typing import Callable, Dict, List, Optional, Sequence

from . import binding as B

# knob name -> candidate values (the setters below return the previous value
# and only query with a negative argument)
SINGLE_KNOBS: Dict[str, Sequence[int]] = {
    "dense_limit": (0, 64, 128, 200),
    "tail_limit": (0, 2048, 10240),
    "small_limit": (0, 8192),
    "bucket_limit": (0, 16760832),
    "scan_occupancy": (0, 1, 2, 4),
    "sparse_limit": (0, 1 << 20),
}
BATCH_KNOBS: Dict[str, Sequence[int]] = {
    "mid_limit": (8192, 12288, 16280),
    "dense_limit": (0, 200),
    "tail_limit": (0, 10240),
    "scan_occupancy": (0, 1, 2),
}
SETTERS: Dict[str, Callable[[int], int]] = {
    "dense_limit": B.mst_set_dense_limit,
    "tail_limit": B.mst_set_tail_limit,
    "small_limit": B.mst_set_small_limit,
    "bucket_limit": B.mst_set_bucket_limit,
    "scan_occupancy": B.mst_set_scan_occupancy,
    "mid_limit": B.mst_set_mid_limit,
    "sparse_limit": B.mst_set_sparse_limit,
}


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def cache_path() -> str:
    p = os.environ.get("MSTX_TUNING_FILE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "mstx", "tuning.json")


def single_class(n: int, m: int) -> str:
    """Workload class of one graph: vertex-count and degree buckets."""
    nb = max(0, math.ceil(math.log2(max(n, 1))))
    deg = 2.0 * m / max(n, 1)
    db = round(math.log2(deg)) if deg > 0 else -1
    return f"single/n2^{nb}/deg2^{db}"


def batch_class(num_graphs: int, sum_m: int) -> str:
    """Workload class of a batch: graph-count and total-edge buckets."""
    gb = max(0, math.ceil(math.log2(max(num_graphs, 1))))
    mb = max(0, math.ceil(math.log2(max(sum_m, 1))))
    return f"batched/g2^{gb}/m2^{mb}"


def device_key() -> str:
    """The device's ISA and compute-unit count (the marketing name is not used:
    the same card reports different names depending on the installed id tables)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', '')}/cu{p.multi_processor_count}"


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return {"version": 1, "entries": {}}
    if not isinstance(doc, dict) or doc.get("version") != 1 or not isinstance(doc.get("entries"), dict):
        return {"version": 1, "entries": {}}
    return doc


def save_cache(doc: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def defaults(names: Sequence[str]) -> Dict[str, int]:
    """The library's current value of every named knob."""
    return {k: int(SETTERS[k](-1)) for k in names}


@contextlib.contextmanager
def knobs(settings: Dict[str, int]):
    """Sets the knobs for the duration of the block, then restores them."""
    prev = {}
    try:
        for k, v in settings.items():
            prev[k] = SETTERS[k](int(v))
        yield
    finally:
        for k, v in prev.items():
            SETTERS[k](v)


def coordinate_search(space: Dict[str, Sequence[int]], start: Dict[str, int],
                      measure: Callable[[Dict[str, int]], float], passes: int = 2,
                      min_gain: float = 0.01) -> tuple:
    """Coordinate descent over `space` from `start`; `measure(settings)` returns
    a time (and may raise if a result differs).  A candidate replaces the best
    setting only if it is faster by more than `min_gain` (relative), so timing
    noise does not move the knobs.  Returns (best settings, best time, list of
    (settings, time) tried)."""
    best = dict(start)
    seen: Dict[tuple, float] = {}

    def timed(s):
        key = tuple(sorted(s.items()))
        if key not in seen:
            seen[key] = measure(s)
        return seen[key]

    best_t = timed(best)
    for _ in range(passes):
        changed = False
        for name, values in space.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best)
                cand[name] = v
                t = timed(cand)
                if t < best_t * (1.0 - min_gain):
                    best, best_t, changed = cand, t, True
        if not changed:
            break
    tried = [(dict(k), t) for k, t in seen.items()]
    return best, best_t, tried


def _event_ms(fn, reps: int) -> float:
    import torch
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune_single(n: int, src, dst, w, reps: int = 5, passes: int = 2, path: Optional[str] = None,
                space: Optional[Dict[str, Sequence[int]]] = None) -> dict:
    """Tunes ``mst_solve`` on this graph (device tensors) and stores the result
    under its class.  Raises if any candidate's result differs from the
    defaults' result."""
    import torch
    space = dict(space or SINGLE_KNOBS)
    m = int(src.numel())
    dev = src.device
    in_mst = torch.empty(m, dtype=torch.uint8, device=dev)
    total = torch.empty(1, dtype=torch.uint64, device=dev)
    base = defaults(list(space))

    def run():
        st = B.mst_solve(n, src, dst, w, in_mst, total)
        if st < 0:
            raise B.MstxError(st)
        return st

    with knobs(base):
        st0 = run()
        torch.cuda.synchronize()
        ref = (st0, in_mst.clone(), int(total.view(torch.int64).item()))

    def measure(s):
        with knobs(s):
            run()  # warm (workspace, code objects)
            t = _event_ms(run, reps)
            st = run()
            torch.cuda.synchronize()
            same = (st == ref[0] and int(total.view(torch.int64).item()) == ref[2]
                    and bool(torch.equal(in_mst, ref[1])))
        if not same:
            raise RuntimeError(f"autotune: knob setting {s} changed the result of the solve")
        return t

    best, best_t, tried = coordinate_search(space, base, measure, passes)
    dflt = [t for st_, t in tried if st_ == base]
    entry = {"knobs": best, "ms": best_t, "default_ms": dflt[0] if dflt else None, "n": n, "m": m,
             "candidates": len(tried)}
    doc = load_cache(path)
    doc["entries"].setdefault(device_key(), {})[single_class(n, m)] = entry
    save_cache(doc, path)
    return entry


def tune_batched(vertex_offsets, edge_offsets, src, dst, w, reps: int = 3, passes: int = 1,
                 path: Optional[str] = None, space: Optional[Dict[str, Sequence[int]]] = None) -> dict:
    """Tunes ``mst_solve_batched`` on this batch and stores the result under its class."""
    import numpy as np
    import torch
    space = dict(space or BATCH_KNOBS)
    vo = np.ascontiguousarray(vertex_offsets, np.int64)
    eo = np.ascontiguousarray(edge_offsets, np.int64)
    G = vo.shape[0] - 1
    m = int(eo[-1])
    dev = src.device
    in_mst = torch.empty(m, dtype=torch.uint8, device=dev)
    total = torch.empty(G, dtype=torch.uint64, device=dev)
    status = torch.empty(G, dtype=torch.int32, device=dev)
    base = defaults(list(space))

    def run():
        rc = B.mst_solve_batched(vo, eo, src, dst, w, in_mst, total, status)
        if rc < 0:
            raise B.MstxError(rc)

    with knobs(base):
        run()
        torch.cuda.synchronize()
        ref = (in_mst.clone(), total.clone(), status.clone())

    def measure(s):
        with knobs(s):
            run()
            t = _event_ms(run, reps)
            torch.cuda.synchronize()
            same = (torch.equal(in_mst, ref[0]) and torch.equal(total.view(torch.int64), ref[1].view(torch.int64))
                    and torch.equal(status, ref[2]))
        if not same:
            raise RuntimeError(f"autotune: knob setting {s} changed the result of the batched solve")
        return t

    best, best_t, tried = coordinate_search(space, base, measure, passes)
    dflt = [t for s, t in tried if s == base]
    entry = {"knobs": best, "ms": best_t, "default_ms": dflt[0] if dflt else None, "graphs": G, "m": m,
             "candidates": len(tried)}
    doc = load_cache(path)
    doc["entries"].setdefault(device_key(), {})[batch_class(G, m)] = entry
    save_cache(doc, path)
    return entry


def lookup(cls: str, path: Optional[str] = None) -> Optional[Dict[str, int]]:
    """The cached knob settings of a workload class on this device, if any:
    from `path` (default: the user cache), else from the shipped file."""
    dev = device_key()
    for p in ([path] if path else [cache_path(), SHIPPED]):
        per_dev = load_cache(p)["entries"].get(dev)
        e = per_dev.get(cls) if isinstance(per_dev, dict) else None
        if isinstance(e, dict) and isinstance(e.get("knobs"), dict):  # a malformed entry is skipped
            return {k: int(v) for k, v in e["knobs"].items() if k in SETTERS}
    return None


@contextlib.contextmanager
def tuned_single(n: int, m: int, path: Optional[str] = None):
    """Applies the cached settings of the class of (n, m), if tuned, for the block."""
    s = lookup(single_class(n, m), path) or {}
    with knobs(s):
        yield s


@contextlib.contextmanager
def tuned_batched(num_graphs: int, sum_m: int, path: Optional[str] = None):
    """Applies the cached settings of the class of a batch, if tuned, for the block."""
    s = lookup(batch_class(num_graphs, sum_m), path) or {}
    with knobs(s):
        yield s


def search_space_size(space: Dict[str, List[int]]) -> int:
    return int(math.prod(len(v) for v in space.values()))


def main(argv=None) -> int:
    """Tunes the benchmark workloads on cuda:0 and writes the user cache (or,
    with --ship, the shipped file beside this module)."""
    import argparse

    import torch

    from . import graphgen as G

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--ship", action="store_true", help="write the shipped tuning.json beside this module")
    ap.add_argument("--workloads", default="random_n1M_d16,grid_1024x1024,rmat_s22_e26,batched_4096")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    path = SHIPPED if args.ship else cache_path()
    B.load_library()
    dev = torch.device("cuda:0")
    for wl in args.workloads.split(","):
        if wl.startswith("batched_"):
            b = G.batch(int(wl.split("_")[1]), seed=5)
            s, d, w = (torch.from_numpy(a).to(dev) for a in (b.src, b.dst, b.w))
            e = tune_batched(b.vertex_offsets, b.edge_offsets, s, d, w, reps=max(2, args.reps // 2), path=path)
        else:
            g = G.workload(wl)
            s, d, w = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.w))
            e = tune_single(g.n, s, d, w, reps=args.reps, path=path)
        print(json.dumps({"workload": wl, **e}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
