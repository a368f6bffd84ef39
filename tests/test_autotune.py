"""The autotuner's host logic (no GPU): workload classes, the cache file, the
knob context manager and the coordinate search, the last with a synthetic
timing function.  The GPU test (results byte-identical under every tuned
setting) is in test_gpu_autotune.py."""

import json

import pytest

from paper_2005_06913_amd import autotune as A


def test_classes():
    assert A.single_class(1 << 20, 1 << 23) == "single/n2^20/deg2^4"
    assert A.single_class(1000, 4000) == "single/n2^10/deg2^3"
    assert A.single_class(1, 0) == "single/n2^0/deg2^-1"
    assert A.batch_class(4096, 334_000_000) == "batched/g2^12/m2^29"


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "t.json")
    assert A.load_cache(p) == {"version": 1, "entries": {}}
    doc = A.load_cache(p)
    doc["entries"]["dev"] = {"single/n2^10/deg2^3": {"knobs": {"dense_limit": 64}, "ms": 1.0}}
    A.save_cache(doc, p)
    assert json.load(open(p))["entries"]["dev"]["single/n2^10/deg2^3"]["knobs"] == {"dense_limit": 64}
    open(p, "w").write("not json")
    assert A.load_cache(p)["entries"] == {}


def test_coordinate_search_finds_separable_optimum():
    space = {"a": (0, 1, 2, 3), "b": (10, 20, 30)}
    cost = lambda s: (s["a"] - 2) ** 2 + abs(s["b"] - 30) / 10.0 + 1.0
    calls = []

    def measure(s):
        calls.append(dict(s))
        return cost(s)

    best, t, tried = A.coordinate_search(space, {"a": 0, "b": 10}, measure, passes=2)
    assert best == {"a": 2, "b": 30} and t == 1.0
    # every setting measured once
    assert len(calls) == len({tuple(sorted(c.items())) for c in calls}) == len(tried)


def test_coordinate_search_propagates_mismatch():
    def measure(s):
        if s["a"] == 1:
            raise RuntimeError("result changed")
        return 1.0

    with pytest.raises(RuntimeError):
        A.coordinate_search({"a": (0, 1)}, {"a": 0}, measure)


def test_knobs_context_restores(monkeypatch):
    state = {"dense_limit": 200}

    def setter(v):
        prev = state["dense_limit"]
        if v >= 0:
            state["dense_limit"] = v
        return prev

    monkeypatch.setitem(A.SETTERS, "dense_limit", setter)
    with A.knobs({"dense_limit": 17}):
        assert state["dense_limit"] == 17
    assert state["dense_limit"] == 200
    with pytest.raises(ValueError):
        with A.knobs({"dense_limit": 5}):
            raise ValueError
    assert state["dense_limit"] == 200


def test_search_spaces_only_known_knobs():
    for space in (A.SINGLE_KNOBS, A.BATCH_KNOBS):
        assert set(space) <= set(A.SETTERS)
        assert A.search_space_size(space) > 1


def test_lookup_skips_malformed_entries(tmp_path, monkeypatch):
    monkeypatch.setattr(A, "device_key", lambda: "dev")
    p = str(tmp_path / "t.json")
    cls = "single/n2^10/deg2^3"
    for entry in ({cls: {"ms": 1.0}}, {cls: "x"}, "not a dict", {cls: {"knobs": [1]}}):
        A.save_cache({"version": 1, "entries": {"dev": entry}}, p)
        assert A.lookup(cls, p) is None
    A.save_cache({"version": 1, "entries": {"dev": {cls: {"knobs": {"dense_limit": 64, "unknown": 1}}}}}, p)
    assert A.lookup(cls, p) == {"dense_limit": 64}
