"""The committed bench lines (profiles/bench_*.json) keep the line contract:
the common keys and their types, one GPU, the roofline's fraction equal to
achieved / peak, the value equal to the work over the time per step, parity
recorded for the single-graph lines, and the oracle baseline on the headline.
The CPU context line (the paper's own variants) is checked against the
speedup the paper reports."""

import glob
import json
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LINES = sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.json")))
GPU_LINES = [p for p in LINES if not p.endswith("bench_cpu_context.json")]


def load(path):
    with open(path) as f:
        return json.load(f)


def workload_of(path):
    return os.path.basename(path)[len("bench_"):-len(".json")]


@pytest.mark.parametrize("path", GPU_LINES, ids=workload_of)
def test_common_keys(path):
    d = load(path)
    for k, t in (("metric", str), ("unit", str), ("dtype", str), ("data", str), ("config", dict),
                 ("steps", int), ("warmup", int), ("n_gpus", int), ("higher_is_better", bool), ("scaling", str)):
        assert isinstance(d.get(k), t), k
    assert isinstance(d["value"], (int, float)) and d["value"] > 0
    assert isinstance(d["ms_per_step"], (int, float)) and d["ms_per_step"] > 0
    assert d["n_gpus"] == 1 and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["data"] == "synthetic"
    assert d["config"]["workload"].startswith(workload_of(path) + ":")


@pytest.mark.parametrize("path", GPU_LINES, ids=workload_of)
def test_roofline(path):
    r = load(path)["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu")
    if r["bound"] == "hbm":
        assert r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0 < r["achieved"] <= r["peak"]
    assert math.isclose(r["frac"], r["achieved"] / r["peak"], rel_tol=1e-9)
    assert r["traffic"] is None or r["traffic"] > 0


@pytest.mark.parametrize("path", [p for p in GPU_LINES if load(p)["unit"] == "edges/s"], ids=workload_of)
def test_single_graph_lines(path):
    d = load(path)
    m = d["config"]["m"]
    assert math.isclose(d["value"], m / (d["ms_per_step"] * 1e-3), rel_tol=1e-9)
    assert d.get("parity_vs_oracle", d.get("parity_vs_closed_form")) is True
    per_step = sum(r["us_per_step"] for r in d["per_round"]) * 1e-3
    # the event-timed rounds cover the solve (events add a few µs per launch)
    assert 0.8 * d["ms_per_step"] < per_step < 1.5 * d["ms_per_step"]


def test_headline_line():
    d = load(os.path.join(ROOT, "profiles", "bench_random_n1M_d16.json"))
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert cb["unit"] == d["unit"] and isinstance(cb["sample"], str) and cb["sample"]
    assert d["roofline"]["traffic"] is not None  # counter traffic of the dominant kernel
    assert d["dtype"] == "u32"


def test_cpu_context_line():
    d = load(os.path.join(ROOT, "profiles", "bench_cpu_context.json"))
    assert d["unit"] == "x" and d["value"] > 0 and d["n_gpus"] == 1
    # the paper's CAS variant: 2.03x over the sequential one at four threads
    assert math.isclose(d["vs_baseline"], d["value"] / 2.03, rel_tol=1e-9)
    assert d["config"]["workload"].startswith("cpu_context:")
