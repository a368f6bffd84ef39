"""The paper's CPU Boruvka variants (libmstx_cpu: sequential, sequential with
covered edges, parallel with permission words, parallel with compare-and-swap)
against the oracle, and a thread-sanitizer run of the parallel ones."""

import os
import subprocess

import numpy as np
import pytest

import gpu_cases
import mst_pins
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def C():
    from paper_2005_06913_amd import build, cpu_baselines
    if not os.path.exists(build.CPU_LIB):
        build.build_cpu_library()
    cpu_baselines.load_library()
    return cpu_baselines


def runs(C):
    for v in C.VARIANTS:
        for t in ((1,) if v in (C.MSTX_CPU_SEQ_PLAIN, C.MSTX_CPU_SEQ_COVERED) else (1, 3, 8)):
            yield v, t


@pytest.mark.parametrize("idx", range(len(gpu_cases.small_cases())))
def test_variants_match_oracle(C, idx):
    g = gpu_cases.small_cases()[idx]
    k = oracle.kruskal(g.n, g.src, g.dst, g.w)
    for v, t in runs(C):
        r = C.mst_cpu_solve(v, t, g.n, g.src, g.dst, g.w)
        assert r.status == k.status, (g.name, C.mst_cpu_variant_name(v), t)
        assert r.total == k.total, (g.name, C.mst_cpu_variant_name(v), t)
        assert np.array_equal(r.in_mst, k.in_mst), (g.name, C.mst_cpu_variant_name(v), t)


def test_variants_golden(C):
    """The paper's figure and the hand-checked fixtures."""
    for fx in mst_pins.all_fixtures():
        for v, t in runs(C):
            r = C.mst_cpu_solve(v, t, fx.n, fx.src, fx.dst, fx.w)
            assert r.status == fx.status and r.total == fx.total, (fx.name, v, t)
            assert np.array_equal(r.in_mst, fx.in_mst), (fx.name, v, t)


def test_sequential_rounds_match_oracle_boruvka(C):
    """Both sequential variants select the same edges per round as the oracle's Boruvka."""
    g = gpu_cases.small_cases()[0]
    b = oracle.boruvka(g.n, g.src, g.dst, g.w)
    for v in (C.MSTX_CPU_SEQ_PLAIN, C.MSTX_CPU_SEQ_COVERED):
        assert C.mst_cpu_solve(v, 1, g.n, g.src, g.dst, g.w).rounds == len(b.stats)


@pytest.mark.parametrize("case", gpu_cases.edge_cases(), ids=[c[0] for c in gpu_cases.edge_cases()])
def test_variants_edge_cases(C, case):
    name, n, src, dst, w = case
    k = oracle.kruskal(n, src, dst, w)
    for v, t in runs(C):
        r = C.mst_cpu_solve(v, t, n, src, dst, w)
        assert r.status == k.status, (name, v, t)
        if k.status >= 0:
            assert r.total == k.total and np.array_equal(r.in_mst, k.in_mst), (name, v, t)


def test_argument_errors(C):
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 5], np.int32)
    w = np.array([1, 2], np.uint32)
    assert C.mst_cpu_solve(C.MSTX_CPU_PAR_CAS, 2, 3, src, dst, w).status == -2  # vertex range
    assert C.mst_cpu_solve(7, 1, 6, src, dst, w).status == -1
    assert C.mst_cpu_solve(C.MSTX_CPU_PAR_LOCK, 0, 6, src, dst, w).status == -1
    assert C.mst_cpu_variant_name(C.MSTX_CPU_PAR_CAS) == "parallel_cas"
    assert C.mst_cpu_variant_name(9) == ""


def test_thread_sanitizer(tmp_path):
    """The parallel variants under -fsanitize=thread: no report, same trees."""
    exe = tmp_path / "tsan_driver"
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=thread", "-pthread", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "cpu_tsan_driver.cpp"),
           os.path.join(ROOT, "paper_2005_06913_amd", "csrc", "mstx_cpu.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in p.stderr, p.stderr[-3000:]
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout + p.stderr[-2000:]
