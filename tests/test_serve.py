"""Serving scheduler on the CPU with a fake executor backed by the oracle.

Checks continuous batching (requests that arrive while batches are running
are admitted by the next free slot), admission by memory budget, rejection
of requests that can never fit, and that every result is the oracle's.
"""

import threading
import time

import numpy as np

import oracle
from paper_2005_06913_amd import graphgen as G
from paper_2005_06913_amd import serve


class FakeExecutor:
    """Solves each request of a batch with the oracle after a short delay."""

    def __init__(self, delay=0.01):
        self.delay = delay
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.seen = []

    def batch_bytes(self, reqs, solo=False):
        return sum(r.data_bytes() + 64 * r.m for r in reqs)

    def execute(self, slot, reqs, solo=False):
        assert not solo or len(reqs) == 1
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.seen.append((slot, len(reqs), self.batch_bytes(reqs)))
        time.sleep(self.delay)
        for r in reqs:
            k = oracle.kruskal(r.n, r.src, r.dst, r.w)
            r.in_mst, r.total, r.status = k.in_mst, k.total, k.status
        with self.lock:
            self.active -= 1


def make_requests(k, seed=0, n_hi=3000):
    b = G.batch(k, seed=seed, n_lo=16, n_hi=n_hi)
    return [serve.Request(i, *(lambda g: (g.n, g.src, g.dst, g.w))(b.graph(i))) for i in range(k)]


def test_results_and_continuous_batching():
    ex = FakeExecutor(delay=0.02)
    srv = serve.MstServer(ex, slots=3, hbm_budget_bytes=3 << 30).start()
    reqs = make_requests(120, seed=1)
    wall = serve.poisson_replay(srv, reqs, qps=2000.0, seed=2)
    srv.close()
    for r in reqs:
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status == 0 and r.total == k.total
        assert np.array_equal(r.in_mst, k.in_mst)
    # arrivals outpace one 20 ms batch: later batches hold several requests, slots overlap
    assert max(len(b[1]) for b in srv.batches) > 1
    assert ex.max_active >= 2
    assert len({b[0] for b in srv.batches}) >= 2
    s = serve.latency_summary(reqs, wall)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_and_rejection():
    ex = FakeExecutor(delay=0.0)
    share_bytes = 4_000_000
    srv = serve.MstServer(ex, slots=2, hbm_budget_bytes=2 * share_bytes).start()
    reqs = make_requests(60, seed=3, n_hi=2000)
    huge = serve.Request(999, 50_000, *(lambda g: (g.src, g.dst, g.w))(G.tree_plus_extra(50_000, 200_000, 4)))
    reqs.append(huge)
    serve.poisson_replay(srv, reqs, qps=5000.0, seed=4)
    srv.close()
    assert huge.status == serve.MSTX_ERR_OUT_OF_MEMORY
    assert all(r.status == 0 for r in reqs[:-1])
    assert all(nbytes <= share_bytes for _, _, nbytes in ex.seen)
    assert srv.peak_in_flight_bytes <= 2 * share_bytes


def test_fifo_order_within_slot():
    ex = FakeExecutor(delay=0.005)
    srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=1 << 30).start()
    reqs = make_requests(40, seed=5)
    serve.poisson_replay(srv, reqs, qps=3000.0, seed=6)
    srv.close()
    order = [rid for _, ids in srv.batches for rid in ids]
    assert order == sorted(order)


def test_large_requests_run_alone_and_caps():
    ex = FakeExecutor(delay=0.002)
    srv = serve.MstServer(ex, slots=2, hbm_budget_bytes=1 << 30, solo_edges=20_000, batch_edges=30_000).start()
    reqs = make_requests(50, seed=7, n_hi=6000)
    serve.poisson_replay(srv, reqs, qps=5000.0, seed=8)
    srv.close()
    by_id = {r.rid: r for r in reqs}
    for _, ids in srv.batches:
        ms = [by_id[i].m for i in ids]
        if any(m >= 20_000 for m in ms):
            assert len(ids) == 1
        else:
            assert sum(ms) <= 30_000 or len(ids) == 1
    assert all(r.status == 0 for r in reqs)


class FailingExecutor(FakeExecutor):
    """Raises on every batch holding request 3; solves the others."""

    def execute(self, slot, reqs, solo=False):
        if any(r.rid == 3 for r in reqs):
            raise RuntimeError("device lost")
        super().execute(slot, reqs, solo)


def test_failed_batch_releases_slot_and_requests():
    """An executor that raises fails that batch's requests (device error status),
    frees its memory share and keeps the worker serving the rest."""
    ex = FailingExecutor(delay=0.005)
    srv = serve.MstServer(ex, slots=2, hbm_budget_bytes=1 << 30).start()
    reqs = make_requests(30, seed=4)
    serve.poisson_replay(srv, reqs, qps=500.0, seed=5)
    srv.close()
    assert srv.in_flight_bytes == 0
    assert srv.errors and any(3 in ids for _, ids, _ in srv.errors)
    failed = {rid for _, ids, _ in srv.errors for rid in ids}
    for r in reqs:
        if r.rid in failed:
            assert r.status == serve.MSTX_ERR_DEVICE and r.in_mst is None
        else:
            k = oracle.kruskal(r.n, r.src, r.dst, r.w)
            assert r.status == k.status == 0 and r.total == k.total
            assert np.array_equal(r.in_mst, k.in_mst)


class StepFakeExecutor(FakeExecutor):
    """FakeExecutor whose large requests run round by round: `rounds` rounds of
    `round_s` seconds each, the result from the oracle at the end."""

    def __init__(self, delay=0.002, rounds=8, round_s=0.01):
        super().__init__(delay)
        self.rounds, self.round_s = rounds, round_s

    def begin_solo(self, slot, r):
        ex = self

        class Job:
            def __init__(self):
                self.t0 = time.perf_counter()

            def advance(self):
                return time.perf_counter() - self.t0 >= ex.rounds * ex.round_s

            def finish(self):
                k = oracle.kruskal(r.n, r.src, r.dst, r.w)
                r.in_mst, r.total, r.status = k.in_mst, k.total, k.status

        return Job()


class WaitingStepExecutor(StepFakeExecutor):
    """StepFakeExecutor whose jobs also wait for their next round (no polling)."""

    def begin_solo(self, slot, r):
        job = super().begin_solo(slot, r)
        ex = self

        def wait_round():
            time.sleep(ex.round_s / 2)
            return job.advance()

        job.wait_round = wait_round
        return job


def test_round_granular_admission_waiting():
    """The same with the worker waiting for rounds instead of polling: small
    requests still run between the large request's rounds."""
    ex = WaitingStepExecutor(delay=0.002, rounds=10, round_s=0.01)
    srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=1 << 30, solo_edges=50_000).start()
    big_g = G.tree_plus_extra(20_000, 60_000, seed=11)
    big = serve.Request(1000, big_g.n, big_g.src, big_g.dst, big_g.w)
    srv.submit(big)
    time.sleep(0.02)
    small = make_requests(8, seed=12, n_hi=500)
    for r in small:
        srv.submit(r)
        time.sleep(0.003)
    for r in small + [big]:
        r.done.wait()
    srv.close()
    assert srv.interleaved and max(r.done_at for r in small) < big.done_at
    for r in small + [big]:
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status == 0 and r.total == k.total
        assert np.array_equal(r.in_mst, k.in_mst)


def test_round_granular_admission():
    """With one slot busy on a large request, small requests that arrive during
    it are solved between its rounds and finish before it does."""
    ex = StepFakeExecutor(delay=0.002, rounds=10, round_s=0.01)
    srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=1 << 30, solo_edges=50_000).start()
    big_g = G.tree_plus_extra(20_000, 60_000, seed=9)
    big = serve.Request(1000, big_g.n, big_g.src, big_g.dst, big_g.w)
    srv.submit(big)
    time.sleep(0.02)
    small = make_requests(12, seed=10, n_hi=500)
    for r in small:
        srv.submit(r)
        time.sleep(0.003)
    for r in small + [big]:
        r.done.wait()
    srv.close()
    assert srv.interleaved and all(big_id == 1000 for _, big_id, _ in srv.interleaved)
    assert max(r.done_at for r in small) < big.done_at
    for r in small + [big]:
        k = oracle.kruskal(r.n, r.src, r.dst, r.w)
        assert r.status == k.status == 0 and r.total == k.total
        assert np.array_equal(r.in_mst, k.in_mst)
    assert srv.in_flight_bytes == 0


class RoutingExecutor:
    """Records how each batch was run (alone or batched) and fills dummy results."""

    def __init__(self):
        self.runs = []  # (solo, [request ids])

    def batch_bytes(self, reqs, solo=False):
        return sum(r.data_bytes() for r in reqs)

    def execute(self, slot, reqs, solo=False):
        self.runs.append((solo, [r.rid for r in reqs]))
        for r in reqs:
            r.in_mst, r.total, r.status = None, 0, 0


def test_default_thresholds_route_by_edge_count():
    """With the default thresholds a request of fewer than 2^22 edges joins a
    batched call (several of them up to 2^23 edges in one) and one of 2^22
    edges or more is solved alone."""
    def req(rid, m):
        z = np.zeros(m, np.int32)
        return serve.Request(rid, 2, z, z, z.view(np.uint32))
    ex = RoutingExecutor()
    srv = serve.MstServer(ex, slots=1, hbm_budget_bytes=1 << 34)
    assert srv.solo_edges == 1 << 22 and srv.batch_edges == 1 << 23
    reqs = [req(0, 3_000_000), req(1, 3_000_000), req(2, 1_000_000), req(3, 5_000_000), req(4, 100)]
    for r in reqs:
        srv.submit(r)  # queued before the worker starts, so the split is deterministic
    srv.start()
    for r in reqs:
        r.done.wait()
    srv.close()
    assert ex.runs == [(False, [0, 1, 2]), (True, [3]), (False, [4])]
