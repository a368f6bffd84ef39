"""Continuous-batching MST server on one GPU.

Requests (one graph each) arrive over time.  The server owns `slots` workers;
each worker has its own HIP stream, and therefore its own library workspace,
so the work of different slots overlaps on the device.  Whenever a worker is
free it takes work from the head of the queue, within its share of the
device-memory budget (admission by HBM budget):

* a request with at least `solo_edges` edges (default 2^22) fills the GPU
  by itself: it is solved alone, round by round (``mst_solve_begin`` / ``mst_solve_advance``
  / ``mst_solve_end``; with nothing to admit the worker sleeps in
  ``mst_solve_wait_round``), and between two of its Boruvka rounds the
  worker admits the small requests queued by then: it solves them with one
  ``mst_solve_batched`` call on the same stream, which the device runs
  after the rounds enqueued so far (round-granular admission: a small
  request waits for at most about two rounds of a large one, not for the
  whole solve);
* otherwise the worker takes the queued requests up to the next large one,
  at most `batch_edges` edges (default 2^23) and `max_batch` requests,
  copies them to the device and solves them with one ``mst_solve_batched``
  call.  Graphs of up to 65,536 vertices are solved there by one workgroup
  each and larger ones as one union per chunk, so requests of up to a few
  million edges go through fewer launches batched than alone: on a stream
  of graphs of 2^10 .. 2^20 vertices the defaults serve 2.3 times the
  solves per second of a 2^19 / 2^22 split.

Requests that arrive while other batches are on the GPU are admitted by the
next free worker, or between the rounds of a large solve: batching is
continuous, not a queue in front of a single solver, and the caps keep
several workers busy at once.

A request's arrays are host arrays (numpy; the executor copies them to the
device on the slot's stream and the flags back) or device tensors already
in HBM, e.g. written by an earlier GPU stage (then nothing crosses PCIe but
the per-request total and status, and the flags stay on the device as a
view of the batch's output).

Every request's result is exactly the minimum spanning forest of its graph
(a disjoint union of graphs has the union of their forests as its forest),
so it is the same whether solved alone or in a mix; ``tests/test_serve.py``
and ``tests/test_gpu_serve.py`` check that.

The scheduling logic is independent of the device: an executor object does
the solving (``GpuExecutor`` here; the CPU tests use one backed by the
oracle).  ``PlainServer`` is the baseline: one request at a time, one
``mst_solve`` per request.
"""

from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

MSTX_ERR_OUT_OF_MEMORY = -4
MSTX_ERR_DEVICE = -5


@dataclass
class Request:
    """One MST query: a graph with local vertex ids [0, n)."""

    rid: int
    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    w: np.ndarray  # uint32 [m]
    arrival: float = 0.0  # time.perf_counter() when submitted
    # filled in on completion
    in_mst: np.ndarray | None = None
    total: int = 0
    status: int = 0
    done_at: float = 0.0
    batch_size: int = 0
    slot: int = -1
    done: threading.Event = field(default_factory=threading.Event)
    # resident requests: an event recorded on the submitting thread's current
    # stream at submit(); the solve's stream waits for it before reading the
    # arrays, so they may still be being written by work enqueued before submit
    ready: object = None

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def resident(self) -> bool:
        """The graph's arrays are device tensors (no host-to-device copy).

        A resident request's in_mst is a view of a tensor the server allocated
        on one of its streams; a caller that uses it on another stream calls
        ``record_stream`` on it, as for any tensor shared between streams."""
        return bool(getattr(self.src, "is_cuda", False))

    def mark_submitted(self) -> None:
        """Arrival time, and for a resident request the event its solve waits for."""
        self.arrival = time.perf_counter()
        if self.resident:
            import torch

            self.ready = torch.cuda.Event()
            self.ready.record(torch.cuda.current_stream(self.src.device))

    def wait_ready(self, stream) -> None:
        """Orders `stream` after the work that wrote a resident request's arrays."""
        if self.ready is not None:
            stream.wait_event(self.ready)

    def flags(self) -> np.ndarray:
        """in_mst as a host array (copied from the device for a resident request)."""
        f = self.in_mst
        return f.cpu().numpy() if hasattr(f, "cpu") else f

    @property
    def latency(self) -> float:
        return self.done_at - self.arrival

    def data_bytes(self) -> int:
        """Device bytes of the request's graph and outputs (src, dst, w, flags)."""
        return 13 * self.m + 16


def batch_offsets(reqs):
    vo = np.zeros(len(reqs) + 1, np.int64)
    eo = np.zeros(len(reqs) + 1, np.int64)
    for i, r in enumerate(reqs):
        vo[i + 1] = vo[i] + r.n
        eo[i + 1] = eo[i] + r.m
    return vo, eo


class GpuExecutor:
    """Solves batches on the GPU with ``mst_solve_batched``, one stream per slot."""

    def __init__(self, slots: int, device=None):
        import torch

        from . import binding as B

        self.torch = torch
        self.B = B
        self.dev = device or torch.device("cuda:0")
        B.load_library()
        # streams keep the default priority
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]

    def batch_bytes(self, reqs, solo: bool = False) -> int:
        if solo:
            (r,) = reqs
            return r.data_bytes() + self.B.mst_workspace_bytes(r.n, r.m)
        vo, eo = batch_offsets(reqs)
        return sum(r.data_bytes() for r in reqs) + self.B.mst_batched_workspace_bytes(vo, eo)

    def begin_solo(self, slot: int, r):
        """Starts the round-by-round solve of one large request on the slot's stream."""
        return _SoloJob(self, slot, r)

    def _tensor(self, a):
        """A request array as a tensor: device tensors as they are, host arrays wrapped."""
        return a if isinstance(a, self.torch.Tensor) else self.torch.from_numpy(a)

    def _on_device(self, a):
        """A request array on the device (host arrays copied on the current stream)."""
        return a if isinstance(a, self.torch.Tensor) else self.torch.from_numpy(a).to(self.dev, non_blocking=True)

    def execute(self, slot: int, reqs, solo: bool = False) -> None:
        torch = self.torch
        stream = self.streams[slot]
        if solo:
            (r,) = reqs
            with torch.cuda.stream(stream):
                r.wait_ready(stream)
                src, dst, w = (self._on_device(a) for a in (r.src, r.dst, r.w))
                in_mst = torch.empty(r.m, dtype=torch.uint8, device=self.dev)
                total = torch.empty(1, dtype=torch.uint64, device=self.dev)
                r.status = self.B.mst_solve(r.n, src, dst, w, in_mst, total, stream)
                r.total = int(total.view(torch.int64).cpu().item())  # waits for the solve
                r.in_mst = in_mst if r.resident else in_mst.cpu().numpy()
            return
        vo, eo = batch_offsets(reqs)
        m = int(eo[-1])
        G = len(reqs)
        with torch.cuda.stream(stream):
            for r in reqs:
                r.wait_ready(stream)
            if all(r.resident for r in reqs):
                # one concatenation per array inside HBM (weights as int32 bits)
                src = torch.cat([r.src for r in reqs])
                dst = torch.cat([r.dst for r in reqs])
                w = torch.cat([r.w.view(torch.int32) for r in reqs]).view(torch.uint32)
            else:
                src = torch.empty(m, dtype=torch.int32, device=self.dev)
                dst = torch.empty(m, dtype=torch.int32, device=self.dev)
                w = torch.empty(m, dtype=torch.uint32, device=self.dev)
                for r, a in zip(reqs, eo[:-1]):
                    a = int(a)
                    # host arrays cross PCIe here; device arrays are copied inside HBM
                    src[a:a + r.m].copy_(self._tensor(r.src), non_blocking=True)
                    dst[a:a + r.m].copy_(self._tensor(r.dst), non_blocking=True)
                    w[a:a + r.m].copy_(self._tensor(r.w), non_blocking=True)
            in_mst = torch.empty(m, dtype=torch.uint8, device=self.dev)
            total = torch.empty(G, dtype=torch.uint64, device=self.dev)
            status = torch.empty(G, dtype=torch.int32, device=self.dev)
            rc = self.B.mst_solve_batched(vo, eo, src, dst, w, in_mst, total, status, stream)
            if rc < 0:
                for r in reqs:
                    r.status = rc
                return
            tot = total.view(torch.int64).cpu().numpy()  # waits for the solve
            st = status.cpu().numpy()
            host_flags = in_mst.cpu().numpy() if not all(r.resident for r in reqs) else None
        for i, r in enumerate(reqs):
            a, b = int(eo[i]), int(eo[i + 1])
            r.in_mst = in_mst[a:b] if r.resident else host_flags[a:b]
            r.total = int(tot[i])
            r.status = int(st[i])

    def release(self):
        for s in self.streams:
            self.B.mst_workspace_release(s)


class _SoloJob:
    """One request solved round by round on a slot's stream (GpuExecutor.begin_solo)."""

    def __init__(self, ex: GpuExecutor, slot: int, r):
        torch = ex.torch
        self.ex, self.r, self.stream = ex, r, ex.streams[slot]
        with torch.cuda.stream(self.stream):
            r.wait_ready(self.stream)
            self.src, self.dst, self.w = (ex._on_device(a) for a in (r.src, r.dst, r.w))
            self.in_mst = torch.empty(r.m, dtype=torch.uint8, device=ex.dev)
            self.total = torch.empty(1, dtype=torch.uint64, device=ex.dev)
            st, self.h = ex.B.mst_solve_begin(r.n, self.src, self.dst, self.w, self.in_mst, self.total, self.stream)
        if st < 0:
            raise ex.B.MstxError(st)

    def advance(self) -> bool:
        """True once the solve has ended (its next round is enqueued otherwise)."""
        return self.h is None or self.ex.B.mst_solve_advance(self.h)

    def wait_round(self) -> bool:
        """Waits for the next round to finish (the host thread sleeps in the
        library, the interpreter lock released); True once the solve has ended."""
        return self.h is None or self.ex.B.mst_solve_wait_round(self.h)

    def finish(self) -> None:
        r, torch = self.r, self.ex.torch
        if self.h is not None:
            r.status = self.ex.B.mst_solve_end(self.h)
            self.h = None
        else:
            r.status = 0
        with torch.cuda.stream(self.stream):
            r.total = int(self.total.view(torch.int64).cpu().item())  # waits for the solve
            r.in_mst = self.in_mst if r.resident else self.in_mst.cpu().numpy()


class MstServer:
    """Continuous batching over `executor` with `slots` concurrent workers.

    hbm_budget_bytes is the device memory all in-flight batches may use
    together; each worker forms its batch within an equal share.  A request
    that does not fit a share on its own is rejected (status
    MSTX_ERR_OUT_OF_MEMORY) instead of blocking the queue.
    """

    def __init__(self, executor, slots: int = 3, hbm_budget_bytes: int = 64 << 30, max_batch: int = 1024,
                 solo_edges: int = 1 << 22, batch_edges: int = 1 << 23, step_poll_s: float = 2e-4):
        self.ex = executor
        self.step_poll_s = step_poll_s  # poll interval for executors whose jobs cannot wait for a round
        self.slots = slots
        self.share = hbm_budget_bytes // slots
        self.max_batch = max_batch
        self.solo_edges = solo_edges
        self.batch_edges = batch_edges
        self.queue: collections.deque = collections.deque()
        self.cv = threading.Condition()
        self.stop = False
        self.workers = []
        self.batches = []  # (slot, request ids) log for tests
        self.interleaved = []  # (slot, large request id, request ids run between its rounds)
        self.errors = []  # (slot, request ids, exception) of batches whose execution raised
        self.in_flight_bytes = 0
        self.peak_in_flight_bytes = 0

    def start(self):
        for s in range(self.slots):
            t = threading.Thread(target=self._worker, args=(s,), daemon=True)
            t.start()
            self.workers.append(t)
        return self

    def submit(self, req: Request) -> Request:
        req.mark_submitted()
        with self.cv:
            self.queue.append(req)
            self.cv.notify()
        return req

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.workers:
            t.join()

    def _take_small(self, budget: int):
        """Small requests from the head of the queue that fit `budget` bytes (lock
        held): (requests, bytes).  Stops at the first large request."""
        batch, used, edges = [], 0, 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            if r.m >= self.solo_edges or edges + r.m > self.batch_edges:
                break
            need = self.ex.batch_bytes(batch + [r])
            if need > budget:
                break
            batch.append(self.queue.popleft())
            used, edges = need, edges + r.m
        return batch, used

    def _take_batch(self):
        """Work for one worker from the head of the queue (called with the lock held):
        (requests, bytes, solo)."""
        while self.queue:
            r = self.queue[0]
            solo = r.m >= self.solo_edges
            need = self.ex.batch_bytes([r], solo)
            if need <= self.share:
                break
            self.queue.popleft()  # can never fit: reject rather than block the queue
            r.status = MSTX_ERR_OUT_OF_MEMORY
            r.done_at = time.perf_counter()
            r.done.set()
        else:
            return [], 0, False
        if solo:
            return [self.queue.popleft()], need, True
        batch, used, edges = [self.queue.popleft()], need, r.m
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            if r.m >= self.solo_edges or edges + r.m > self.batch_edges:
                break
            need = self.ex.batch_bytes(batch + [r])
            if need > self.share:
                break
            batch.append(self.queue.popleft())
            used, edges = need, edges + r.m
        return batch, used, False

    def _worker(self, slot: int):
        while True:
            with self.cv:
                while not self.queue and not self.stop:
                    self.cv.wait()
                if self.stop and not self.queue:
                    return
                batch, used, solo = self._take_batch()
                self.in_flight_bytes += used
                self.peak_in_flight_bytes = max(self.peak_in_flight_bytes, self.in_flight_bytes)
            if not batch:
                continue
            if solo and hasattr(self.ex, "begin_solo"):
                self._run_stepwise(slot, batch[0], used)
            else:
                self._run_batch(slot, batch, used, solo)

    def _fail(self, slot, batch, exc):
        code = getattr(exc, "status", MSTX_ERR_DEVICE)
        for r in batch:
            r.status = code if isinstance(code, int) and code < 0 else MSTX_ERR_DEVICE
            r.in_mst = None
            r.total = 0
        self.errors.append((slot, [r.rid for r in batch], repr(exc)))

    def _complete(self, slot, batch, used):
        now = time.perf_counter()
        with self.cv:
            self.in_flight_bytes -= used
            self.batches.append((slot, [r.rid for r in batch]))
        for r in batch:
            r.done_at = now
            r.batch_size = len(batch)
            r.slot = slot
            r.done.set()

    def _run_batch(self, slot, batch, used, solo=False):
        try:
            self.ex.execute(slot, batch, solo)
        except Exception as exc:  # a failed batch fails its requests, not the worker
            self._fail(slot, batch, exc)
        finally:
            self._complete(slot, batch, used)

    def _run_stepwise(self, slot, r, used):
        """One large request round by round; the small requests queued between two
        of its rounds run on this slot then, within what is left of its share.
        With nothing to admit the worker waits for the next round inside the
        library (no polling), so a small request waits for at most about one
        round of the large one."""
        try:
            job = self.ex.begin_solo(slot, r)
            wait = getattr(job, "wait_round", None)
            done = job.advance()
            while not done:
                with self.cv:
                    small, sused = self._take_small(self.share - used)
                    if small:
                        self.in_flight_bytes += sused
                        self.peak_in_flight_bytes = max(self.peak_in_flight_bytes, self.in_flight_bytes)
                    elif wait is None:
                        self.cv.wait(timeout=self.step_poll_s)
                if small:
                    self.interleaved.append((slot, r.rid, [x.rid for x in small]))
                    self._run_batch(slot, small, sused)
                    done = job.advance()
                else:
                    done = wait() if wait is not None else job.advance()
            job.finish()
        except Exception as exc:
            self._fail(slot, [r], exc)
        finally:
            self._complete(slot, [r], used)


class PlainServer:
    """Baseline: one worker, one request at a time, one ``mst_solve`` per request."""

    def __init__(self, device=None):
        import torch

        from . import binding as B

        self.torch = torch
        self.B = B
        self.dev = device or torch.device("cuda:0")
        B.load_library()
        self.queue: collections.deque = collections.deque()
        self.cv = threading.Condition()
        self.stop = False
        self.stream = torch.cuda.Stream(device=self.dev)
        self.worker = None

    def start(self):
        self.worker = threading.Thread(target=self._run, daemon=True)
        self.worker.start()
        return self

    def submit(self, req: Request) -> Request:
        req.mark_submitted()
        with self.cv:
            self.queue.append(req)
            self.cv.notify()
        return req

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        self.worker.join()

    def _run(self):
        torch = self.torch
        while True:
            with self.cv:
                while not self.queue and not self.stop:
                    self.cv.wait()
                if self.stop and not self.queue:
                    return
                r = self.queue.popleft()
            with torch.cuda.stream(self.stream):
                r.wait_ready(self.stream)
                src, dst, w = (a if isinstance(a, torch.Tensor) else torch.from_numpy(a).to(self.dev, non_blocking=True)
                               for a in (r.src, r.dst, r.w))
                in_mst = torch.empty(r.m, dtype=torch.uint8, device=self.dev)
                total = torch.empty(1, dtype=torch.uint64, device=self.dev)
                r.status = self.B.mst_solve(r.n, src, dst, w, in_mst, total, self.stream)
                r.total = int(total.view(torch.int64).cpu().item())  # waits for the solve
                r.in_mst = in_mst if r.resident else in_mst.cpu().numpy()
            r.done_at = time.perf_counter()
            r.batch_size = 1
            r.done.set()


def poisson_replay(server, requests, qps: float, seed: int = 0):
    """Submit `requests` with exponential inter-arrival times (rate qps) and wait for all."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, len(requests))
    t0 = time.perf_counter()
    due = t0 + np.cumsum(gaps)
    for r, t in zip(requests, due):
        delay = t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
    for r in requests:
        r.done.wait()
    return time.perf_counter() - t0


def latency_summary(requests, wall_s: float) -> dict:
    lat = np.array([r.latency for r in requests]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "solves_per_s": len(requests) / wall_s,
            "mean_batch": float(np.mean([r.batch_size for r in requests]))}
