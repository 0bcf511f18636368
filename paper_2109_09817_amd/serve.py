"""Continuous-batching prediction server over a resident GP model.

Requests (one molecule's pair-feature rows each) arrive at any time.  A
scheduler thread packs queued requests into batches and launches each batch on
one of S execution slots (a HIP stream with its own pre-allocated device
buffers and workspace): a request that arrives while other batches are on the
GPU joins the next batch as soon as a slot and memory budget are free, so the
work of several batches overlaps on the device.  Each row's result is
independent of the other rows of its batch (the library fixes the reduction
order per row), so a request gets bitwise the same answer alone or in a mix.

The executor that runs a batch is pluggable: ``GpuExecutor`` calls
``gp_predict_run`` through a ``gp.PredictModel``; tests use a CPU executor.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future
from typing import Callable, Deque, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rows: np.ndarray  # (m, d) float64
    future: Future
    t_arrival: float
    rid: int


@dataclasses.dataclass
class Result:
    mean: np.ndarray
    var: Optional[np.ndarray]
    latency_s: float
    batch_rows: int


class Executor:
    """Runs batches on slots.  launch() must not block on the device."""

    slots: int
    max_rows: int

    def batch_bytes(self, m: int) -> int:
        raise NotImplementedError

    def launch(self, slot: int, Z: np.ndarray):
        raise NotImplementedError

    def ready(self, slot: int) -> bool:
        raise NotImplementedError

    def fetch(self, slot: int, m: int):
        """(mean, var) host arrays of the finished batch on `slot`."""
        raise NotImplementedError


class GpuExecutor(Executor):
    """Slots = HIP streams with pinned staging buffers and a fixed device workspace each."""

    def __init__(self, model, slots: int = 4, max_rows: int = 2048):
        import torch
        self.torch = torch
        self.model = model
        self.slots = slots
        self.max_rows = max_rows
        dev = model.device
        d = model.kern.d
        self.with_var = model.kc > 0
        self.ws_bytes = model.workspace_bytes(max_rows)
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(slots)]
        self.ws = [torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev) for _ in range(slots)]
        self.zdev = [torch.empty((max_rows, d), dtype=torch.float64, device=dev) for _ in range(slots)]
        self.mdev = [torch.empty(max_rows, dtype=torch.float64, device=dev) for _ in range(slots)]
        self.vdev = [torch.empty(max_rows, dtype=torch.float64, device=dev) for _ in range(slots)]
        self.zpin = [torch.empty((max_rows, d), dtype=torch.float64).pin_memory() for _ in range(slots)]
        self.mpin = [torch.empty(max_rows, dtype=torch.float64).pin_memory() for _ in range(slots)]
        self.vpin = [torch.empty(max_rows, dtype=torch.float64).pin_memory() for _ in range(slots)]
        self.events = [None] * slots

    def batch_bytes(self, m: int) -> int:
        return self.model.workspace_bytes(m) + m * (self.model.kern.d + 2) * 8

    def launch(self, slot: int, Z: np.ndarray):
        torch = self.torch
        m = Z.shape[0]
        self.zpin[slot][:m].numpy()[:] = Z
        st = self.streams[slot]
        with torch.cuda.stream(st):
            self.zdev[slot][:m].copy_(self.zpin[slot][:m], non_blocking=True)
            mean, var = self.model(self.zdev[slot][:m], with_var=self.with_var, ws=self.ws[slot],
                                   mean=self.mdev[slot][:m], var=self.vdev[slot][:m] if self.with_var else None,
                                   stream=st)
            self.mpin[slot][:m].copy_(mean, non_blocking=True)
            if self.with_var:
                self.vpin[slot][:m].copy_(var, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.events[slot] = ev

    def ready(self, slot: int) -> bool:
        return self.events[slot] is not None and self.events[slot].query()

    def fetch(self, slot: int, m: int):
        self.events[slot].synchronize()
        self.events[slot] = None
        mean = self.mpin[slot][:m].numpy().copy()
        var = self.vpin[slot][:m].numpy().copy() if self.with_var else None
        return mean, var


class Server:
    """Admission by slot, row cap and memory budget; FIFO order; continuous batching."""

    def __init__(self, executor: Executor, d: int, hbm_budget: int = 2 << 30, poll_s: float = 5e-5,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.d = d
        self.budget = int(hbm_budget)
        self.poll_s = poll_s
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.cv = threading.Condition()
        self.inflight = {}  # slot -> (requests, offsets, rows, bytes)
        self.used = 0
        self.stop = False
        self.error = None  # what stopped the scheduler thread, if anything did
        self.next_id = 0
        self.completed = 0
        self.batches = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # -- client side
    def submit(self, rows) -> Future:
        fut: Future = Future()
        Z = np.ascontiguousarray(np.asarray(rows, dtype=np.float64))
        if Z.ndim != 2 or Z.shape[1] != self.d or Z.shape[0] < 1 or Z.shape[0] > self.ex.max_rows:
            fut.set_exception(ValueError(f"request must be (m, {self.d}) with 1 <= m <= {self.ex.max_rows}"))
            return fut
        if not np.all(np.isfinite(Z)):
            fut.set_exception(ValueError("request rows must be finite"))
            return fut
        with self.cv:
            if self.stop:
                fut.set_exception(RuntimeError("prediction server is closed"))
                return fut
            req = Request(Z, fut, self.clock(), self.next_id)
            self.next_id += 1
            self.queue.append(req)
            self.cv.notify()
        return fut

    def close(self):
        """Drain the queue and stop; raises what stopped the scheduler, if it died."""
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()
        if self.error is not None:
            raise RuntimeError("prediction server stopped on a scheduler failure") from self.error

    # -- scheduler
    def _complete(self, slot):
        reqs, offs, m, nbytes = self.inflight.pop(slot)
        self.used -= nbytes
        try:
            mean, var = self.ex.fetch(slot, m)
        except Exception as e:  # a batch whose device work failed fails its own requests only
            for r in reqs:
                if not r.future.done():
                    r.future.set_exception(e)
            return
        now = self.clock()
        for r, o in zip(reqs, offs):
            k = r.rows.shape[0]
            res = Result(mean[o:o + k].copy(), None if var is None else var[o:o + k].copy(), now - r.t_arrival, m)
            r.future.set_result(res)
        self.completed += len(reqs)

    def _admit(self, slot) -> bool:
        batch: List[Request] = []
        rows = 0
        while self.queue:
            r = self.queue[0]
            k = r.rows.shape[0]
            if rows + k > self.ex.max_rows:
                break
            if self.used + self.ex.batch_bytes(rows + k) > self.budget and batch:
                break
            batch.append(self.queue.popleft())
            rows += k
        if not batch:
            return False
        nbytes = self.ex.batch_bytes(rows)
        if self.used + nbytes > self.budget and self.inflight:
            # over budget: wait for a running batch to finish (keep FIFO order)
            for r in reversed(batch):
                self.queue.appendleft(r)
            return False
        Z = np.concatenate([r.rows for r in batch], axis=0)
        offs = np.cumsum([0] + [r.rows.shape[0] for r in batch[:-1]]).tolist()
        try:
            self.ex.launch(slot, Z)
        except Exception as e:  # a failing batch fails its own requests only
            for r in batch:
                r.future.set_exception(e)
            return True
        self.inflight[slot] = (batch, offs, rows, nbytes)
        self.used += nbytes
        self.batches += 1
        return True

    def _loop(self):
        try:
            self._schedule()
        except BaseException as e:  # the scheduler cannot go on: no client may wait forever
            with self.cv:
                self.stop = True
                self.error = e
                pending = [r for reqs, _, _, _ in self.inflight.values() for r in reqs] + list(self.queue)
                self.inflight.clear()
                self.queue.clear()
            for r in pending:
                if not r.future.done():
                    r.future.set_exception(RuntimeError(f"prediction server stopped: {e!r}"))

    def _schedule(self):
        while True:
            with self.cv:
                if self.stop and not self.queue and not self.inflight:
                    return
                for slot in list(self.inflight):
                    if self.ex.ready(slot):
                        self._complete(slot)
                progressed = False
                for slot in range(self.ex.slots):
                    if slot not in self.inflight and self.queue:
                        progressed |= self._admit(slot)
                if not progressed:
                    # poll the running batches; with none, sleep until a request or close() arrives
                    self.cv.wait(timeout=self.poll_s if self.inflight else None)


def latency_summary(results: List[Result], wall_s: float) -> dict:
    lat = np.array([r.latency_s for r in results]) * 1e3
    rows = sum(r.mean.shape[0] for r in results)
    return {
        "requests": len(results),
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "max_ms": float(lat.max()) if len(lat) else None,
        "predictions_per_s": rows / wall_s if wall_s > 0 else None,
        "requests_per_s": len(results) / wall_s if wall_s > 0 else None,
        "mean_batch_rows": float(np.mean([r.batch_rows for r in results])) if results else None,
    }
