"""Continuous-batching request loop over the batched sampler.

Requests (a circuit from |0...0>, a measured list and a shot count) arrive
over time. The server admits a request once its device working set fits in a
byte budget, and every free worker immediately takes *all* admitted requests
that are not yet running as one batch (`sq_batch_sample` on the worker's own
HIP stream). Requests that arrive while batches are on the GPU are admitted as
memory frees up and join the next batch; batches of different workers overlap
on the device. Each request's result is bit-for-bit what it gives alone (the
batched path is exact), which the tests check.

Nothing here computes simulation arithmetic: this module only schedules calls
into libsq.so.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import binding


def request_bytes(n: int, count: int, shots: int) -> int:
    """Device working set of one request in a batch: tableau (x and z
    columns), symbolic sign columns, affine forms, coins and outputs."""
    K = (n + 63) // 64
    Ls = (2 * K + 15) // 16 * 16
    Ks = (K + 15) // 16 * 16
    CW = (count + 63) // 64
    return 2 * n * Ls * 8 + (count + 1) * Ks * 8 + count * CW * 8 + 2 * shots * CW * 8 + 2 * count


@dataclass
class Request:
    rid: int
    n: int
    ops: np.ndarray
    qubits: np.ndarray
    shots: int
    seed: int = 0
    shot_begin: int = 0
    meas_base: int = 0
    arrival: float = 0.0          # seconds after the start of the run
    # filled by the server
    admitted: float = float("nan")
    started: float = float("nan")
    finished: float = float("nan")
    result: Optional[np.ndarray] = None
    bytes: int = 0

    def as_batch_dict(self) -> dict:
        return dict(n=self.n, ops=self.ops, qubits=self.qubits, shots=self.shots, seed=self.seed,
                    shot_begin=self.shot_begin, meas_base=self.meas_base)


@dataclass
class ServeStats:
    requests: int
    shots: int
    makespan_s: float
    shots_per_s: float
    latency_p50_s: float
    latency_p99_s: float
    batches: int
    mean_batch: float
    max_in_flight_bytes: int
    budget_bytes: int
    latencies: List[float] = field(default_factory=list)


class Server:
    def __init__(self, budget_bytes: int = 8 << 30, workers: int = 2, batch_kwargs: Optional[Dict] = None):
        self.budget = int(budget_bytes)
        self.workers = int(workers)
        self.batch_kwargs = dict(batch_kwargs or {})
        self._cv = threading.Condition()
        self._pending: List[Request] = []     # arrived, waiting for memory
        self._ready: List[Request] = []       # admitted, not yet running
        self._in_flight = 0
        self._max_in_flight = 0
        self._done = 0
        self._total = 0
        self._arrivals_over = False
        self._error: Optional[BaseException] = None
        self._batches: List[int] = []
        self._t0 = 0.0

    # -- admission ----------------------------------------------------------
    def _admit_locked(self, now: float):
        still = []
        for r in self._pending:
            if self._in_flight + r.bytes <= self.budget:
                self._in_flight += r.bytes
                self._max_in_flight = max(self._max_in_flight, self._in_flight)
                r.admitted = now
                self._ready.append(r)
            else:
                still.append(r)
        self._pending = still

    def _now(self) -> float:
        return time.perf_counter() - self._t0

    # -- workers ------------------------------------------------------------
    def _worker(self, stream):
        if stream is not None:
            import torch
            torch.cuda.set_device(0)
        while True:
            with self._cv:
                while True:
                    if self._error is not None:
                        return
                    if self._ready:
                        break
                    if self._arrivals_over and not self._pending:
                        return  # nothing left to start
                    self._cv.wait(timeout=0.05)
                batch, self._ready = self._ready, []
                now = self._now()
                for r in batch:
                    r.started = now
            try:
                outs = binding.batch_sample([r.as_batch_dict() for r in batch], stream=stream, **self.batch_kwargs)
            except BaseException as e:  # surface the first failure to run()
                with self._cv:
                    self._error = e
                    self._cv.notify_all()
                return
            with self._cv:
                now = self._now()
                for r, o in zip(batch, outs):
                    r.result = o
                    r.finished = now
                    self._in_flight -= r.bytes
                self._done += len(batch)
                self._batches.append(len(batch))
                self._admit_locked(now)
                self._cv.notify_all()

    # -- driver -------------------------------------------------------------
    def run(self, requests: List[Request], use_gpu_streams: bool = True) -> ServeStats:
        for r in requests:
            r.bytes = request_bytes(r.n, len(r.qubits), r.shots)
            if r.bytes > self.budget:  # could never be admitted
                raise binding.SqError(binding.SQ_ENOMEM,
                                      f"request {r.rid} needs {r.bytes} bytes, budget {self.budget}")
        order = sorted(requests, key=lambda r: r.arrival)
        self._total = len(order)
        if use_gpu_streams:
            import torch
            streams = [torch.cuda.Stream() for _ in range(self.workers)]
        else:
            streams = [None] * self.workers
        self._t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in streams]
        for th in threads:
            th.start()
        try:
            for r in order:
                delay = r.arrival - self._now()
                if delay > 0:
                    time.sleep(delay)
                with self._cv:
                    if self._error is not None:
                        break
                    self._pending.append(r)
                    self._admit_locked(self._now())
                    self._cv.notify_all()
        finally:
            with self._cv:
                self._arrivals_over = True
                self._cv.notify_all()
            for th in threads:
                th.join()
        if self._error is not None:
            raise self._error
        lat = [r.finished - r.arrival for r in order]
        shots = sum(r.shots for r in order)
        first = min(r.arrival for r in order)
        last = max(r.finished for r in order)
        span = max(last - first, 1e-9)
        return ServeStats(
            requests=len(order), shots=shots, makespan_s=span, shots_per_s=shots / span,
            latency_p50_s=float(np.percentile(lat, 50)), latency_p99_s=float(np.percentile(lat, 99)),
            batches=len(self._batches), mean_batch=float(np.mean(self._batches)) if self._batches else 0.0,
            max_in_flight_bytes=self._max_in_flight, budget_bytes=self.budget, latencies=lat)
