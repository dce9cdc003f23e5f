"""Continuous-batching request loop over libsq.so.

Two kinds of work share one device-memory budget and a pool of workers, each
with its own HIP stream:

* one-shot circuits (``CircuitRequest``: a circuit from |0...0>, a measured
  list and a shot count): every free worker takes all admitted circuits not
  yet running as one batch (``sq_batch_sample``), so circuits that arrive
  while other batches are on the GPU join the next batch and batches of
  different workers overlap on the device;
* sessions, tableaux kept resident on the device between requests:
  ``OpenSession`` creates one and applies its circuit, ``SampleRequest`` and
  ``MeasureRequest`` act on it, ``CloseSession`` frees it. A session's
  requests run in arrival order, one at a time; sampling requests queued
  back to back on the same measured list are served together by one
  ``sq_sample_many`` call, which runs the measurement sweep once for all of
  them (only the coins differ between them).

Admission: a request is admitted once the bytes it holds on the device fit
in the budget next to those in flight (the library's own figures:
``sq_batch_item_bytes``, ``sq_bytes_required``, ``sq_sample_bytes``). A
session's tableau stays counted until the session closes. A request that can
never fit is refused on its own, at once. Failures stay local: a batch whose
library call fails fails only its own requests and frees their bytes; a
request can be cancelled until a worker takes it; a request still waiting at
its deadline fails with ``DeadlineExceeded``. Latency is completion minus
arrival; the loop reports p50/p99 beside throughput.

Nothing here computes simulation arithmetic: this module only schedules calls
into libsq.so (through ``backend``), and every result equals the same request
run alone, which the tests check.
"""
from __future__ import annotations

import itertools
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

from . import binding


class DeadlineExceeded(RuntimeError):
    """A request was still waiting for a worker at its deadline."""


class Cancelled(RuntimeError):
    """A request was cancelled before a worker took it."""


class Refused(RuntimeError):
    """A request can never fit in the server's device-memory budget."""


# ---------------------------------------------------------------- backend
class GpuBackend:
    """The libsq calls the server makes, on the worker's stream."""

    def circuit_bytes(self, r: "CircuitRequest", batch_kwargs: dict) -> int:
        return binding.batch_item_bytes(r.n, len(r.ops), len(r.qubits), r.shots,
                                        block=batch_kwargs.get("block", 0),
                                        max_batch_n=batch_kwargs.get("max_batch_n", 0))

    def tableau_bytes(self, n: int) -> int:
        return binding.bytes_required(n)

    def sample_bytes(self, n: int, count: int, shots: int) -> int:
        return binding.sample_bytes(n, count, shots)

    def batch_sample(self, items: List[dict], stream, batch_kwargs: dict) -> List[np.ndarray]:
        return binding.batch_sample(items, stream=stream, **batch_kwargs)

    def open(self, n: int, ops, stream):
        t = binding.Tableau(n, stream=stream)
        try:
            if ops is not None and len(ops):
                t.apply_gates(ops)
            t.sync()
        except BaseException:
            t.close()
            raise
        return t

    def sample_many(self, handle, qubits, sets: List[dict]) -> List[np.ndarray]:
        return handle.sample_many(qubits, sets)

    def measure(self, handle, qubits, seed: int, shot: int, meas_base: int):
        return handle.measure(qubits, seed=seed, shot=shot, meas_base=meas_base)

    def close(self, handle):
        handle.close()


# ---------------------------------------------------------------- requests
_rids = itertools.count()


@dataclass
class _Base:
    arrival: float = 0.0               # seconds after the start of the run
    deadline: Optional[float] = None   # seconds after the start; must be taken by a worker before it
    rid: int = field(default_factory=lambda: next(_rids))
    # filled by the server
    bytes: int = 0
    admitted: float = float("nan")
    started: float = float("nan")
    finished: float = float("nan")
    result: Any = None
    error: Optional[BaseException] = None
    state: str = "new"   # new, pending, ready, running, done, failed, cancelled

    @property
    def ok(self) -> bool:
        return self.state == "done"


@dataclass
class CircuitRequest(_Base):
    n: int = 0
    ops: np.ndarray = None
    qubits: np.ndarray = None
    shots: int = 0
    seed: int = 0
    shot_begin: int = 0
    meas_base: int = 0

    def as_batch_dict(self) -> dict:
        return dict(n=self.n, ops=self.ops, qubits=self.qubits, shots=self.shots, seed=self.seed,
                    shot_begin=self.shot_begin, meas_base=self.meas_base)


# The one-shot request of earlier versions of this module.
Request = CircuitRequest


@dataclass
class OpenSession(_Base):
    session: str = ""
    n: int = 0
    ops: np.ndarray = None


@dataclass
class SampleRequest(_Base):
    session: str = ""
    qubits: np.ndarray = None
    shots: int = 0
    seed: int = 0
    shot_begin: int = 0
    meas_base: int = 0


@dataclass
class MeasureRequest(_Base):
    session: str = ""
    qubits: np.ndarray = None
    seed: int = 0
    shot: int = 0
    meas_base: int = 0


@dataclass
class CloseSession(_Base):
    session: str = ""


@dataclass
class ServeStats:
    requests: int
    completed: int
    failed: int
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


class _Session:
    def __init__(self, name: str, n: int):
        self.name = name
        self.n = n
        self.queue: List[_Base] = []   # admitted requests, in arrival order
        self.busy = False
        self.handle = None
        self.failed: Optional[BaseException] = None
        self.bytes = 0                 # the tableau's bytes, held until close
        self.closed = False


# ---------------------------------------------------------------- server
class Server:
    def __init__(self, budget_bytes: int = 8 << 30, workers: int = 2, batch_kwargs: Optional[Dict] = None,
                 backend=None, max_batch: int = 256):
        self.budget = int(budget_bytes)
        self.workers = int(workers)
        self.batch_kwargs = dict(batch_kwargs or {})
        self.backend = backend if backend is not None else GpuBackend()
        self.max_batch = int(max_batch)
        self._cv = threading.Condition()
        self._pending: List[_Base] = []     # arrived, waiting for memory
        self._circuits: List[CircuitRequest] = []  # admitted circuits, not yet running
        self._sessions: Dict[str, _Session] = {}
        self._in_flight = 0
        self._max_in_flight = 0
        self._all: List[_Base] = []
        self._batches: List[int] = []
        self._batch_kinds: List[str] = []   # circuits, open, sample, measure, close
        self._closing = False
        self._threads: List[threading.Thread] = []
        self._t0 = 0.0

    # -- clock ----------------------------------------------------------------
    def _now(self) -> float:
        return time.perf_counter() - self._t0

    # -- sizes ------------------------------------------------------------------
    def _bytes_of(self, r: _Base) -> int:
        b = self.backend
        if isinstance(r, CircuitRequest):
            return int(b.circuit_bytes(r, self.batch_kwargs))
        if isinstance(r, OpenSession):
            return int(b.tableau_bytes(r.n))
        if isinstance(r, SampleRequest):
            s = self._sessions.get(r.session)
            n = s.n if s is not None else 1
            return int(b.sample_bytes(n, len(r.qubits), r.shots))
        if isinstance(r, MeasureRequest):
            return 6 * len(r.qubits)
        return 0

    # -- request lifecycle (all under self._cv) ---------------------------------
    def _finish_locked(self, r: _Base, result=None, error: Optional[BaseException] = None, state=None):
        now = self._now()
        r.finished = now
        if error is None:
            r.result = result
            r.state = state or "done"
        else:
            r.error = error
            r.state = state or "failed"
        self._cv.notify_all()

    def _release_locked(self, r: _Base):
        if not isinstance(r, OpenSession):  # a session's tableau stays counted until it closes
            self._in_flight -= r.bytes

    def submit(self, r: _Base) -> _Base:
        """Queue a request now (arrival = now if it is unset)."""
        with self._cv:
            now = self._now()
            if not r.arrival or r.arrival < 0:
                r.arrival = now
            self._all.append(r)
            if isinstance(r, OpenSession):
                if r.session in self._sessions and not self._sessions[r.session].closed:
                    self._finish_locked(r, error=ValueError(f"session {r.session!r} is already open"))
                    return r
                self._sessions[r.session] = _Session(r.session, r.n)
            elif isinstance(r, (SampleRequest, MeasureRequest, CloseSession)):
                s = self._sessions.get(r.session)
                if s is None or s.closed:
                    self._finish_locked(r, error=KeyError(f"no open session {r.session!r}"))
                    return r
            r.bytes = self._bytes_of(r)
            if r.bytes > self.budget:
                self._finish_locked(r, error=Refused(f"request {r.rid} needs {r.bytes} bytes, budget {self.budget}"))
                if isinstance(r, OpenSession):
                    self._sessions[r.session].failed = r.error
                    self._sessions[r.session].closed = True
                return r
            r.state = "pending"
            self._pending.append(r)
            self._admit_locked()
            self._cv.notify_all()
        return r

    def cancel(self, r: _Base) -> bool:
        """Cancel a request no worker has taken yet; True if it was cancelled."""
        with self._cv:
            if r.state == "pending":
                self._pending.remove(r)
            elif r.state == "ready":
                self._release_locked(r)
                if isinstance(r, CircuitRequest):
                    self._circuits.remove(r)
                else:
                    self._sessions[r.session].queue.remove(r)
                    if isinstance(r, OpenSession):
                        self._in_flight -= r.bytes
            else:
                return False
            self._finish_locked(r, error=Cancelled(f"request {r.rid} cancelled"), state="cancelled")
            if isinstance(r, OpenSession):
                s = self._sessions[r.session]
                s.failed = r.error
            self._admit_locked()
            return True

    def _admit_locked(self):
        still = []
        now = self._now()
        blocked = set()  # sessions with an earlier request still waiting: keep their order
        for r in self._pending:
            sess = getattr(r, "session", None)
            if sess is not None and sess in blocked:
                still.append(r)
                continue
            if self._in_flight + r.bytes <= self.budget:
                self._in_flight += r.bytes
                self._max_in_flight = max(self._max_in_flight, self._in_flight)
                r.admitted = now
                r.state = "ready"
                if isinstance(r, CircuitRequest):
                    self._circuits.append(r)
                else:
                    self._sessions[r.session].queue.append(r)
            else:
                still.append(r)
                if sess is not None:
                    blocked.add(sess)
        self._pending = still

    def _expire_locked(self):
        """Fail waiting requests whose deadline has passed."""
        now = self._now()
        late = [r for r in self._pending if r.deadline is not None and now > r.deadline]
        for r in late:
            self._pending.remove(r)
            self._finish_locked(r, error=DeadlineExceeded(f"request {r.rid} not started by {r.deadline:.3f} s"))
        for r in [c for c in self._circuits if c.deadline is not None and now > c.deadline]:
            self._circuits.remove(r)
            self._release_locked(r)
            self._finish_locked(r, error=DeadlineExceeded(f"request {r.rid} not started by {r.deadline:.3f} s"))
        for s in self._sessions.values():
            for r in [q for q in s.queue if q.deadline is not None and now > q.deadline]:
                s.queue.remove(r)
                self._release_locked(r)
                if isinstance(r, OpenSession):
                    self._in_flight -= r.bytes
                    s.failed = DeadlineExceeded(f"session {s.name!r} was not opened in time")
                self._finish_locked(r, error=DeadlineExceeded(f"request {r.rid} not started by {r.deadline:.3f} s"))
        if late:
            self._admit_locked()

    # -- work selection (under self._cv) ---------------------------------------
    def _take_locked(self):
        """The next unit of work: ('circuits', [reqs]) or ('session', session,
        [reqs]); None if nothing can run now."""
        best = None
        if self._circuits:
            best = ("circuits", self._circuits[0].arrival)
        for s in self._sessions.values():
            if s.busy or not s.queue:
                continue
            a = s.queue[0].arrival
            if best is None or a < best[1]:
                best = ("session", a, s)
        if best is None:
            return None
        now = self._now()
        if best[0] == "circuits":
            batch, self._circuits = self._circuits[:self.max_batch], self._circuits[self.max_batch:]
            for r in batch:
                r.state, r.started = "running", now
            return ("circuits", batch)
        s = best[2]
        head = s.queue[0]
        take = [head]
        if isinstance(head, SampleRequest):
            # samples of the same list queued back to back share one sweep
            for r in s.queue[1:]:
                if not isinstance(r, SampleRequest) or not np.array_equal(r.qubits, head.qubits):
                    break
                take.append(r)
                if len(take) >= self.max_batch:
                    break
        del s.queue[:len(take)]
        s.busy = True
        for r in take:
            r.state, r.started = "running", now
        return ("session", s, take)

    # -- workers --------------------------------------------------------------
    def _run_circuits(self, batch, stream):
        try:
            outs = self.backend.batch_sample([r.as_batch_dict() for r in batch], stream, self.batch_kwargs)
            err = None
        except Exception as e:  # the batch fails alone
            outs, err = None, e
        with self._cv:
            for k, r in enumerate(batch):
                self._release_locked(r)
                if err is None:
                    self._finish_locked(r, result=outs[k])
                else:
                    self._finish_locked(r, error=err)
            self._batches.append(len(batch))
            self._batch_kinds.append("circuits")
            self._admit_locked()

    def _run_session(self, s: _Session, reqs, stream):
        head = reqs[0]
        results, err = None, None
        try:
            if s.failed is not None and not isinstance(head, CloseSession):
                raise RuntimeError(f"session {s.name!r} failed to open: {s.failed}")
            if isinstance(head, OpenSession):
                s.handle = self.backend.open(head.n, head.ops, stream)
                results = [True]
            elif isinstance(head, SampleRequest):
                sets = [dict(shots=r.shots, seed=r.seed, shot_begin=r.shot_begin, meas_base=r.meas_base) for r in reqs]
                results = self.backend.sample_many(s.handle, head.qubits, sets)
            elif isinstance(head, MeasureRequest):
                results = [self.backend.measure(s.handle, head.qubits, head.seed, head.shot, head.meas_base)]
            elif isinstance(head, CloseSession):
                if s.handle is not None:
                    self.backend.close(s.handle)
                    s.handle = None
                results = [True]
        except Exception as e:  # only these requests fail
            err = e
        with self._cv:
            if isinstance(head, OpenSession):
                if err is not None:
                    s.failed = err
                    self._in_flight -= head.bytes  # no tableau was kept
                    s.bytes = 0
                else:
                    s.bytes = head.bytes
            if isinstance(head, CloseSession):
                self._in_flight -= s.bytes
                s.bytes = 0
                s.closed = True
            for k, r in enumerate(reqs):
                self._release_locked(r)
                if err is None:
                    self._finish_locked(r, result=results[k])
                else:
                    self._finish_locked(r, error=err)
            s.busy = False
            self._batches.append(len(reqs))
            self._batch_kinds.append({OpenSession: "open", SampleRequest: "sample", MeasureRequest: "measure",
                                      CloseSession: "close"}[type(head)])
            self._admit_locked()

    def _worker(self, stream):
        if stream is not None:
            import torch
            torch.cuda.set_device(0)
        while True:
            with self._cv:
                while True:
                    self._expire_locked()
                    work = self._take_locked()
                    if work is not None:
                        break
                    if self._closing and not self._pending and not self._circuits and \
                            not any(s.queue or s.busy for s in self._sessions.values()):
                        return
                    self._cv.wait(timeout=0.02)
            if work[0] == "circuits":
                self._run_circuits(work[1], stream)
            else:
                self._run_session(work[1], work[2], stream)

    def start(self, use_gpu_streams: bool = True):
        if use_gpu_streams:
            import torch
            streams = [torch.cuda.Stream() for _ in range(self.workers)]
        else:
            streams = [None] * self.workers
        self._t0 = time.perf_counter()
        self._threads = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in streams]
        for th in self._threads:
            th.start()

    def stop(self):
        """Wait for every admitted or waiting request to finish, then stop the workers."""
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        for th in self._threads:
            th.join()
        self._threads = []

    def run(self, requests: List[_Base], use_gpu_streams: bool = True) -> ServeStats:
        """Submit `requests` at their arrival times (seconds after the start),
        wait for all of them, and return the statistics of the run. Refused,
        cancelled, late and failed requests carry their error and do not stop
        the others."""
        order = sorted(requests, key=lambda r: r.arrival)
        self.start(use_gpu_streams)
        try:
            for r in order:
                delay = r.arrival - self._now()
                if delay > 0:
                    time.sleep(delay)
                self.submit(r)
        finally:
            self.stop()
        return self.stats(order)

    def batch_sizes(self, kind: str) -> List[int]:
        """Sizes of the calls made for one kind of work (e.g. 'sample': requests per shared sweep)."""
        return [b for b, k in zip(self._batches, self._batch_kinds) if k == kind]

    def stats(self, reqs: Optional[List[_Base]] = None) -> ServeStats:
        reqs = self._all if reqs is None else reqs
        done = [r for r in reqs if r.state == "done"]
        lat = [r.finished - r.arrival for r in done]
        shots = sum(getattr(r, "shots", 0) for r in done if isinstance(r, (CircuitRequest, SampleRequest)))
        if done:
            span = max(max(r.finished for r in done) - min(r.arrival for r in reqs), 1e-9)
        else:
            span = 1e-9
        return ServeStats(
            requests=len(reqs), completed=len(done), failed=len(reqs) - len(done), shots=shots, makespan_s=span,
            shots_per_s=shots / span,
            latency_p50_s=float(np.percentile(lat, 50)) if lat else float("nan"),
            latency_p99_s=float(np.percentile(lat, 99)) if lat else float("nan"),
            batches=len(self._batches), mean_batch=float(np.mean(self._batches)) if self._batches else 0.0,
            max_in_flight_bytes=self._max_in_flight, budget_bytes=self.budget, latencies=lat)
