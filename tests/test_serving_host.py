"""Host logic of the serving loop (no GPU), with a fake backend standing in
for libsq: admission by the memory budget, continuous batching of circuits,
resident sessions whose sampling requests share a sweep, per-request
refusal, failure isolation, cancellation and deadlines."""
import threading
import time

import numpy as np
import pytest

from paper_2603_14641_amd import binding, serving


class FakeBackend:
    """Records calls and bytes in flight; returns outputs that name their request."""

    def __init__(self, delay=0.01, fail_on_n=None, fail_open=None, gate=None):
        self.delay = delay
        self.fail_on_n = fail_on_n
        self.fail_open = fail_open
        self.gate = gate  # an Event the first batch waits on (to hold a worker busy)
        self.lock = threading.Lock()
        self.batches = []
        self.sample_calls = []
        self.log = []
        self.active = 0
        self.max_active = 0

    # sizes
    def circuit_bytes(self, r, kw):
        return 1000 * r.n + 8 * r.shots

    def tableau_bytes(self, n):
        return 100 * n

    def sample_bytes(self, n, count, shots):
        return 10 * n + shots

    def _busy(self):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        if self.gate is not None:
            self.gate.wait(5)
        time.sleep(self.delay)
        with self.lock:
            self.active -= 1

    def batch_sample(self, items, stream, kw):
        with self.lock:
            self.batches.append([r["n"] for r in items])
        self._busy()
        if self.fail_on_n is not None and any(r["n"] == self.fail_on_n for r in items):
            raise binding.SqError(binding.SQ_EDEVICE, "injected kernel failure")
        return [np.full((r["shots"], (len(r["qubits"]) + 63) // 64), r["n"], dtype=np.uint64) for r in items]

    def open(self, n, ops, stream):
        self._busy()
        if self.fail_open == n:
            raise binding.SqError(binding.SQ_ENOMEM, "injected allocation failure")
        with self.lock:
            self.log.append(("open", n))
        return {"n": n, "measured": 0}

    def sample_many(self, handle, qubits, sets):
        with self.lock:
            self.sample_calls.append(len(sets))
            self.log.append(("sample", len(sets)))
        self._busy()
        return [np.full((e["shots"], 1), e["seed"], dtype=np.uint64) for e in sets]

    def measure(self, handle, qubits, seed, shot, meas_base):
        self._busy()
        handle["measured"] += len(qubits)
        with self.lock:
            self.log.append(("measure", handle["measured"]))
        return np.full(len(qubits), seed % 2, np.uint8), np.zeros(len(qubits), np.uint8)

    def close(self, handle):
        with self.lock:
            self.log.append(("close", handle["n"]))


def _circuits(k, rate=200.0, seed=0):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(k):
        n = int(rng.integers(16, 400))
        t += float(rng.exponential(1 / rate))
        out.append(serving.CircuitRequest(n=n, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(n, dtype=np.uint32),
                                          shots=int(rng.integers(1, 50)), arrival=t))
    return out


def test_all_circuits_complete_with_their_own_results():
    fake = FakeBackend()
    reqs = _circuits(60)
    st = serving.Server(budget_bytes=1 << 30, workers=2, backend=fake).run(reqs, use_gpu_streams=False)
    assert st.requests == 60 and st.completed == 60
    for r in reqs:
        assert r.ok and r.result.shape[0] == r.shots and np.all(r.result == r.n)
        assert r.arrival <= r.admitted <= r.started <= r.finished
    assert st.latency_p50_s <= st.latency_p99_s
    assert sum(len(b) for b in fake.batches) == 60
    assert max(len(b) for b in fake.batches) > 1, "circuits arriving during a batch must be batched together"
    assert fake.max_active == 2, "two workers overlap their batches"


def test_budget_limits_bytes_in_flight():
    fake = FakeBackend(delay=0.02)
    reqs = _circuits(40, rate=1000.0, seed=1)
    biggest = max(fake.circuit_bytes(r, {}) for r in reqs)
    budget = 3 * biggest
    srv = serving.Server(budget_bytes=budget, workers=3, backend=fake)
    st = srv.run(reqs, use_gpu_streams=False)
    assert st.max_in_flight_bytes <= budget
    assert st.completed == 40
    assert srv._in_flight == 0


def test_oversized_request_is_refused_alone():
    fake = FakeBackend()
    reqs = _circuits(10, seed=3)
    budget = max(fake.circuit_bytes(r, {}) for r in reqs) + 1
    big = serving.CircuitRequest(n=10**6, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(4, dtype=np.uint32),
                                 shots=1, arrival=reqs[4].arrival)
    st = serving.Server(budget_bytes=budget, workers=2, backend=fake).run(reqs + [big], use_gpu_streams=False)
    assert isinstance(big.error, serving.Refused) and big.state == "failed"
    assert all(r.ok for r in reqs)
    assert st.completed == 10 and st.failed == 1


def test_failed_batch_fails_only_its_requests_and_frees_their_bytes():
    reqs = _circuits(30, rate=500.0, seed=2)
    fake = FakeBackend(fail_on_n=reqs[7].n)
    srv = serving.Server(budget_bytes=1 << 30, workers=2, backend=fake)
    st = srv.run(reqs, use_gpu_streams=False)
    failed = [r for r in reqs if not r.ok]
    assert reqs[7] in failed
    assert all(isinstance(r.error, binding.SqError) for r in failed)
    # the failing batch holds reqs[7]; every request of another batch completed
    bad_batches = [b for b in fake.batches if reqs[7].n in b]
    assert len(failed) <= sum(len(b) for b in bad_batches)
    assert st.completed == 30 - len(failed) > 0
    assert srv._in_flight == 0, "bytes of the failed batch were not freed"


def test_cancel_before_start():
    gate = threading.Event()
    fake = FakeBackend(gate=gate)
    srv = serving.Server(budget_bytes=1 << 30, workers=1, backend=fake)
    srv.start(use_gpu_streams=False)
    first = srv.submit(serving.CircuitRequest(n=20, ops=np.zeros((0, 3), np.uint32),
                                              qubits=np.arange(20, dtype=np.uint32), shots=3))
    time.sleep(0.05)  # the worker holds `first` at the gate
    second = srv.submit(serving.CircuitRequest(n=30, ops=np.zeros((0, 3), np.uint32),
                                               qubits=np.arange(30, dtype=np.uint32), shots=3))
    assert srv.cancel(second)
    assert not srv.cancel(first), "a running request cannot be cancelled"
    gate.set()
    srv.stop()
    assert first.ok and second.state == "cancelled" and isinstance(second.error, serving.Cancelled)
    assert srv._in_flight == 0
    assert [30] not in fake.batches


def test_deadline_passes_while_waiting_for_memory():
    gate = threading.Event()
    fake = FakeBackend(gate=gate)
    budget = fake.circuit_bytes(serving.CircuitRequest(n=100, shots=1), {})
    srv = serving.Server(budget_bytes=budget, workers=2, backend=fake)
    srv.start(use_gpu_streams=False)
    hog = srv.submit(serving.CircuitRequest(n=100, ops=np.zeros((0, 3), np.uint32),
                                            qubits=np.arange(100, dtype=np.uint32), shots=1))
    late = srv.submit(serving.CircuitRequest(n=90, ops=np.zeros((0, 3), np.uint32),
                                             qubits=np.arange(90, dtype=np.uint32), shots=1,
                                             deadline=srv._now() + 0.05))
    time.sleep(0.2)
    gate.set()
    srv.stop()
    assert hog.ok
    assert late.state == "failed" and isinstance(late.error, serving.DeadlineExceeded)


def test_session_samples_share_a_sweep_and_run_in_order():
    gate = threading.Event()
    fake = FakeBackend(gate=gate)
    srv = serving.Server(budget_bytes=1 << 30, workers=2, backend=fake)
    srv.start(use_gpu_streams=False)
    q = np.arange(50, dtype=np.uint32)
    op = srv.submit(serving.OpenSession(session="a", n=50, ops=np.zeros((0, 3), np.uint32)))
    time.sleep(0.05)  # `open` is held at the gate; these queue behind it
    samples = [srv.submit(serving.SampleRequest(session="a", qubits=q, shots=5 + k, seed=100 + k)) for k in range(6)]
    meas = srv.submit(serving.MeasureRequest(session="a", qubits=q[:10], seed=7))
    after = srv.submit(serving.SampleRequest(session="a", qubits=q, shots=2, seed=55))
    close = srv.submit(serving.CloseSession(session="a"))
    gate.set()
    srv.stop()
    assert op.ok and meas.ok and after.ok and close.ok
    for k, s in enumerate(samples):
        assert s.ok and s.result.shape == (5 + k, 1) and np.all(s.result == 100 + k)
    # the six queued samples shared one call; the measurement came after them
    # and the last sample after it, then the close
    assert fake.sample_calls == [6, 1]
    assert [e[0] for e in fake.log] == ["open", "sample", "measure", "sample", "close"]
    assert srv._in_flight == 0, "the session's tableau bytes were not freed at close"
    st = srv.stats()
    assert st.mean_batch > 1


def test_session_bytes_held_until_close_and_failed_open_isolated():
    fake = FakeBackend(fail_open=77)
    srv = serving.Server(budget_bytes=1 << 30, workers=2, backend=fake)
    srv.start(use_gpu_streams=False)
    good = srv.submit(serving.OpenSession(session="g", n=40, ops=None))
    bad = srv.submit(serving.OpenSession(session="b", n=77, ops=None))
    time.sleep(0.1)
    assert good.ok and srv._in_flight == fake.tableau_bytes(40)
    s_bad = srv.submit(serving.SampleRequest(session="b", qubits=np.arange(3, dtype=np.uint32), shots=1))
    s_good = srv.submit(serving.SampleRequest(session="g", qubits=np.arange(3, dtype=np.uint32), shots=1, seed=9))
    s_none = srv.submit(serving.SampleRequest(session="zzz", qubits=np.arange(3, dtype=np.uint32), shots=1))
    srv.submit(serving.CloseSession(session="g"))
    srv.submit(serving.CloseSession(session="b"))
    srv.stop()
    assert bad.state == "failed" and s_bad.state == "failed"
    assert s_good.ok and np.all(s_good.result == 9)
    assert s_none.state == "failed" and isinstance(s_none.error, KeyError)
    assert srv._in_flight == 0


def test_gpu_backend_sizes_come_from_the_library():
    """The default backend's byte counts are the library's own figures."""
    be = serving.GpuBackend()
    n = 5000
    r = serving.CircuitRequest(n=n, ops=np.zeros((1000, 3), np.uint32), qubits=np.arange(n, dtype=np.uint32),
                               shots=64)
    big = be.circuit_bytes(r, {})
    assert big == binding.batch_item_bytes(n, 1000, n, 64)
    assert big >= binding.bytes_required(n) + binding.sample_bytes(n, n, 64)
    small = serving.CircuitRequest(n=200, ops=np.zeros((10, 3), np.uint32), qubits=np.arange(200, dtype=np.uint32),
                                   shots=8)
    assert 0 < be.circuit_bytes(small, {}) < binding.bytes_required(200)
    assert be.tableau_bytes(n) == binding.bytes_required(n)
    assert binding.sample_bytes(n, n, 1) < binding.sample_bytes(n, n, 4096)
    # routing follows the batch options: a 200-qubit item above max_batch_n takes the plain path
    assert binding.batch_item_bytes(200, 10, 200, 8, max_batch_n=128) >= binding.bytes_required(200)
    assert binding.batch_item_bytes(200, 10, 0, 8) == 0
