"""Host logic of the serving loop (no GPU): admission by the memory budget,
continuous batching, completion and failure propagation, with a fake
batched backend standing in for libsq."""
import threading
import time

import numpy as np
import pytest

from paper_2603_14641_amd import binding, serving


class FakeBackend:
    """Records batches and the bytes in flight; returns per-request marker outputs."""

    def __init__(self, delay=0.01, fail_on=None):
        self.delay = delay
        self.fail_on = fail_on
        self.lock = threading.Lock()
        self.batches = []
        self.active = 0
        self.max_active = 0

    def __call__(self, reqs, stream=None, **kw):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.batches.append([r["n"] for r in reqs])
        time.sleep(self.delay)
        with self.lock:
            self.active -= 1
        if self.fail_on is not None and any(r["n"] == self.fail_on for r in reqs):
            raise binding.SqError(binding.SQ_EDEVICE, "injected kernel failure")
        return [np.full((r["shots"], (len(r["qubits"]) + 63) // 64), r["n"], dtype=np.uint64) for r in reqs]


def _requests(k, rate=200.0, seed=0):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(k):
        n = int(rng.integers(16, 400))
        t += float(rng.exponential(1 / rate))
        out.append(serving.Request(rid=i, n=n, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(n, dtype=np.uint32),
                                   shots=int(rng.integers(1, 50)), arrival=t))
    return out


def test_all_requests_complete_with_their_own_results(monkeypatch):
    fake = FakeBackend()
    monkeypatch.setattr(binding, "batch_sample", fake)
    reqs = _requests(60)
    st = serving.Server(budget_bytes=1 << 30, workers=2).run(reqs, use_gpu_streams=False)
    assert st.requests == 60 and all(r.result is not None for r in reqs)
    for r in reqs:
        assert r.result.shape[0] == r.shots and np.all(r.result == r.n)
        assert r.arrival <= r.admitted <= r.started <= r.finished
    assert st.latency_p50_s <= st.latency_p99_s
    assert sum(len(b) for b in fake.batches) == 60
    assert max(len(b) for b in fake.batches) > 1, "requests arriving during a batch must be batched together"
    assert fake.max_active == 2, "two workers overlap their batches"


def test_budget_limits_bytes_in_flight(monkeypatch):
    fake = FakeBackend(delay=0.02)
    monkeypatch.setattr(binding, "batch_sample", fake)
    reqs = _requests(40, rate=1000.0, seed=1)
    biggest = max(serving.request_bytes(r.n, len(r.qubits), r.shots) for r in reqs)
    budget = 3 * biggest
    st = serving.Server(budget_bytes=budget, workers=3).run(reqs, use_gpu_streams=False)
    assert st.max_in_flight_bytes <= budget
    assert st.requests == 40


def test_request_larger_than_budget_is_refused(monkeypatch):
    monkeypatch.setattr(binding, "batch_sample", FakeBackend())
    reqs = _requests(5)
    with pytest.raises(binding.SqError):
        serving.Server(budget_bytes=1000, workers=1).run(reqs, use_gpu_streams=False)


def test_backend_failure_propagates(monkeypatch):
    reqs = _requests(20, seed=2)
    fake = FakeBackend(fail_on=reqs[7].n)
    monkeypatch.setattr(binding, "batch_sample", fake)
    with pytest.raises(binding.SqError):
        serving.Server(budget_bytes=1 << 30, workers=2).run(reqs, use_gpu_streams=False)
