"""The serving loop on the GPU (needs an MI355X): every request's result,
served in the mix with overlapping batches and memory-bounded admission,
equals the same request run alone (tolerance 0): one-shot circuits, and
sampling and measurement requests against resident tableaux (sessions), whose
queued sampling requests share one measurement sweep."""
import numpy as np
import pytest

from workload import circuit_ops, served_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _gates(r):
    ops = circuit_ops(r.config(), final_measure=False)
    return np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)


def test_served_circuits_equal_alone():
    from paper_2603_14641_amd import batch_sample, serving
    reqs = []
    for r in served_requests(count=512, rate_hz=400.0):
        if r.n > 2000:
            continue
        reqs.append(serving.CircuitRequest(n=r.n, ops=_gates(r), qubits=np.arange(r.n, dtype=np.uint32),
                                           shots=r.shots, seed=r.coin_seed, arrival=r.arrival_s))
        if len(reqs) == 60:
            break
    be = serving.GpuBackend()
    budget = 3 * max(be.circuit_bytes(r, {}) for r in reqs)
    too_big = serving.CircuitRequest(n=16000, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(16000, dtype=np.uint32),
                                     shots=4, arrival=reqs[10].arrival)
    st = serving.Server(budget_bytes=budget, workers=2).run(reqs + [too_big])
    assert isinstance(too_big.error, serving.Refused), "an oversized request must be refused on its own"
    assert st.completed == len(reqs) and st.max_in_flight_bytes <= budget
    assert st.mean_batch > 1.0, "arrivals during running batches should be batched together"
    for r in reqs:
        alone = batch_sample([r.as_batch_dict()])[0]
        assert np.array_equal(r.result, alone), f"request {r.rid} (n={r.n}) differs between served and alone"
    print(f"served {st.completed} requests, {st.shots} shots in {st.makespan_s:.2f}s, "
          f"p50 {st.latency_p50_s*1e3:.1f} ms, p99 {st.latency_p99_s*1e3:.1f} ms, {st.batches} batches")


def test_sessions_equal_alone():
    """Three resident tableaux; sampling and measurement requests against
    them arrive together, so queued samples share sweeps; each result equals
    the same call made alone on a tableau in the same state."""
    from paper_2603_14641_amd import Tableau, serving
    pick = [r for r in served_requests() if 300 <= r.n <= 3000][:3]
    rng = np.random.default_rng(5)
    srv = serving.Server(budget_bytes=4 << 30, workers=2)
    srv.start()
    opens = [srv.submit(serving.OpenSession(session=f"s{k}", n=r.n, ops=_gates(r))) for k, r in enumerate(pick)]
    plan = []  # (session index, kind, args) in submission order
    for i in range(30):
        k = int(rng.integers(3))
        n = pick[k].n
        if i % 7 == 6:
            qs = np.sort(rng.choice(n, 12, replace=False)).astype(np.uint32)
            plan.append((k, "measure", dict(qubits=qs, seed=int(rng.integers(1 << 30)), shot=0, meas_base=i)))
        else:
            plan.append((k, "sample", dict(qubits=np.arange(n, dtype=np.uint32), shots=int(rng.integers(1, 300)),
                                           seed=int(rng.integers(1 << 30)))))
    reqs = []
    for k, kind, a in plan:
        if kind == "sample":
            reqs.append(srv.submit(serving.SampleRequest(session=f"s{k}", **a)))
        else:
            reqs.append(srv.submit(serving.MeasureRequest(session=f"s{k}", **a)))
    for k in range(3):
        srv.submit(serving.CloseSession(session=f"s{k}"))
    srv.stop()
    assert all(o.ok for o in opens)
    assert all(r.ok for r in reqs), [str(r.error) for r in reqs if not r.ok][:3]
    assert max(srv.batch_sizes("sample")) > 1, "queued samples on one session should share a sweep"
    # alone: replay each session's requests in order on its own tableau
    alone_tabs = []
    for r in pick:
        t = Tableau(r.n)
        t.apply_gates(_gates(r))
        alone_tabs.append(t)
    for (k, kind, a), r in zip(plan, reqs):
        t = alone_tabs[k]
        if kind == "sample":
            want = t.sample(a["qubits"], a["shots"], seed=a["seed"])
            assert np.array_equal(r.result, want), f"sample on session {k} differs from alone"
        else:
            bits, rnd = t.measure(a["qubits"], seed=a["seed"], shot=a["shot"], meas_base=a["meas_base"])
            assert np.array_equal(r.result[0], bits) and np.array_equal(r.result[1], rnd), \
                f"measurement on session {k} differs from alone"
    for t in alone_tabs:
        t.close()
    assert srv._in_flight == 0
