"""The serving loop on the GPU: every request's shots, served in the mix with
overlapping batches and memory-bounded admission, equal its shots run alone
(tolerance 0). Needs an MI355X."""
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


def test_served_equals_alone():
    from paper_2603_14641_amd import batch_sample, serving
    reqs = []
    for r in served_requests(count=512, rate_hz=400.0):
        if r.n > 2000:
            continue
        cfg = r.config()
        ops = circuit_ops(cfg, final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(serving.Request(rid=r.index, n=cfg.n, ops=ops, qubits=np.arange(cfg.n, dtype=np.uint32),
                                    shots=r.shots, seed=r.coin_seed, arrival=r.arrival_s))
        if len(reqs) == 60:
            break
    budget = 3 * max(serving.request_bytes(r.n, r.n, r.shots) for r in reqs)
    st = serving.Server(budget_bytes=budget, workers=2).run(reqs)
    assert st.requests == len(reqs) and st.max_in_flight_bytes <= budget
    assert st.mean_batch > 1.0, "arrivals during running batches should be batched together"
    for r in reqs:
        alone = batch_sample([r.as_batch_dict()])[0]
        assert np.array_equal(r.result, alone), f"request {r.rid} (n={r.n}) differs between served and alone"
    print(f"served {st.requests} requests, {st.shots} shots in {st.makespan_s:.2f}s, "
          f"p50 {st.latency_p50_s*1e3:.1f} ms, p99 {st.latency_p99_s*1e3:.1f} ms, {st.batches} batches")
