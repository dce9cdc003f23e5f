"""The whole batched/served mix (512 generator circuits, n log-uniform in
[16, 16384], depth 10..500, 1..4096 shots of measuring every qubit): the
batched path (sq_batch_sample, default schedule) against the single-tableau
path on every shot of every request, and against the oracle's per-shot CHP
outcomes stored in tests/golden/served_mix_oracle.json (every shot where
n <= 256; shots {0, 1, S-1} and 5 seeded others where n <= 2048; shots
{0, S-1} of 8 seeded requests with 2048 < n <= 8192), compared through the SHA-256
of the checked shots' outcome words. Needs an MI355X."""
import hashlib
import json
import os
import time

import numpy as np
import pytest

from workload import circuit_ops, served_requests

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "served_mix_oracle.json")


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _requests():
    reqs = []
    for r in served_requests():
        ops = circuit_ops(r.config(), final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(dict(n=r.n, ops=ops, qubits=np.arange(r.n, dtype=np.uint32), shots=r.shots, seed=r.coin_seed))
    return reqs


def _digest(words, shots):
    return hashlib.sha256(np.ascontiguousarray(words[shots]).tobytes()).hexdigest()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_served_mix_all_requests_batched_plain_and_oracle():
    from paper_2603_14641_amd import Tableau, batch_sample
    doc = json.load(open(GOLDEN))
    assert doc.get("complete", False), "the oracle fixture is incomplete: rerun its script"
    golden = doc["requests"]
    t0 = time.time()
    reqs = _requests()
    print(f"512 requests drawn in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    got = batch_sample(reqs)
    print(f"batched in {time.time() - t0:.1f} s", flush=True)
    checked = 0
    for k, (req, g) in enumerate(zip(reqs, got)):
        entry = golden.get(str(k))
        if entry is not None:
            assert entry["n"] == req["n"] and entry["shots_total"] == req["shots"], f"request {k}: fixture mismatch"
            assert _digest(g, entry["shots"]) == entry["sha256"], \
                f"request {k} (n={req['n']}): shots {entry['shots'][:5]}... differ from the oracle"
            checked += len(entry["shots"])
    assert checked > 100000
    print(f"oracle shots checked: {checked}", flush=True)
    t0 = time.time()
    for k, (req, g) in enumerate(zip(reqs, got)):
        t = Tableau(req["n"])
        t.apply_gates(req["ops"])
        want = t.sample(req["qubits"], req["shots"], seed=req["seed"])
        t.close()
        assert np.array_equal(g, want), f"request {k} (n={req['n']}): batched differs from the single-tableau path"
    print(f"single-tableau path in {time.time() - t0:.1f} s", flush=True)
