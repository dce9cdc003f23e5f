"""Batched execution (sq_batch_sample): every circuit's shots must be bit-for-bit
the single-tableau path's (sq_create + sq_apply_gates + sq_sample), and the
oracle's per-shot CHP where the oracle is affordable. Needs an MI355X."""
import numpy as np
import pytest

from gpu_util import mixed_program
from oracle import oracle as orc
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


def _gates(ops):
    a = np.asarray(ops)
    return a[a[:, 0] != orc.MEASURE] if a.ndim == 2 else a


def plain(req):
    from paper_2603_14641_amd import Tableau
    t = Tableau(req["n"])
    t.apply_gates(req["ops"])
    out = t.sample(req["qubits"], req["shots"], seed=req.get("seed", 0), shot_begin=req.get("shot_begin", 0),
                   meas_base=req.get("meas_base", 0))
    t.close()
    return out


def oracle_words(req, shots_idx):
    n = req["n"]
    ref = orc.Tableau(n)
    ref.run(req["ops"])
    x, z, r = ref.rows_array()
    ops = np.array([[orc.MEASURE, int(q), 0] for q in req["qubits"]], dtype=np.uint32).reshape(-1, 3)
    W = (len(req["qubits"]) + 63) // 64
    out = {}
    for s in shots_idx:
        t = orc.Tableau(n)
        t.set_rows(x, z, r)
        bits, _, _ = t.run(ops, seed=req.get("seed", 0), shot=req.get("shot_begin", 0) + s,
                           meas_base=req.get("meas_base", 0))
        w = np.zeros(W, dtype=np.uint64)
        for i, b in enumerate(bits):
            w[i >> 6] |= np.uint64(int(b) << (i & 63))
        out[s] = w
    return out


def _mixed_requests(rng, k, nmax):
    reqs = []
    for i in range(k):
        n = int(rng.integers(1, nmax))
        ops = mixed_program(rng, n, int(rng.integers(1, 12)), p_meas=0.0)
        qubits = [int(q) for q in rng.integers(0, n, int(rng.integers(1, 2 * n + 2)))]
        reqs.append(dict(n=n, ops=ops, qubits=qubits, shots=int(rng.integers(1, 70)), seed=int(rng.integers(1 << 30)),
                         shot_begin=int(rng.integers(1000)), meas_base=int(rng.integers(1000))))
    return reqs


@pytest.mark.parametrize("block", [64, 256, 512])
def test_batch_equals_plain_and_oracle(block):
    from paper_2603_14641_amd import batch_sample
    rng = np.random.default_rng(block)
    reqs = _mixed_requests(rng, 40, 300)
    reqs = [r for r in reqs if 2 * ((r["n"] + 63) // 64) <= 2 * block]
    got = batch_sample(reqs, block=block)
    for k, (req, g) in enumerate(zip(reqs, got)):
        want = plain(req)
        assert np.array_equal(g, want), f"request {k} (n={req['n']}) differs from the single-tableau path"
        if req["n"] <= 80:
            ow = oracle_words(req, range(req["shots"]))
            for s, w in ow.items():
                assert np.array_equal(g[s], w), f"request {k} shot {s} differs from the oracle"


def test_batch_all_gate_types():
    """Batched circuits with CY, SWAP and iSWAP (pair micro-op products) against the oracle."""
    from paper_2603_14641_amd import batch_sample
    rng = np.random.default_rng(77)
    reqs = []
    for i in range(16):
        n = int(rng.integers(2, 70))
        ops = mixed_program(rng, n, int(rng.integers(2, 10)), p_meas=0.0, extra=True)
        qubits = [int(q) for q in rng.permutation(n)]
        reqs.append(dict(n=n, ops=ops, qubits=qubits, shots=int(rng.integers(1, 20)), seed=i, shot_begin=0,
                         meas_base=0))
    got = batch_sample(reqs, block=256)
    for k, (req, g) in enumerate(zip(reqs, got)):
        ow = oracle_words(req, range(req["shots"]))
        for s, w in ow.items():
            assert np.array_equal(g[s], w), f"request {k} shot {s} differs from the oracle"
        assert np.array_equal(g, plain(req))


def test_batch_routes_large_items_to_single_path():
    from paper_2603_14641_amd import batch_sample
    rng = np.random.default_rng(9)
    reqs = _mixed_requests(rng, 12, 200)
    got = batch_sample(reqs, block=128, max_batch_n=64)
    for req, g in zip(reqs, got):
        assert np.array_equal(g, plain(req))


def test_served_mix_subset_parity():
    """The first 48 requests of the batched/served mix (n up to 16384): batched
    vs single-tableau for every shot; the oracle on every shot where n <= 256
    and on shots {0, 1, S-1} plus 5 seeded others where n <= 2048."""
    from paper_2603_14641_amd import batch_sample
    reqs = []
    for r in served_requests()[:48]:
        cfg = r.config()
        ops = circuit_ops(cfg, final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(dict(n=cfg.n, ops=ops, qubits=list(range(cfg.n)), shots=r.shots, seed=r.coin_seed))
    got = batch_sample(reqs)
    rng = np.random.default_rng(0)
    checked = 0
    for k, (req, g) in enumerate(zip(reqs, got)):
        if req["n"] <= 4096:
            assert np.array_equal(g, plain(req)), f"request {k} (n={req['n']}) differs from the single-tableau path"
        S = req["shots"]
        if req["n"] <= 256:
            idx = range(S)
        elif req["n"] <= 2048:
            idx = sorted({0, 1 % S, S - 1} | {int(v) for v in rng.integers(0, S, 5)})
        else:
            continue
        for s, w in oracle_words(req, idx).items():
            assert np.array_equal(g[s], w), f"request {k} (n={req['n']}) shot {s} differs from the oracle"
            checked += 1
    assert checked > 100
