"""sq_sample parity: every shot must equal the oracle's per-shot CHP run on a
copy of the same state with that shot's coins (tolerance 0), and sampling must
leave the tableau unchanged. Needs an MI355X."""
import numpy as np
import pytest

from gpu_util import gpu_run_calls, mixed_program
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


def oracle_shots(ref, qubits, seed, shot_begin, shots, meas_base):
    """Definition: per shot, CHP measurement of the list on a copy of ref."""
    x, z, r = ref.rows_array()
    ops = np.array([[orc.MEASURE, int(q), 0] for q in qubits], dtype=np.uint32).reshape(-1, 3)
    outs = np.zeros((shots, len(qubits)), dtype=np.uint8)
    nrand = 0
    for s in range(shots):
        t = orc.Tableau(ref.n)
        t.set_rows(x, z, r)
        bits, rnd, _ = t.run(ops, seed=seed, shot=shot_begin + s, meas_base=meas_base)
        assert bits.size == len(qubits)
        outs[s] = bits
        nrand = int(rnd.sum())
    return outs, nrand


def _gpu_from_oracle(ref):
    from paper_2603_14641_amd import Tableau
    t = Tableau(ref.n)
    t.import_(*ref.rows_array())
    return t


def _check(t, ref, qubits, seed, shot_begin, shots, meas_base):
    want, nrand = oracle_shots(ref, qubits, seed, shot_begin, shots, meas_base)
    got = t.sample_bits(qubits, shots, seed=seed, shot_begin=shot_begin, meas_base=meas_base)
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{bad.shape[0]} shot bits differ, first (shot, i) {bad[:5].tolist()}")
    x, z, r = t.export()
    rx, rz, rr = ref.rows_array()
    assert np.array_equal(x, rx) and np.array_equal(z, rz) and np.array_equal(r, rr), "sampling changed the tableau"
    assert t.error_flags() == 0
    return nrand


@pytest.mark.parametrize("n", [1, 5, 64, 65, 200, 700])
def test_sample_all_qubits(n):
    rng = np.random.default_rng(300 + n)
    ref = orc.Tableau(n)
    ref.run(mixed_program(rng, n, 8, p_meas=0.1), seed=3)
    t = _gpu_from_oracle(ref)
    shots = 40 if n <= 200 else 8
    _check(t, ref, list(range(n)), seed=17, shot_begin=int(rng.integers(1 << 20)), shots=shots,
           meas_base=int(rng.integers(1000)))


@pytest.mark.parametrize("mb", [1, 2, 32])
def test_sample_block_sizes_agree_with_oracle(mb):
    """The sampling sweep with 1 (one at a time), 2 and 32 random measurements
    per pass; n = 1500, every qubit, with deterministic ones mixed in."""
    n = 1500
    rng = np.random.default_rng(4242)
    ref = orc.Tableau(n)
    ref.run(mixed_program(rng, n, 6, p_meas=0.05), seed=8)
    t = _gpu_from_oracle(ref)
    t.set_tuning(meas_block=mb)
    qs = list(rng.permutation(n)) + list(range(0, n, 97))
    _check(t, ref, qs, seed=5, shot_begin=11, shots=6, meas_base=2)


def test_sample_blocked_equals_single_at_4000():
    """n = 4000: the blocked sweep gives the one-at-a-time sweep's bits for 300 shots."""
    from paper_2603_14641_amd import Program, Tableau
    n = 4000
    rng = np.random.default_rng(77)
    prog = Program(n, mixed_program(rng, n, 10, p_meas=0.02))
    outs = []
    for mb in (1, 32):
        t = Tableau(n)
        t.set_tuning(meas_block=mb)
        t.run_to_host(prog, seed=1, shot=0)
        qs = list(rng.permutation(n)) if mb == 1 else qs_keep
        qs_keep = qs
        outs.append(t.sample_bits(qs, 300, seed=9, shot_begin=0, meas_base=0))
        t.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("n", [3, 40, 130])
def test_sample_unordered_with_repeats(n):
    """Random order, repeated qubits (re-measurements are deterministic with
    affine forms in the earlier coins)."""
    rng = np.random.default_rng(400 + n)
    ref = orc.Tableau(n)
    ref.run(mixed_program(rng, n, 6, p_meas=0.0))
    t = _gpu_from_oracle(ref)
    qubits = [int(q) for q in rng.integers(0, n, 3 * n)]
    _check(t, ref, qubits, seed=5, shot_begin=0, shots=64, meas_base=7)


@pytest.mark.parametrize("n", [12, 40, 200])
def test_sample_scrambled_generators(n):
    """Deterministic outcomes with nonzero phase sums inside the sweep."""
    from test_gpu_parity import _scrambled_state
    rng = np.random.default_rng(n * 10 + 1)
    ref = _scrambled_state(n, rng, seed=n)
    t = _gpu_from_oracle(ref)
    qubits = list(range(0, n, 2)) + [int(q) for q in rng.permutation(n)[: n // 2]] + list(range(n))
    _check(t, ref, qubits, seed=9, shot_begin=100, shots=32, meas_base=0)


def test_sample_served_requests_small():
    """A few circuits of the batched/served mix (the smaller ones), all their
    shots, final all-qubit measurement."""
    reqs = [r for r in served_requests() if r.n <= 120 and r.shots <= 200][:6]
    assert reqs
    from paper_2603_14641_amd import Tableau
    for req in reqs:
        cfg = req.config()
        ops = circuit_ops(cfg, final_measure=False)
        ref = orc.Tableau(cfg.n)
        ref.run(ops)
        t = Tableau(cfg.n)
        gpu_run_calls(t, ops, seed=0)
        _check(t, ref, list(range(cfg.n)), seed=req.coin_seed, shot_begin=0, shots=req.shots, meas_base=0)


def test_sample_zero_shots_and_errors():
    from paper_2603_14641_amd import SqError, Tableau
    t = Tableau(10)
    assert t.sample([0, 1], 0).shape == (0, 1)
    with pytest.raises(SqError):
        t.sample([0, 10], 4)
