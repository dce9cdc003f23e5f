"""Pauli-frame sampling on the GPU (sq_frame_sample) against the frame
oracle, bit for bit, with the same reference sample (the oracle's CHP run)."""
import numpy as np
import pytest

from gpu_util import mixed_program
from oracle import oracle as orc
from workload import CONFIGS, circuit_ops

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()


def _check(n, ops, seed, shots):
    from paper_2603_14641_amd import Program
    ref, _, _ = orc.Tableau(n).run(ops, seed=seed, shot=0)
    want = orc.frame_sample(n, ops, ref, seed=seed + 1, shots=shots)
    got = Program(n, ops).frame_sample(shots, seed=seed + 1, ref=ref)
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{bad.shape[0]} words differ, first (shot, word) {bad[:4].tolist()}")


@pytest.mark.parametrize("n", [1, 5, 64, 65, 300, 1500])
@pytest.mark.parametrize("shots", [1, 63, 64, 65, 200, 1000])
def test_frames_match_oracle(n, shots):
    rng = np.random.default_rng(n * 7 + shots)
    ops = mixed_program(rng, n, 6 if n >= 300 else 10, p_meas=0.2 if n > 1 else 0.5, extra=True)
    if not np.any(ops[:, 0] == orc.MEASURE):
        ops = np.concatenate([ops, np.array([[orc.MEASURE, 0, 0]], dtype=np.uint32)])
    _check(n, ops, seed=int(rng.integers(1 << 30)), shots=shots)


def test_frames_repeated_qubit_in_one_segment():
    n = 4
    ops = np.array([[orc.H, 0, 0], [orc.CX, 0, 1], [orc.MEASURE, 0, 0], [orc.MEASURE, 0, 0], [orc.MEASURE, 1, 0],
                    [orc.H, 0, 0], [orc.MEASURE, 0, 0], [orc.MEASURE, 0, 0]], dtype=np.uint32)
    _check(n, ops, seed=3, shots=300)


def test_frames_config2_full():
    """n = 4096, depth 100, nine mid-circuit rounds of 409 qubits, then all 4096 (7777 measurements), 130 shots."""
    cfg = CONFIGS[2]
    o = circuit_ops(cfg)
    ops = np.stack([o["type"], o["q0"], o["q1"]], 1).astype(np.uint32)
    _check(cfg.n, ops, seed=cfg.seed, shots=130)


def test_frames_edge_cases():
    from paper_2603_14641_amd import Program, SqError
    n = 3
    ops = np.array([[orc.H, 0, 0], [orc.MEASURE, 0, 0]], dtype=np.uint32)
    p = Program(n, ops)
    assert p.frame_sample(0, ref=[0]).shape == (0, 1)
    with pytest.raises(SqError):
        p.frame_sample(10, ref=[2])
    gates_only = Program(n, np.array([[orc.H, 0, 0]], dtype=np.uint32))
    assert gates_only.frame_sample(5, ref=[]).shape == (5, 0)
