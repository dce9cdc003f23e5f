"""The row-contiguous layout (the in-place tile transpose, Algorithm
alg:transpose) and CHP measurements on whole rows, against the CPU oracle,
bit for bit (needs an MI355X).

  * the transposed block itself, read from its torch-owned device buffer
    (sq_create_in): slot r holds D_r's and S_r's bits exactly as the
    oracle's rows, and slots past n are zero; transposing back restores the
    column layout word for word;
  * measurements in the row layout (random and deterministic, repeated
    qubits, mid-circuit rounds with gate layers between them, which switch
    back to columns) equal the oracle's outcomes, flags and whole tableau;
  * at full size (n = 65,536 and 180,000, depth 1000): the first 128 final
    measurements in the row layout equal the oracle's stored outcomes, and
    the sampled rows after them its stored row digests.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import gpu_run_calls, mixed_program, oracle_run, segments
from oracle import oracle as orc
from workload import CONFIGS, circuit_ops

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        idx = np.argwhere(got != want)
        raise AssertionError(f"{what}: {idx.shape[0]} mismatches, first at {idx[:5].tolist()}")


def _torch_tableau(n):
    import torch
    from paper_2603_14641_amd import Tableau, binding
    info = binding.layout(n)
    buf = torch.empty(info["bytes"], dtype=torch.uint8, device="cuda")
    return Tableau(n, buffer=buf), buf, info


def _slots(buf, info, which):
    """All 64K slots of X (which=0) or Z (1) as a (64K, Ls) uint64 array."""
    import torch
    K, Ls = info["K"], info["Ls"]
    off = (info["x_offset"] if which == 0 else info["z_offset"]) // 8
    words = buf.view(torch.int64)[off:off + 64 * K * Ls]
    return words.view(64 * K, Ls).cpu().numpy().view(np.uint64)


# K = ceil(n / 64) covers the stabilizer half's grid shifts K mod 16 = 0, 1, 2, 4, 15
@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 960, 1024, 1100, 2047, 4100])
def test_transposed_block_is_row_major(n):
    from paper_2603_14641_amd import LAYOUT_COLUMNS, LAYOUT_ROWS
    rng = np.random.default_rng(n)
    ops = mixed_program(rng, n, 5, p_meas=0.1, extra=n > 1)
    _, _, x, z, r, _ = oracle_run(n, ops, seed=3)
    t, buf, info = _torch_tableau(n)
    gpu_run_calls(t, ops, seed=3)
    K = info["K"]
    t.sync()
    cols_x, cols_z = _slots(buf, info, 0).copy(), _slots(buf, info, 1).copy()
    t.set_layout(LAYOUT_ROWS)
    assert t.layout == LAYOUT_ROWS
    t.sync()
    for which, rows in ((0, x), (1, z)):
        s = _slots(buf, info, which)
        _assert_same(s[:n, :K], rows[:n], f"slot D-half words ({'xz'[which]})")
        _assert_same(s[:n, K:2 * K], rows[n:], f"slot S-half words ({'xz'[which]})")
        assert not s[n:, :2 * K].any(), "slots past n must stay zero"
    t.set_layout(LAYOUT_COLUMNS)
    t.sync()
    _assert_same(_slots(buf, info, 0)[:, :2 * K], cols_x[:, :2 * K], "x back in columns")
    _assert_same(_slots(buf, info, 1)[:, :2 * K], cols_z[:, :2 * K], "z back in columns")
    ex, ez, er = t.export()
    _assert_same(ex, x, "export x")
    _assert_same(ez, z, "export z")
    _assert_same(er, r, "export signs")
    t.close()


def _run_rows(t, ops, seed, shot=0, meas_base=0):
    """Measurement segments in the row layout, gates in columns (switched
    automatically by the gate calls)."""
    from paper_2603_14641_amd import LAYOUT_ROWS
    bits, rnd = [], []
    m = meas_base
    for kind, arr in segments(ops):
        if kind == "gates":
            t.apply_gates(arr)
        else:
            t.set_layout(LAYOUT_ROWS)
            b, r = t.measure(arr, seed=seed, shot=shot, meas_base=m)
            bits.append(b)
            rnd.append(r)
            m += arr.size
    if not bits:
        return np.zeros(0, np.uint8), np.zeros(0, np.uint8)
    return np.concatenate(bits), np.concatenate(rnd)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 130, 700, 2500, 5000])
def test_row_measurements_match_oracle(n):
    from paper_2603_14641_amd import Tableau
    rng = np.random.default_rng(300 + n)
    for trial in range(2):
        ops = mixed_program(rng, n, 5, p_meas=0.3, extra=n > 1)
        # then every qubit, then a repeat of some (deterministic)
        tail = np.concatenate([rng.permutation(n), rng.choice(n, max(1, n // 3), replace=False)])
        ops = np.concatenate([ops, np.stack([np.full(tail.size, orc.MEASURE), tail, np.zeros(tail.size)], 1)
                              .astype(np.uint32)])
        seed = int(rng.integers(1 << 40))
        rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=2, meas_base=9)
        t = Tableau(n)
        bits, rnd = _run_rows(t, ops, seed, shot=2, meas_base=9)
        _assert_same(bits, rb, f"n={n} trial {trial} outcomes")
        _assert_same(rnd, rr, f"n={n} trial {trial} random flags")
        ex, ez, er = t.export()
        _assert_same(ex, x, f"n={n} trial {trial} x")
        _assert_same(ez, z, f"n={n} trial {trial} z")
        _assert_same(er, r, f"n={n} trial {trial} signs")
        assert t.error_flags() == 0
        st = t.measure_stats()
        assert st.n_random == int(rr.sum()) and st.n_det == int(rr.size - rr.sum())
        t.close()


def test_rows_program_and_noalloc_paths():
    """sq_run measurement segments and sq_measure_noalloc in the row layout."""
    import ctypes
    from paper_2603_14641_amd import LAYOUT_ROWS, Program, Tableau, binding
    n = 900
    rng = np.random.default_rng(12)
    gates = mixed_program(rng, n, 6, p_meas=0.0, extra=True)
    meas = rng.permutation(n).astype(np.uint32)
    ops = np.concatenate([gates, np.stack([np.full(n, orc.MEASURE), meas, np.zeros(n)], 1).astype(np.uint32)])
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed=5)
    t = Tableau(n)
    t.apply_gates(gates)
    t.set_layout(LAYOUT_ROWS)
    bits, rnd = t.run_to_host(Program(n, ops[len(gates):]), seed=5)
    _assert_same(bits, rb, "program outcomes")
    _assert_same(rnd, rr, "program flags")
    _assert_same(t.export()[0], x, "program x")
    u = Tableau(n)
    u.apply_gates(gates)
    u.set_layout(LAYOUT_ROWS)
    out = np.zeros(n, np.uint8)
    fl = np.zeros(n, np.uint8)
    binding._check(u.lib.sq_measure_noalloc(u.h, meas.ctypes.data, n, 5, 0, 0, out.ctypes.data, fl.ctypes.data))
    _assert_same(out, rb, "noalloc outcomes")
    _assert_same(fl, rr, "noalloc flags")
    ex, ez, er = u.export()
    _assert_same(ex, x, "noalloc x")
    _assert_same(er, r, "noalloc signs")


def _row_digest(x, z, r):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(z, dtype="<u8").tobytes())
    h.update(bytes([int(r)]))
    return h.hexdigest()


@pytest.mark.slow
@pytest.mark.parametrize("cfg_id", [3, 4])
@pytest.mark.timeout(600)
def test_full_size_rows_against_stored_oracle(cfg_id):
    import torch
    from paper_2603_14641_amd import LAYOUT_ROWS, Program, Tableau
    fix = json.load(open(GOLDEN))["configs"][str(cfg_id)]
    cfg = CONFIGS[cfg_id]
    ops = circuit_ops(cfg, final_measure=False)
    gates = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
    m = int(fix["measurements"])
    print(f"config {cfg_id}: n={cfg.n}, row layout", flush=True)
    t = Tableau(cfg.n)
    prog = Program(cfg.n, gates)
    t.run(prog, cfg.seed, 0, 0, 0, 0)
    prog.close()
    t.set_layout(LAYOUT_ROWS)
    bits, flags = t.measure(np.arange(m), seed=cfg.seed, shot=0, meas_base=0)
    _assert_same(bits, np.array([int(c) for c in fix["outcomes"]], np.uint8), "outcomes")
    _assert_same(flags, np.array([int(c) for c in fix["random"]], np.uint8), "random flags")
    rows = fix["rows"]
    x, z, r = t.export_rows(rows)
    bad = [rows[i] for i in range(len(rows)) if _row_digest(x[i], z[i], r[i]) != fix["row_sha256"][i]]
    assert not bad, f"{len(bad)} of {len(rows)} sampled rows differ from the oracle, first {bad[:8]}"
    t.set_layout(LAYOUT_ROWS)
    again, r2 = t.measure(np.arange(m), seed=cfg.seed + 1, shot=1, meas_base=m)
    _assert_same(again, bits, "re-measured outcomes")
    assert not r2.any()
    assert t.error_flags() == 0
    t.close()
    torch.cuda.empty_cache()
