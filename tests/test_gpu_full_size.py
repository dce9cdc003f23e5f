"""Full-size checks of configs 3 and 4 (n = 65,536 and 180,000, depth 1000)
in the launch configuration bench.py times (needs an MI355X).

Two kinds of evidence, both bit-exact:
  * the oracle on sampled rows (tests/golden/full_size_oracle.json, written
    by tests/golden/make_full_size_fixtures.py, which calls only oracle/ and
    workload/): rows evolve independently under gates and the random-case
    update of a row needs only that row and S_p, so an oracle holding a
    sample of rows plus the stabilizer prefix that contains every pivot
    reproduces those rows and the first outcomes exactly;
  * the whole final sweep (every qubit measured, in order) checked by
    properties that hold at any size, on the tableau read in place from its
    torch-owned device block (sq_create_in): every stabilizer is a Z string
    whose sign is its parity over the outcomes, each one a single +-Z_q when
    every outcome was random, the symplectic form intact (Freivalds probes),
    and re-measured qubits deterministic with the same outcomes.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import tableau_checks as tc
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


def _gates(cfg):
    ops = circuit_ops(cfg, final_measure=False)
    return np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)


def _torch_tableau(n):
    """A tableau in a torch-owned device block, and its views."""
    import torch
    from paper_2603_14641_amd import Tableau, binding
    info = binding.layout(n)
    buf = torch.empty(info["bytes"], dtype=torch.uint8, device="cuda")
    t = Tableau(n, buffer=buf)
    return t, buf, info


def _meas_ops(qubits):
    return np.array([[orc.MEASURE, int(q), 0] for q in qubits], dtype=np.uint32).reshape(-1, 3)


def _row_digest(x, z, r):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(z, dtype="<u8").tobytes())
    h.update(bytes([int(r)]))
    return h.hexdigest()


def _full_depth_then_sweep(cfg_id, seed_again):
    """Gates of the full circuit; the first M final measurements and the
    sampled rows against the oracle's stored result; then the rest of the
    sweep and its invariants."""
    import torch
    from paper_2603_14641_amd import Program
    fix = json.load(open(GOLDEN))["configs"][str(cfg_id)]
    cfg = CONFIGS[cfg_id]
    n = cfg.n
    assert fix["n"] == n and fix["depth"] == cfg.depth and fix["seed"] == cfg.seed
    gates = _gates(cfg)
    assert gates.shape[0] == fix["gates"]
    m = int(fix["measurements"])
    rows = fix["rows"]
    print(f"config {cfg_id}: n={n}, {gates.shape[0]} gates", flush=True)
    t, buf, info = _torch_tableau(n)
    prog = Program(n, gates)
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    rnd = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t.run(prog, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    prog.close()
    # the first measurements of the final sweep, against the oracle
    bits, flags = t.measure(np.arange(m), seed=cfg.seed, shot=0, meas_base=0)
    _assert_same(bits, np.array([int(c) for c in fix["outcomes"]], dtype=np.uint8), "outcomes")
    _assert_same(flags, np.array([int(c) for c in fix["random"]], dtype=np.uint8), "random flags")
    x, z, r = t.export_rows(rows)
    bad = [rows[i] for i in range(len(rows)) if _row_digest(x[i], z[i], r[i]) != fix["row_sha256"][i]]
    assert not bad, f"{len(bad)} of {len(rows)} sampled rows differ from the oracle, first {bad[:8]}"
    assert t.error_flags() == 0
    print(f"config {cfg_id}: oracle parity on {len(rows)} rows and {m} outcomes", flush=True)
    # the rest of the sweep, as one program segment (index base m)
    rest = Program(n, _meas_ops(range(m, n)))
    t.run(rest, cfg.seed, 0, m, out[m:].data_ptr(), rnd[m:].data_ptr())
    t.sync()
    rest.close()
    assert t.error_flags() == 0
    allbits = np.concatenate([bits, out.cpu().numpy()[m:]])
    allrnd = np.concatenate([flags, rnd.cpu().numpy()[m:]])
    print(f"config {cfg_id}: sweep done, {int(allrnd.sum())} of {n} random", flush=True)
    X, Z, R = tc.views(buf, info)
    K = info["K"]
    x_zero, signs_ok = tc.basis_state_stabilizers(X, Z, R, n, K, allbits)
    assert x_zero, "a stabilizer still has an x bit after every qubit was measured"
    assert signs_ok, "a stabilizer sign differs from its Z string's parity over the outcomes"
    if allrnd.all():
        assert tc.stabilizers_are_distinct_single_z(Z, n, K), "stabilizers are not distinct single Z's"
    assert tc.freivalds_symplectic(X, Z, n, K, probes=3, seed=cfg_id) == 0, "symplectic form broken"
    # re-measuring gives the same outcomes, deterministically
    rng = np.random.default_rng(seed_again)
    again = np.sort(rng.choice(n, 24, replace=False))
    b2, r2 = t.measure(again, seed=cfg.seed + 1, shot=1, meas_base=n)
    _assert_same(b2, allbits[again], "re-measured outcomes")
    assert not r2.any(), "a re-measurement was random"
    assert t.error_flags() == 0
    t.close()
    del buf
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_config3_full_depth_and_full_sweep():
    _full_depth_then_sweep(3, seed_again=303)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_config4_full_depth_and_full_sweep():
    _full_depth_then_sweep(4, seed_again=404)
