"""The CX-injection collapse (operator tableau, Algorithm alg:stim) on the GPU
against the operator-tableau oracle (oracle/stim_oracle.c), bit for bit:
the four bit matrices, both sign vectors, outcomes and random flags, with
tolerance 0 (needs an MI355X).

Mapping of the library's export in this mode onto the oracle's arrays:
row i < n of x/z is the destabilizer half (XD, ZD rows), row n + i the
stabilizer half (XS, ZS rows); sign byte i < n is SignsD[i] (the image of
X_i), n + i is SignsS[i] (the image of Z_i).

Larger sizes are checked against fixtures the oracle wrote
(tests/golden/inject_oracle.json, tests/golden/make_inject_fixtures.py),
and at full size (n = 65,536 and 180,000, depth 1000) by the outcomes of the
first final measurements, which equal the CHP oracle's stored outcomes
(tests/golden/full_size_oracle.json): both collapses give the same outcomes
under the same coins.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import mixed_program, segments
from oracle import oracle as orc
from workload import CONFIGS, circuit_ops

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _tab(n, **tuning):
    from paper_2603_14641_amd import COLLAPSE_INJECT, Tableau
    t = Tableau(n, collapse=COLLAPSE_INJECT)
    if tuning:
        t.set_tuning(**tuning)
    return t


def _assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        idx = np.argwhere(got != want)
        raise AssertionError(f"{what}: {idx.shape[0]} mismatches, first at {idx[:5].tolist()}")


def _sign_bytes(vec, n):
    return np.unpackbits(np.ascontiguousarray(vec, dtype="<u8").view(np.uint8), bitorder="little")[:n]


def _oracle_state(ot):
    xs, xd, zs, zd, ss, sd = ot.arrays()
    n = ot.n
    x = np.concatenate([xd, xs])
    z = np.concatenate([zd, zs])
    r = np.concatenate([_sign_bytes(sd, n), _sign_bytes(ss, n)]).astype(np.uint8)
    return x, z, r


def _compare(t, ot, what=""):
    x, z, r = t.export()
    rx, rz, rr = _oracle_state(ot)
    _assert_same(x, rx, f"{what} x bits")
    _assert_same(z, rz, f"{what} z bits")
    _assert_same(r, rr, f"{what} image signs")
    assert t.error_flags() == 0


def _run_calls(t, ops, seed, shot=0, meas_base=0):
    bits, rnd = [], []
    m = meas_base
    for kind, arr in segments(ops):
        if kind == "gates":
            t.apply_gates(arr)
        else:
            b, r = t.measure(arr, seed=seed, shot=shot, meas_base=m)
            bits.append(b)
            rnd.append(r)
            m += arr.size
    if not bits:
        return np.zeros(0, np.uint8), np.zeros(0, np.uint8)
    return np.concatenate(bits), np.concatenate(rnd)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 130, 700, 2500])
@pytest.mark.parametrize("path", ["calls", "program"])
def test_random_circuits(n, path):
    from paper_2603_14641_amd import Program
    rng = np.random.default_rng(900 + n)
    for trial in range(2):
        ops = mixed_program(rng, n, 6, p_meas=0.25, extra=n > 1)
        seed = int(rng.integers(1 << 40))
        ot = orc.OTableau(n)
        rb, rr = ot.run(ops, seed=seed, shot=3, meas_base=5)
        assert ot.odd_count == 0
        t = _tab(n)
        if path == "program":
            bits, rnd = t.run_to_host(Program(n, ops), seed=seed, shot=3, meas_base=5)
        else:
            bits, rnd = _run_calls(t, ops, seed, shot=3, meas_base=5)
        _assert_same(bits, rb, f"n={n} trial {trial} outcomes")
        _assert_same(rnd, rr, f"n={n} trial {trial} random flags")
        _compare(t, ot, f"n={n} trial {trial}")
        t.close()


@pytest.mark.parametrize("n", [1, 64, 65, 300, 1500])
def test_gate_passes_only(n):
    """Every gate type (CY, SWAP, iSWAP included) without measurements:
    multi-qubit groups of the pass compiler, bits and image signs."""
    rng = np.random.default_rng(40 + n)
    ops = mixed_program(rng, n, 12, p_meas=0.0, extra=n > 1)
    ot = orc.OTableau(n)
    ot.run(ops)
    t = _tab(n)
    t.apply_gates(ops)
    _compare(t, ot, f"n={n}")


def test_same_outcomes_as_rowsum_mode():
    """Both collapses give the same outcomes under the same coins, and
    gates move the same bits in both modes."""
    from paper_2603_14641_amd import Tableau
    n = 777
    rng = np.random.default_rng(5)
    ops = mixed_program(rng, n, 10, p_meas=0.3, extra=True)
    a = _tab(n)
    b = Tableau(n)
    ab, ar = _run_calls(a, ops, seed=99)
    bb, br = _run_calls(b, ops, seed=99)
    _assert_same(ab, bb, "outcomes")
    _assert_same(ar, br, "random flags")
    g = mixed_program(rng, n, 5, p_meas=0.0, extra=True)
    a.reset()
    b.reset()
    a.apply_gates(g)
    b.apply_gates(g)
    xa, za, _ = a.export()
    xb, zb, _ = b.export()
    _assert_same(xa, xb, "gate bits x")
    _assert_same(za, zb, "gate bits z")


def test_deep_pivots_and_sparse_targets():
    """Superpositions only on the first few and the last qubits of a wide
    register, so pivots and targets sit in far-apart words (and some
    measurements have no target besides the pivot)."""
    n = 20000
    rng = np.random.default_rng(17)
    ops = []
    hot = list(range(6)) + list(range(n - 150, n))
    for q in hot:
        ops.append([orc.H, q, 0])
    for _ in range(3):
        perm = rng.permutation(hot)
        for k in range(0, len(perm) - 1, 2):
            ops.append([orc.CX, int(perm[k]), int(perm[k + 1])])
        for q in rng.choice(hot, 40, replace=False):
            ops.append([int(rng.choice([orc.H, orc.S, orc.SDG, orc.Y])), int(q), 0])
    meas = list(rng.permutation(hot)) + [7, 8, n - 200] + list(rng.choice(hot, 30, replace=False))
    ops += [[orc.MEASURE, int(q), 0] for q in meas]
    ops = np.array(ops, dtype=np.uint32)
    ot = orc.OTableau(n)
    rb, rr = ot.run(ops, seed=123)
    t = _tab(n)
    bits, rnd = _run_calls(t, ops, seed=123)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    assert rnd.any() and not rnd.all()
    _compare(t, ot)


def test_program_graph_replay_and_reset():
    """A program run twice on the same tableau (its gate segments replay as
    graphs the second time), with a reset between: both runs equal the
    oracle. Switching the mode resets to |0...0>."""
    from paper_2603_14641_amd import COLLAPSE_INJECT, COLLAPSE_ROWSUM, Program, Tableau
    n = 400
    rng = np.random.default_rng(31)
    ops = mixed_program(rng, n, 8, p_meas=0.2, extra=True)
    ot = orc.OTableau(n)
    rb, rr = ot.run(ops, seed=8)
    t = _tab(n)
    prog = Program(n, ops)
    for k in range(3):
        t.reset()
        bits, rnd = t.run_to_host(prog, seed=8)
        _assert_same(bits, rb, f"run {k} outcomes")
        _assert_same(rnd, rr, f"run {k} flags")
        _compare(t, ot, f"run {k}")
    assert t.collapse == COLLAPSE_INJECT
    t.set_collapse(COLLAPSE_ROWSUM)
    assert t.collapse == COLLAPSE_ROWSUM
    z = Tableau(n)
    _assert_same(t.export()[0], z.export()[0], "reset x")
    t.set_collapse(COLLAPSE_INJECT)
    t.apply_gates(np.array([[orc.H, 0, 0]], dtype=np.uint32))
    with pytest.raises(Exception):
        t.sample([0], 4)


def test_import_export_roundtrip():
    """An oracle-made operator tableau imported, measured and exported."""
    n = 321
    rng = np.random.default_rng(77)
    ops = mixed_program(rng, n, 6, p_meas=0.1, extra=True)
    ot = orc.OTableau(n)
    ot.run(ops, seed=2)
    x, z, r = _oracle_state(ot)
    t = _tab(n)
    t.import_(x, z, r)
    _compare(t, ot, "imported")
    qs = rng.permutation(n)[:150].astype(np.uint32)
    meas = np.stack([np.full(qs.size, orc.MEASURE, np.uint32), qs, np.zeros(qs.size, np.uint32)], 1)
    rb, rr = ot.run(meas, seed=4, meas_base=10)
    bits, rnd = t.measure(qs, seed=4, meas_base=10)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare(t, ot, "measured")


def _digest_state(x, z, r):
    h = hashlib.sha256()
    for a in (x, z):
        h.update(np.ascontiguousarray(a, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(r, dtype=np.uint8).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("cfg_id", [1, 2])
def test_configs_against_stored_oracle(cfg_id):
    """Configs 1 and 2 in full (n = 64 and 4,096 with nine mid-circuit rounds),
    program path: outcomes, flags and the SHA-256 of the final operator
    tableau as the oracle stored them."""
    from paper_2603_14641_amd import Program
    fix = json.load(open(os.path.join(GOLDEN, "inject_oracle.json")))["configs"][str(cfg_id)]
    cfg = CONFIGS[cfg_id]
    ops = circuit_ops(cfg)
    t = _tab(cfg.n)
    bits, rnd = t.run_to_host(Program(cfg.n, ops), seed=fix["seed"], shot=0)
    _assert_same(bits, np.array([int(c) for c in fix["outcomes"]], np.uint8), "outcomes")
    _assert_same(rnd, np.array([int(c) for c in fix["random"]], np.uint8), "random flags")
    x, z, r = t.export()
    assert _digest_state(x, z, r) == fix["state_sha256"], "final operator tableau differs from the oracle's"
    assert t.error_flags() == 0


@pytest.mark.slow
@pytest.mark.parametrize("cfg_id", [3, 4])
@pytest.mark.timeout(600)
def test_full_size_outcomes_equal_chp_oracle(cfg_id):
    """Full depth (1000 layers) then the first final measurements, in the
    launch configuration the bench times: the outcomes equal the CHP oracle's
    stored outcomes, and the deterministic re-measurements repeat them."""
    import torch
    from paper_2603_14641_amd import Program
    fix = json.load(open(os.path.join(GOLDEN, "full_size_oracle.json")))["configs"][str(cfg_id)]
    cfg = CONFIGS[cfg_id]
    ops = circuit_ops(cfg, final_measure=False)
    gates = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
    m = int(fix["measurements"])
    print(f"config {cfg_id}: n={cfg.n}, inject collapse", flush=True)
    t = _tab(cfg.n)
    prog = Program(cfg.n, gates)
    t.run(prog, cfg.seed, 0, 0, 0, 0)
    prog.close()
    bits, flags = t.measure(np.arange(m), seed=cfg.seed, shot=0, meas_base=0)
    _assert_same(bits, np.array([int(c) for c in fix["outcomes"]], np.uint8), "outcomes")
    _assert_same(flags, np.array([int(c) for c in fix["random"]], np.uint8), "random flags")
    again, r2 = t.measure(np.arange(m), seed=cfg.seed + 1, shot=1, meas_base=m)
    _assert_same(again, bits, "re-measured outcomes")
    assert not r2.any()
    assert t.error_flags() == 0
    st = t.measure_stats()
    assert st.n_random == int(flags.sum()) and st.inject_bytes > 0
    t.close()
    torch.cuda.empty_cache()
