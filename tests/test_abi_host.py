"""CPU-only checks of the C ABI library: it loads, exports every declared
symbol, agrees on type codes, validates arguments, and its host-side gate-pass
compiler preserves program order semantics (checked with the oracle)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workload
from oracle import oracle as orc
from paper_2603_14641_amd import binding as sqb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sq_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sqb.load()
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sqb.EXPORTED)


def test_type_codes_agree():
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(SQ_[A-Z]+) = (\d+)", text))
    for name in ["I", "H", "S", "SDG", "X", "Y", "Z", "CX", "CZ", "CY", "SWAP", "ISWAP", "MEASURE"]:
        assert codes["SQ_" + name] == getattr(sqb, name) == getattr(orc, name)
    assert workload.GATE_CX == sqb.CX and workload.GATE_CZ == sqb.CZ and workload.OP_MEASURE == sqb.MEASURE
    assert workload.GATE_SDG == sqb.SDG and workload.GATE_Y == sqb.Y
    assert (workload.GATE_CY, workload.GATE_SWAP, workload.GATE_ISWAP) == (sqb.CY, sqb.SWAP, sqb.ISWAP)


def test_bytes_required():
    assert sqb.bytes_required(0) == 0
    assert sqb.bytes_required(2**20 + 1) == 0
    b = sqb.bytes_required(180000)
    tableau = 2 * 180000 * 5632 * 8
    assert tableau < b < tableau * 1.05


def test_version_and_last_error():
    assert "sq" in sqb.version()
    lib = sqb.load()
    assert lib.sq_sync(None) == sqb.SQ_EINVAL
    assert b"NULL" in lib.sq_last_error()


def test_null_handles_are_rejected_without_a_device():
    """Entry points given a NULL handle or output return SQ_EINVAL with a
    message, before touching any device."""
    import ctypes
    lib = sqb.load()
    c, r = ctypes.c_uint64(0), ctypes.c_uint64(0)
    calls = [
        lambda: lib.sq_set_graphs(None, 1),
        lambda: lib.sq_graph_stats(None, ctypes.byref(c), ctypes.byref(r)),
        lambda: lib.sq_apply_gates(None, None, 0),
        lambda: lib.sq_reset(None),
        lambda: lib.sq_run(None, None, 0, 0, 0, None, None),
        lambda: lib.sq_set_tuning(None, None),
        lambda: lib.sq_profile_enable(None, 1),
        lambda: lib.sq_set_collapse(None, sqb.COLLAPSE_INJECT),
        lambda: lib.sq_set_layout(None, sqb.LAYOUT_ROWS),
        lambda: lib.sq_measure_noalloc(None, None, 1, 0, 0, 0, None, None),
    ]
    for call in calls:
        assert call() == sqb.SQ_EINVAL
        assert lib.sq_last_error()
    assert lib.sq_get_collapse(None) == sqb.COLLAPSE_ROWSUM
    assert lib.sq_get_layout(None) == sqb.LAYOUT_COLUMNS


def test_layout_holds_64k_slots():
    """X and Z are allocated with 64 * ceil(n / 64) column slots (the row
    layout needs each half to be a square bit matrix), at the reported
    offsets, and the block is large enough for both."""
    for n in (1, 63, 64, 65, 180000):
        info = sqb.layout(n)
        K, Ls = info["K"], info["Ls"]
        assert info["L"] == 2 * K and Ls % 16 == 0 and Ls >= 2 * K
        assert info["z_offset"] - info["x_offset"] >= 64 * K * Ls * 8
        assert info["r_offset"] - info["z_offset"] >= 64 * K * Ls * 8
        assert info["bytes"] == sqb.bytes_required(n)


# ---------------------------------------------------------------- pass compiler
WOP_1Q = {1: orc.H, 2: orc.S, 3: orc.SDG, 4: orc.X, 5: orc.Y, 6: orc.Z}
MAXQ, MAXOPS = 8, 32


def plan_to_gates(plan):
    """Turn a pass plan back into a flat gate list (pass by pass, group by group)."""
    gates = []
    for groups in plan:
        qubits = []
        for hdr, qs, uops in groups:
            qubits += qs
            for u in uops:
                t, a, b = u & 15, (u >> 4) & 15, (u >> 8) & 15
                if t in WOP_1Q:
                    gates.append([WOP_1Q[t], qs[a], 0])
                else:
                    assert a != b
                    gates.append([{7: orc.CX, 8: orc.CZ, 9: orc.SWAP}[t], qs[a], qs[b]])
        assert len(set(qubits)) == len(qubits), "groups of a pass must be disjoint"
    return np.array(gates, dtype=np.uint32).reshape(-1, 3)


def changed_flags(qs, uops):
    """x and z change flags per slot, from the gate rules: H changes both, S/S^dagger z,
    CX(c, t) x_t and z_c, CZ both z; X/Y/Z only signs."""
    dx = dz = 0
    for u in uops:
        t, a, b = u & 15, (u >> 4) & 15, (u >> 8) & 15
        if t == 1:
            dx |= 1 << a
            dz |= 1 << a
        elif t in (2, 3):
            dz |= 1 << a
        elif t == 7:
            dx |= 1 << b
            dz |= 1 << a
        elif t == 8:
            dz |= (1 << a) | (1 << b)
        elif t == 9:
            dx |= (1 << a) | (1 << b)
            dz |= (1 << a) | (1 << b)
    return (dx << 16) | (dz << 24)


def check_group(hdr, qs, uops):
    assert 1 <= len(qs) <= MAXQ and 1 <= len(uops) <= MAXOPS
    assert (hdr & 15) == len(qs) and ((hdr >> 4) & 63) == len(uops)
    assert (hdr & 0xFFFF0000) == changed_flags(qs, uops)
    assert len(set(qs)) == len(qs)
    used = set()
    for u in uops:
        used.add((u >> 4) & 15)
        if (u & 15) >= 7:
            used.add((u >> 8) & 15)
    assert used == set(range(len(qs))), "every slot is used and no other"


def random_gates(rng, n, count):
    out = []
    for _ in range(count):
        t = int(rng.integers(0, 12 if n > 1 else 7))
        if t in orc.TWO_QUBIT:
            a, b = rng.choice(n, 2, replace=False)
            out.append([t, int(a), int(b)])
        else:
            out.append([t, int(rng.integers(n)), 0])
    return np.array(out, dtype=np.uint32).reshape(-1, 3)


def tableau_after(n, gates):
    t = orc.Tableau(n)
    t.run(gates)
    return t.rows_array()


@pytest.mark.parametrize("n,count", [(1, 30), (2, 60), (3, 200), (7, 300), (40, 600)])
def test_pass_plan_equals_program_order(n, count):
    rng = np.random.default_rng(n * 1000 + count)
    for _ in range(5):
        gates = random_gates(rng, n, count)
        plan = sqb.plan_gates(n, gates)
        for groups in plan:
            for g in groups:
                check_group(*g)
        flat = plan_to_gates(plan)
        want = tableau_after(n, gates)
        got = tableau_after(n, flat)
        for u, v in zip(want, got):
            assert np.array_equal(u, v)


def test_chunked_plan_equals_program_order():
    """Gate lists of 2^20 ops or more are compiled in chunks of 2^19 ops on
    helper threads; the concatenated plan must still apply the gates in
    program order (here three chunks, every gate type, n = 12)."""
    rng = np.random.default_rng(77)
    n, count = 12, (1 << 20) + 12345
    t = rng.integers(0, 12, count).astype(np.uint32)
    a = rng.integers(0, n, count).astype(np.uint32)
    b = ((a + 1 + rng.integers(0, n - 1, count)) % n).astype(np.uint32)
    two = np.isin(t, orc.TWO_QUBIT)
    gates = np.stack([t, a, np.where(two, b, 0)], 1).astype(np.uint32)
    plan = sqb.plan_gates(n, gates)
    for groups in plan[::97]:
        for g in groups:
            check_group(*g)
    flat = plan_to_gates(plan)
    want = tableau_after(n, gates)
    got = tableau_after(n, flat)
    for u, v in zip(want, got):
        assert np.array_equal(u, v)


def test_plan_of_generator_layers_spans_several_layers_per_pass():
    """Groups keep absorbing later layers on their qubits, so a pass covers
    more than one generator layer and streams fewer columns than one per
    qubit and layer."""
    depth = 20
    cfg = workload.circuits.CircuitConfig("gen4096", 4096, depth, 1, cz=True, mid_measure=False)
    ops = workload.circuit_ops(cfg, final_measure=False)
    plan = sqb.plan_gates(cfg.n, ops)
    assert len(plan) < 0.6 * depth
    cols = 0
    for groups in plan:
        for g in groups:
            check_group(*g)
            cols += len(g[1])
    assert cols < 0.5 * cfg.n * depth
    gates = ops[ops["type"] != workload.GATE_I]
    flat = plan_to_gates(plan)
    assert flat.shape[0] == gates.shape[0]


def test_plan_long_single_qubit_runs_split():
    # 40 gates on one qubit need two groups of at most 32 micro-ops
    gates = np.array([[orc.S, 0, 0]] * 40, dtype=np.uint32)
    plan = sqb.plan_gates(1, gates)
    assert [len(p) for p in plan] == [1, 1]
    assert [len(p[0][2]) for p in plan] == [32, 8]
    assert plan_to_gates(plan).shape[0] == 40


def test_plan_cx_chain_caps_group_size():
    """A CX chain links every qubit: groups stop at 8 qubits and the rest
    moves to later passes, in order."""
    n = 30
    gates = np.array([[orc.CX, q, q + 1] for q in range(n - 1)], dtype=np.uint32)
    plan = sqb.plan_gates(n, gates)
    assert len(plan) > 1
    for groups in plan:
        for g in groups:
            check_group(*g)
    want = tableau_after(n, gates)
    got = tableau_after(n, plan_to_gates(plan))
    for u, v in zip(want, got):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("bad,status", [
    ([[orc.CX, 0, 0]], sqb.SQ_EINVAL),
    ([[orc.H, 5, 0]], sqb.SQ_ERANGE),
    ([[orc.CZ, 1, 9]], sqb.SQ_ERANGE),
    ([[11, 0, 0]], sqb.SQ_EINVAL),
    ([[orc.MEASURE, 0, 0]], sqb.SQ_EINVAL),
])
def test_plan_rejects_bad_ops(bad, status):
    with pytest.raises(sqb.SqError) as e:
        sqb.plan_gates(5, np.array(bad, dtype=np.uint32))
    assert e.value.status == status


def test_batch_sample_joins_workers_when_the_batch_allocation_fails():
    """sq_batch_sample with one item for the persistent launch and one for the
    worker threads, on a machine where every device call fails: the batch's
    device allocation fails while a worker thread may still run, and the call
    must return an error (joining its workers) rather than end the process.
    Run in a child process so that a termination would fail the test instead
    of the test session."""
    import subprocess
    import sys
    code = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_2603_14641_amd import binding as sqb
reqs = [dict(n=16, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(16, dtype=np.uint32), shots=2),
        dict(n=3000, ops=np.zeros((0, 3), np.uint32), qubits=np.arange(3000, dtype=np.uint32), shots=2)]
try:
    sqb.batch_sample(reqs, max_batch_n=1024, streams=1)
except sqb.SqError as e:
    print("status", e.status)
    sys.exit(0)
print("no error")
sys.exit(3)
'''
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1")
    res = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True, timeout=120, env=env)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr[-2000:])
    assert "status" in res.stdout
