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
    for name in ["I", "H", "S", "SDG", "X", "Y", "Z", "CX", "CZ", "MEASURE"]:
        assert codes["SQ_" + name] == getattr(sqb, name) == getattr(orc, name)
    assert workload.GATE_CX == sqb.CX and workload.GATE_CZ == sqb.CZ and workload.OP_MEASURE == sqb.MEASURE
    assert workload.GATE_SDG == sqb.SDG and workload.GATE_Y == sqb.Y


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


# ---------------------------------------------------------------- pass compiler
UOP_1Q = {1: orc.H, 2: orc.S, 3: orc.SDG, 4: orc.X, 5: orc.Y, 6: orc.Z}


def plan_to_gates(plan):
    """Turn a pass plan back into a flat gate list (pass by pass, group by group)."""
    gates = []
    for groups in plan:
        qubits = []
        for q0w, q1, ops in groups:
            a = q0w & 0xFFFFFF
            qubits.append(a)
            if q1 != 0xFFFFFFFF:
                qubits.append(q1)
            while ops:
                c = ops & 15
                ops >>= 4
                if c <= 6:
                    gates.append([UOP_1Q[c], a, 0])
                elif c <= 12:
                    gates.append([UOP_1Q[c - 6], q1, 0])
                elif c == 13:
                    gates.append([orc.CX, a, q1])
                elif c == 14:
                    gates.append([orc.CX, q1, a])
                else:
                    gates.append([orc.CZ, a, q1])
        assert len(set(qubits)) == len(qubits), "groups of a pass must be disjoint"
    return np.array(gates, dtype=np.uint32).reshape(-1, 3)


def changed_flags(ops):
    f = 0
    while ops:
        c = ops & 15
        ops >>= 4
        f |= {1: 3, 2: 2, 3: 2, 7: 12, 8: 8, 9: 8, 13: 6, 14: 9, 15: 10}.get(c, 0)
    return f


def random_gates(rng, n, count):
    out = []
    for _ in range(count):
        t = int(rng.integers(0, 9 if n > 1 else 7))
        if t in (orc.CX, orc.CZ):
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
            for q0w, q1, ops in groups:
                assert (q0w >> 24) == changed_flags(ops)
        flat = plan_to_gates(plan)
        want = tableau_after(n, gates)
        got = tableau_after(n, flat)
        for u, v in zip(want, got):
            assert np.array_equal(u, v)


def test_plan_of_generator_layer_is_one_pass_per_layer():
    cfg = workload.CONFIGS[2]
    ops = workload.circuit_ops(cfg, depth=3, final_measure=False)
    plan = sqb.plan_gates(cfg.n, ops)
    assert len(plan) == 3
    gates = ops[ops["type"] != workload.GATE_I]
    flat = plan_to_gates(plan)
    assert flat.shape[0] == gates.shape[0]


def test_plan_long_single_qubit_runs_split():
    # 40 gates on one qubit need three groups of at most 16 micro-ops
    gates = np.array([[orc.S, 0, 0]] * 40, dtype=np.uint32)
    plan = sqb.plan_gates(1, gates)
    assert [len(p) for p in plan] == [1, 1, 1]
    assert plan_to_gates(plan).shape[0] == 40


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
