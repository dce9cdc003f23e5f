"""The OpenQASM 2.0 reader (host only): records, register numbering,
broadcasting, gate definitions, and every rejection path with its line."""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2603_14641_amd import binding as sqb

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse(text):
    return sqb.parse_qasm(text)


def test_ghz_file_over_two_registers():
    n, ops = parse(open(os.path.join(GOLDEN, "ghz_registers.qasm")).read())
    assert n == 5
    want = [[sqb.H, 0, 0], [sqb.CX, 0, 1], [sqb.CX, 1, 2], [sqb.CX, 2, 3], [sqb.CX, 3, 4]]
    want += [[sqb.MEASURE, q, 0] for q in range(5)]
    assert ops.tolist() == want
    # the oracle on the parsed circuit: a GHZ state, every outcome equals the first
    for seed in range(8):
        bits, rnd, _ = orc.Tableau(n).run(ops, seed=seed)
        assert len(set(bits.tolist())) == 1 and rnd.tolist() == [1, 0, 0, 0, 0]


def test_broadcast_and_whole_register_measure():
    n, ops = parse("""OPENQASM 2.0; qreg p[2]; qreg r[2]; creg c[2];
        h p; cx p, r; s r[1]; sdg p[0]; y r; measure r -> c;""")
    assert n == 4
    assert ops.tolist() == [[sqb.H, 0, 0], [sqb.H, 1, 0], [sqb.CX, 0, 2], [sqb.CX, 1, 3], [sqb.S, 3, 0],
                            [sqb.SDG, 0, 0], [sqb.Y, 2, 0], [sqb.Y, 3, 0], [sqb.MEASURE, 2, 0], [sqb.MEASURE, 3, 0]]


def test_every_gate_name():
    n, ops = parse("""qreg q[2];
        id q[0]; x q[0]; y q[0]; z q[0]; h q[0]; s q[0]; sdg q[0];
        cx q[0],q[1]; CX q[1],q[0]; cy q[0],q[1]; cz q[0],q[1]; swap q[0],q[1]; iswap q[1],q[0];""")
    assert n == 2
    assert [int(t) for t in ops[:, 0]] == [sqb.X, sqb.Y, sqb.Z, sqb.H, sqb.S, sqb.SDG, sqb.CX, sqb.CX, sqb.CY,
                                          sqb.CZ, sqb.SWAP, sqb.ISWAP]
    assert ops[7].tolist() == [sqb.CX, 1, 0] and ops[-1].tolist() == [sqb.ISWAP, 1, 0]


def test_gate_definitions_expand_in_order():
    n, ops = parse("""qreg q[3];
        gate bell a, b { h a; cx a, b; }
        gate chain a, b, c { bell a, b; barrier a, b, c; cx b, c; }
        chain q[2], q[0], q[1];""")
    assert ops.tolist() == [[sqb.H, 2, 0], [sqb.CX, 2, 0], [sqb.CX, 0, 1]]


def test_definition_of_a_known_gate_keeps_the_builtin():
    """Qiskit writes a definition of iswap before using it; the reader keeps
    its own iswap, and the written body gives the same tableau."""
    body = "s q0; s q1; h q0; cx q0, q1; cx q1, q0; h q1;"
    _, ops = parse("qreg q[2]; gate iswap q0, q1 { " + body + " } iswap q[0], q[1];")
    assert ops.tolist() == [[sqb.ISWAP, 0, 1]]
    _, expanded = parse("qreg q[2]; gate my_iswap q0, q1 { " + body + " } my_iswap q[0], q[1];")
    assert len(expanded) == 6
    prefix = np.array([[sqb.H, 0, 0], [sqb.S, 1, 0], [sqb.CX, 0, 1], [sqb.H, 1, 0]], dtype=np.uint32)
    a = orc.Tableau(2)
    a.run(np.concatenate([prefix, ops]))
    b = orc.Tableau(2)
    b.run(np.concatenate([prefix, expanded]))
    for u, v in zip(a.rows_array(), b.rows_array()):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("text,line,what", [
    ("qreg q[2];\nrz(pi/2) q[0];", 2, "parameters"),
    ("qreg q[2];\n\nreset q[0];", 3, "not supported"),
    ("qreg q[2];\nt q[0];", 2, "unknown gate 't'"),
    ("qreg q[2];\nh q[2];", 2, "out of range"),
    ("qreg q[2];\nh q[0]\nh q[1];", 3, "expected ';'"),
    ("qreg q[2]; creg c[1];\nmeasure q -> c;", 2, "differ in size"),
    ("qreg q[2];\ncx q[1], q[1];", 2, "same qubit twice"),
    ("qreg q[2]; qreg r[3];\ncx q, r;", 2, "different sizes"),
    ("qreg q[2];\nh r[0];", 2, "unknown quantum register"),
    ("OPENQASM 3.0;", 1, "only OpenQASM 2.0"),
    ("qreg q[1];\ngate g(t) a { h a; }", 2, "parameters"),
    ("qreg q[1];\nif (c == 1) x q[0];", 2, "not supported"),
    ("qreg q[2];\ncx q[0];", 2, "takes 2 qubit"),
])
def test_rejections_name_the_line(text, line, what):
    with pytest.raises(sqb.SqError) as e:
        parse(text)
    assert e.value.status == sqb.SQ_EINVAL
    msg = str(e.value)
    assert f"line {line}" in msg and what in msg, msg


def test_empty_and_comment_only():
    n, ops = parse("// nothing here\nOPENQASM 2.0;\n")
    assert n == 0 and ops.shape == (0, 3)
