"""OpenQASM in, GPU out: a random circuit written as OpenQASM 2.0 text, read
by the library, run through a compiled program on the GPU and compared bit
for bit with the oracle on the same records."""
import numpy as np
import pytest

from gpu_util import mixed_program, oracle_run
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

NAMES = {orc.H: "h", orc.S: "s", orc.SDG: "sdg", orc.X: "x", orc.Y: "y", orc.Z: "z", orc.CX: "cx", orc.CZ: "cz",
         orc.CY: "cy", orc.SWAP: "swap", orc.ISWAP: "iswap"}


def to_qasm(n, ops):
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n}];", f"creg c[{n}];"]
    for t, a, b in ops.tolist():
        if t == orc.MEASURE:
            lines.append(f"measure q[{a}] -> c[{a}];")
        elif t in (orc.CX, orc.CZ, orc.CY, orc.SWAP, orc.ISWAP):
            lines.append(f"{NAMES[t]} q[{a}], q[{b}];")
        else:
            lines.append(f"{NAMES[t]} q[{a}];")
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()


@pytest.mark.parametrize("n", [3, 70, 400])
def test_qasm_program_matches_oracle(n):
    from paper_2603_14641_amd import Program, Tableau, parse_qasm
    rng = np.random.default_rng(900 + n)
    ops = mixed_program(rng, n, 10, p_meas=0.2, extra=True)
    n2, parsed = parse_qasm(to_qasm(n, ops))
    assert n2 == n and np.array_equal(parsed, ops)
    rb, rr, x, z, r, _ = oracle_run(n, parsed, seed=7)
    t = Tableau(n)
    bits, rnd = t.run_to_host(Program(n, parsed), seed=7, shot=0)
    assert np.array_equal(bits, rb) and np.array_equal(rnd, rr)
    gx, gz, gr = t.export()
    assert np.array_equal(gx, x) and np.array_equal(gz, z) and np.array_equal(gr, r)
