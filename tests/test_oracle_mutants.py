"""Planted mistakes: each plausible slip in the oracle must fail a pin.

Every mutant is a copy of oracle/chp_oracle.c with one textual change,
compiled on the CPU into a temporary library and run through compact versions
of the pins in test_oracle_pins.py (numpy Philox, gate conjugation by
matrices, brute-force state vectors with the Born rule, and the matrix form of
the measurement update). A mutant that survives every pin means the pins are
too weak.

Swapping the two operands of g is not listed: CHP only multiplies commuting
rows, whose phase sum is 0 or 2 (mod 4) and so is the same in either order.
"""
import os
import tempfile

import numpy as np
import pytest

import statevec as sv
from oracle import oracle as orc

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "chp_oracle.c")

MUTANTS = {
    "H drops sign": ("      *r ^= (uint8_t)(xa & za);\n      putb(x, a, za);", "      putb(x, a, za);"),
    "S writes x": ("    case SQO_S:\n      *r ^= (uint8_t)(xa & za);\n      putb(z, a, za ^ xa);",
                   "    case SQO_S:\n      *r ^= (uint8_t)(xa & za);\n      putb(x, a, za ^ xa);"),
    "SDG sign as S": ("*r ^= (uint8_t)(xa & (za ^ 1));", "*r ^= (uint8_t)(xa & za);"),
    "Y sign and": ("*r ^= (uint8_t)(xa ^ za);", "*r ^= (uint8_t)(xa & za);"),
    "CX sign term": ("(xb ^ za ^ 1)", "(xb ^ za)"),
    "CX target z": ("putb(z, a, za ^ zb);", "putb(z, b, za ^ zb);"),
    "CZ misses b": ("putb(z, b, zb ^ xa);", "putb(z, b, zb);"),
    "rowsum drops r_i": ("int e = 2 * (int)*rh + 2 * (int)ri + g;", "int e = 2 * (int)*rh + g;"),
    "g table Y sign": ("(p_y & ~x2 & z2)", "(p_y & x2 & ~z2)"),
    "pivot is largest": ("{ p = (int32_t)i; break; }", "{ p = (int32_t)i; }"),
    "skip D rows": ("if ((uint32_t)h == sp || (int32_t)h == dp) continue;",
                    "if ((uint32_t)h == sp || (int32_t)h == dp || t->gid[h] < t->n) continue;"),
    "D_p not replaced": ("if (dp >= 0) {", "if (0) {"),
    "S_p sign not coin": ("t->r[sp] = (uint8_t)coin;", "t->r[sp] = 0;"),
    "det uses S half": ("if (!getb(ROWX(t, (uint32_t)t->local[i]), q)) continue;",
                        "if (!getb(ROWX(t, (uint32_t)t->local[n + i]), q)) continue;"),
    "philox 9 rounds": ("round < 10", "round < 9"),
    "coin from word 1": ("return (int)(out[0] & 1);", "return (int)(out[1] & 1);"),
    "SWAP keeps z_a": ("      putb(z, a, zb);\n", ""),
    "CY S order": ("    gate_on_row(x, z, r, SQO_SDG, b, 0);\n    gate_on_row(x, z, r, SQO_CX, a, b);\n"
                   "    gate_on_row(x, z, r, SQO_S, b, 0);",
                   "    gate_on_row(x, z, r, SQO_S, b, 0);\n    gate_on_row(x, z, r, SQO_CX, a, b);\n"
                   "    gate_on_row(x, z, r, SQO_SDG, b, 0);"),
    "frames start at z = 0": ("    for (uint32_t q = 0; q < n; ++q) putb(z, q, sqo_frame_bit(seed, (uint64_t)s, q));\n", ""),
    "frames keep z after measuring": ("        putb(z, a, sqo_frame_bit(seed, (uint64_t)s, (uint64_t)n + i));\n", ""),
    "frames record z": ("const int bit = (int)(ref[i] & 1) ^ getb(x, a);", "const int bit = (int)(ref[i] & 1) ^ getb(z, a);"),
    "frames drop the reference": ("const int bit = (int)(ref[i] & 1) ^ getb(x, a);", "const int bit = getb(x, a);"),
    "iSWAP drops S_b": ("    gate_on_row(x, z, r, SQO_S, b, 0);\n    gate_on_row(x, z, r, SQO_CZ, a, b);",
                        "    gate_on_row(x, z, r, SQO_CZ, a, b);"),
}


def _program(rng, n, length, p_meas):
    ops = []
    for _ in range(length):
        if rng.random() < p_meas:
            ops.append([orc.MEASURE, int(rng.integers(n)), 0])
            continue
        t = int(rng.integers(1, 12))
        if t in orc.TWO_QUBIT:
            a, b = rng.choice(n, 2, replace=False)
            ops.append([t, int(a), int(b)])
        else:
            ops.append([t, int(rng.integers(n)), 0])
    return np.array(ops, dtype=np.uint32).reshape(-1, 3)


def pin_philox(lib):
    bg = np.random.Philox(key=np.array([5, 6], dtype=np.uint64), counter=8)
    want = bg.random_raw(4).astype(np.uint64)
    c = np.array([9, 0, 0, 0], dtype=np.uint64)
    k = np.array([5, 6], dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.sqo_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    assert np.array_equal(out, want)
    for m in range(1, 40):
        bg = np.random.Philox(key=np.array([2, 3], dtype=np.uint64), counter=m - 1)
        assert lib.sqo_coin(2, 3, m) == int(bg.random_raw(1)[0]) & 1


def pin_gates(lib):
    n = 2
    for typ in range(1, 12):
        placements = [(0, 1), (1, 0)] if typ in orc.TWO_QUBIT else [(0, 0), (1, 0)]
        for a, b in placements:
            u = sv.gate_unitary(n, typ, a, b)
            for code in range(16):
                t = orc.Tableau(n, lib=lib)
                x, z, r = t.rows_array()
                x[:] = 0
                z[:] = 0
                r[:] = 0
                x[0, 0] = code & 3
                z[0, 0] = code >> 2
                t.set_rows(x, z, r)
                t.run(np.array([[typ, a, b]], dtype=np.uint32))
                x2, z2, r2 = t.rows_array()
                want = u @ sv.row_matrix(x[0], z[0], 0, n) @ u.conj().T
                assert np.allclose(sv.row_matrix(x2[0], z2[0], int(r2[0]), n), want)


def pin_state_vector(lib):
    rng = np.random.default_rng(17)
    for n in (3, 4):
        for trial in range(8):
            prog = _program(rng, n, 40, 0.2)
            t = orc.Tableau(n, lib=lib)
            psi = sv.zero_state(n)
            m = 0
            for op in prog:
                if op[0] != orc.MEASURE:
                    t.run(op.reshape(1, 3))
                    psi = sv.apply_gate(psi, n, int(op[0]), int(op[1]), int(op[2]))
                    continue
                q = int(op[1])
                bits, rnd, _ = t.run(op.reshape(1, 3), seed=trial, shot=0, meas_base=m)
                p1 = sv.prob_one(psi, n, q)
                if abs(p1 - 0.5) < 1e-9:
                    assert rnd[0] == 1
                    bg = np.random.Philox(key=np.array([trial, 0], dtype=np.uint64),
                                          counter=m - 1 if m else 2**256 - 1)
                    assert bits[0] == int(bg.random_raw(1)[0]) & 1
                else:
                    assert rnd[0] == 0 and abs(p1 - bits[0]) < 1e-9
                psi = sv.project(psi, q, int(bits[0]))
                m += 1
                x, z, r = t.rows_array()
                for i in range(n):
                    s = sv.row_matrix(x[n + i], z[n + i], int(r[n + i]), n)
                    assert np.allclose(s @ psi, psi, atol=1e-8)
                sp = sv.symplectic_products(x, z)
                want = np.zeros((2 * n, 2 * n), dtype=np.uint8)
                for i in range(n):
                    want[i, n + i] = want[n + i, i] = 1
                assert np.array_equal(sp, want)


def pin_measure_update(lib):
    rng = np.random.default_rng(23)
    n = 4
    done = 0
    while done < 15:
        t = orc.Tableau(n, lib=lib)
        t.run(_program(rng, n, 30, 0.0))
        q = int(rng.integers(n))
        x, z, r = t.rows_array()
        before = [sv.row_matrix(x[k], z[k], int(r[k]), n) for k in range(2 * n)]
        xq = [sv.bit(x[k], q) for k in range(2 * n)]
        stab = [k for k in range(n) if xq[n + k]]
        if not stab:
            continue
        p = stab[0]
        bits, rnd, _ = t.run(np.array([[orc.MEASURE, q, 0]], dtype=np.uint32), seed=1, shot=0, meas_base=0)
        x2, z2, r2 = t.rows_array()
        for k in range(2 * n):
            got = sv.row_matrix(x2[k], z2[k], int(r2[k]), n)
            if k == p:
                want = before[n + p]
            elif k == n + p:
                want = sv.pauli_matrix([0] * n, [int(j == q) for j in range(n)], int(bits[0]))
            elif xq[k]:
                want = before[n + p] @ before[k]
            else:
                want = before[k]
            assert np.allclose(got, want)
        done += 1


def pin_rowsum(lib):
    """rowsum(h, i) of random commuting rows equals the matrix product P_i P_h."""
    rng = np.random.default_rng(29)
    n = 3
    checked = 0
    while checked < 200:
        t = orc.Tableau(n, lib=lib)
        x, z, r = t.rows_array()
        x[:, 0] = rng.integers(0, 8, 2 * n).astype(np.uint64)
        z[:, 0] = rng.integers(0, 8, 2 * n).astype(np.uint64)
        r[:] = rng.integers(0, 2, 2 * n).astype(np.uint8)
        t.set_rows(x, z, r)
        h, i = (int(v) for v in rng.choice(2 * n, 2, replace=False))
        ph = sv.row_matrix(x[h], z[h], int(r[h]), n)
        pi = sv.row_matrix(x[i], z[i], int(r[i]), n)
        if not np.allclose(ph @ pi, pi @ ph):
            continue
        t.rowsum(h, i)
        x2, z2, r2 = t.rows_array()
        assert np.allclose(sv.row_matrix(x2[h], z2[h], int(r2[h]), n), pi @ ph)
        checked += 1


def pin_frames(lib):
    """Frame samples lie in the support of the exact outcome distribution and
    match its frequencies (compact form of test_oracle_frames)."""
    from test_oracle_frames import _program, _strings, exact_distribution
    rng = np.random.default_rng(31)
    shots = 3000
    for n in (2, 3, 4):
        for trial in range(3):
            ops = _program(rng, n, 14, 0.25)
            m = int(np.count_nonzero(ops[:, 0] == orc.MEASURE))
            dist = exact_distribution(n, ops)
            ref, _, _ = orc.Tableau(n, lib=lib).run(ops, seed=trial, shot=0)
            got = _strings(orc.frame_sample(n, ops, ref, seed=50 + trial, shots=shots, lib=lib), m)
            counts = {}
            for g in got:
                assert g in dist
                counts[g] = counts.get(g, 0) + 1
            for g, p in dist.items():
                sd = np.sqrt(shots * max(p * (1 - p), 0.0))
                assert abs(counts.get(g, 0) - shots * p) <= 5 * sd + 1


PINS = [pin_philox, pin_gates, pin_state_vector, pin_measure_update, pin_rowsum, pin_frames]


def test_unmutated_oracle_passes_compact_pins():
    lib = orc.load()
    for pin in PINS:
        pin(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        so = orc.build_oracle(path, os.path.join(d, "libmutant.so"))
        lib = orc.load(so)
        caught = []
        for pin in PINS:
            try:
                pin(lib)
            except (AssertionError, ValueError):
                caught.append(pin.__name__)
        assert caught, f"mutant '{name}' survived every pin"
