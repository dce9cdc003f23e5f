"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value comes from
numpy's Philox generator, from 2x2 / 4x4 Pauli and gate matrices, from a
brute-force state vector (Born rule), from the paper's printed examples
(tests/golden), or from the algebraic invariants of a destabilizer tableau.
"""
import itertools
import json
import os

import numpy as np
import pytest

import statevec as sv
from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")
NAME_TO_TYPE = {"H": orc.H, "S": orc.S, "SDG": orc.SDG, "X": orc.X, "Y": orc.Y, "Z": orc.Z,
                "CX": orc.CX, "CZ": orc.CZ, "CY": orc.CY, "SWAP": orc.SWAP, "ISWAP": orc.ISWAP}


def ops_of(*gates):
    out = []
    for g in gates:
        t = NAME_TO_TYPE[g[0]] if isinstance(g[0], str) else g[0]
        out.append([t, g[1], g[2] if len(g) > 2 else 0])
    return np.array(out, dtype=np.uint32).reshape(-1, 3)


def meas(q):
    return [orc.MEASURE, q, 0]


# ---------------------------------------------------------------- Philox
@pytest.mark.parametrize("key,ctr", [
    ((0, 0), 1), ((1, 2), 1), ((1, 2), 7), ((2**64 - 1, 12345), 2**40 + 3),
    ((0xDEADBEEF, 0), 99), ((3, 1 << 63), 5)])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox (Philox4x64-10) increments its 256-bit counter before
    # drawing, so a generator started at c-1 yields block c first.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=ctr - 1)
    want = bg.random_raw(4).astype(np.uint64)
    got = orc.philox4x64_10([ctr & (2**64 - 1), ctr >> 64, 0, 0], key)
    assert np.array_equal(got, want)


def test_philox_full_counter_words_match_numpy():
    rng = np.random.default_rng(5)
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        c_int = sum(v << (64 * i) for i, v in enumerate(ctr))
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=c_int - 1)
        assert np.array_equal(orc.philox4x64_10(ctr, key), bg.random_raw(4).astype(np.uint64))


def test_coin_is_bit0_of_word0():
    for seed, shot, m in [(0, 0, 0), (7, 3, 11), (1000, 4095, 180000)]:
        bg = np.random.Philox(key=np.array([seed, shot], dtype=np.uint64), counter=m - 1 if m else 2**256 - 1)
        assert orc.coin(seed, shot, m) == int(bg.random_raw(1)[0]) & 1


def test_coins_are_balanced():
    c = [orc.coin(123, 0, m) for m in range(4000)]
    assert 1800 < sum(c) < 2200


# ---------------------------------------------------------------- g table
def test_g_function_against_pauli_matrices():
    lib = orc.load()
    for (x1, z1), (x2, z2) in itertools.product([(0, 0), (1, 0), (0, 1), (1, 1)], repeat=2):
        p1, p2 = sv.PAULI_BY_BITS[(x1, z1)], sv.PAULI_BY_BITS[(x2, z2)]
        p3 = sv.PAULI_BY_BITS[(x1 ^ x2, z1 ^ z2)]
        prod = p1 @ p2
        g = lib.sqo_g(x1, z1, x2, z2)
        assert np.allclose(prod, (1j ** g) * p3), (x1, z1, x2, z2, g)


def test_gsum_word_equals_per_bit_sum():
    lib = orc.load()
    rng = np.random.default_rng(1)
    for _ in range(300):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, np.iinfo(np.uint64).max, 4, dtype=np.uint64, endpoint=True))
        want = sum(lib.sqo_g((x1 >> b) & 1, (z1 >> b) & 1, (x2 >> b) & 1, (z2 >> b) & 1)
                   for b in range(64)) % 4
        assert lib.sqo_gsum_word(x1, z1, x2, z2) == want


# ---------------------------------------------------------------- gate rules
def _set_single_row(t, n, xbits, zbits, sign):
    x, z, r = t.rows_array()
    x[:] = 0
    z[:] = 0
    r[:] = 0
    for j in range(n):
        x[0, j >> 6] |= np.uint64(xbits[j] << (j & 63))
        z[0, j >> 6] |= np.uint64(zbits[j] << (j & 63))
    r[0] = sign
    t.set_rows(x, z, r)


@pytest.mark.parametrize("gate", ["H", "S", "SDG", "X", "Y", "Z", "CX", "CZ", "CY", "SWAP", "ISWAP"])
def test_gate_rules_against_conjugation(gate):
    """Every Pauli P (with sign) on 2 qubits must map to U P U^dagger."""
    n = 2
    typ = NAME_TO_TYPE[gate]
    placements = [(0, 1), (1, 0)] if typ in orc.TWO_QUBIT else [(0, 0), (1, 0)]
    for a, b in placements:
        u = sv.gate_unitary(n, typ, a, b)
        for code in range(16):
            xb = [(code >> 0) & 1, (code >> 1) & 1]
            zb = [(code >> 2) & 1, (code >> 3) & 1]
            for sign in (0, 1):
                t = orc.Tableau(n)
                _set_single_row(t, n, xb, zb, sign)
                t.run(ops_of((typ, a, b)))
                x, z, r = t.rows_array()
                got = sv.row_matrix(x[0], z[0], int(r[0]), n)
                want = u @ sv.pauli_matrix(xb, zb, sign) @ u.conj().T
                assert np.allclose(got, want), (gate, a, b, xb, zb, sign)


# ---------------------------------------------------------------- paper examples
def _row_bits(x_row, z_row, r, n):
    return [sv.bit(x_row, j) for j in range(n)] + [sv.bit(z_row, j) for j in range(n)] + [int(r)]


def test_paper_encoding_example():
    g = json.load(open(GOLDEN))["encoding_example"]
    n = g["n"]
    for row, want in zip(g["rows"], g["generators"]):
        xw = np.array([sum(row[j] << j for j in range(n))], dtype=np.uint64)
        zw = np.array([sum(row[n + j] << j for j in range(n))], dtype=np.uint64)
        assert sv.pauli_string(xw, zw, row[2 * n], n) == want


def test_paper_example_independent_gates():
    g = json.load(open(GOLDEN))["example_independent_gates"]
    n = g["n"]
    t = orc.Tableau(n)
    x, z, r = t.rows_array()
    assert [_row_bits(x[n + i], z[n + i], r[n + i], n) for i in range(n)] == g["initial_stabilizers"]
    for (name, q), want in zip(g["gates"], g["stabilizers_after_each_gate"]):
        t.run(ops_of((name, q)))
        x, z, r = t.rows_array()
        assert [_row_bits(x[n + i], z[n + i], r[n + i], n) for i in range(n)] == want


def test_paper_product_state_plus01():
    g = json.load(open(GOLDEN))["product_state_plus01"]
    n = g["n"]
    t = orc.Tableau(n)
    t.run(ops_of(*[(name, q) for name, q in g["reach_with_gates"]]))
    x, z, r = t.rows_array()
    stab = [_row_bits(x[n + i], z[n + i], r[n + i], n) for i in range(n)]
    assert stab == g["stabilizers"]
    dest = [_row_bits(x[i], z[i], r[i], n) for i in range(n)]
    for got, want in zip(dest, g["destabilizers"]):
        assert got[:2 * n] == want[:2 * n]
    # signs: first two as printed; the third is + under the gate derivation
    assert [d[-1] for d in dest] == [0, 0, 0]


# ---------------------------------------------------------------- brute force
def _random_program(rng, n, length, p_meas=0.15, gates=(1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11)):
    ops = []
    for _ in range(length):
        if rng.random() < p_meas:
            ops.append([orc.MEASURE, int(rng.integers(n)), 0])
            continue
        t = int(rng.choice(gates))
        if t in orc.TWO_QUBIT:
            if n < 2:
                continue
            a, b = rng.choice(n, 2, replace=False)
            ops.append([t, int(a), int(b)])
        else:
            ops.append([t, int(rng.integers(n)), 0])
    return np.array(ops, dtype=np.uint32).reshape(-1, 3)


def _check_stabilizers(psi, t, n):
    x, z, r = t.rows_array()
    for i in range(n):
        s = sv.row_matrix(x[n + i], z[n + i], int(r[n + i]), n)
        assert np.allclose(s @ psi, psi, atol=1e-8), f"S_{i} does not stabilize the state"


def _check_symplectic(t, n):
    x, z, _ = t.rows_array()
    m = sv.symplectic_products(x, z)
    want = np.zeros((2 * n, 2 * n), dtype=np.uint8)
    for i in range(n):
        want[i, n + i] = want[n + i, i] = 1
    assert np.array_equal(m[:2 * n, :2 * n], want)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_random_circuits_against_state_vector(n):
    """Outcomes follow the Born rule (p in {0, 1/2, 1}); deterministic values
    and the random/deterministic split match; every stabilizer row stabilizes
    the state after every step; the tableau keeps its symplectic structure."""
    rng = np.random.default_rng(100 + n)
    for trial in range(12 if n < 8 else 4):
        prog = _random_program(rng, n, 40)
        seed = int(rng.integers(1 << 30))
        t = orc.Tableau(n)
        psi = sv.zero_state(n)
        m = 0
        for op in prog:
            if op[0] != orc.MEASURE:
                t.run(op.reshape(1, 3))
                psi = sv.apply_gate(psi, n, int(op[0]), int(op[1]), int(op[2]))
            else:
                q = int(op[1])
                bits, rnd, _ = t.run(op.reshape(1, 3), seed=seed, shot=trial, meas_base=m)
                p1 = sv.prob_one(psi, n, q)
                if abs(p1 - 0.5) < 1e-9:
                    assert rnd[0] == 1
                    assert bits[0] == orc.coin(seed, trial, m)
                else:
                    assert rnd[0] == 0
                    assert abs(p1 - bits[0]) < 1e-9
                psi = sv.project(psi, q, int(bits[0]))
                m += 1
            _check_stabilizers(psi, t, n)
            _check_symplectic(t, n)
        assert t.odd_count == 0 and t.badscratch_count == 0


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_destabilizers_are_conjugated_x(n):
    """Gate-only circuits: D_i = U X_i U^dagger and S_i = U Z_i U^dagger exactly (signs included)."""
    rng = np.random.default_rng(7 + n)
    for _ in range(6):
        prog = _random_program(rng, n, 25, p_meas=0.0)
        t = orc.Tableau(n)
        t.run(prog)
        u = np.eye(2 ** n, dtype=complex)
        for op in prog:
            u = sv.gate_unitary(n, int(op[0]), int(op[1]), int(op[2])) @ u
        x, z, r = t.rows_array()
        for i in range(n):
            e = [int(j == i) for j in range(n)]
            zero = [0] * n
            assert np.allclose(sv.row_matrix(x[i], z[i], int(r[i]), n),
                               u @ sv.pauli_matrix(e, zero, 0) @ u.conj().T)
            assert np.allclose(sv.row_matrix(x[n + i], z[n + i], int(r[n + i]), n),
                               u @ sv.pauli_matrix(zero, e, 0) @ u.conj().T)


def test_rowsum_is_the_matrix_product():
    """rowsum(h, i) must leave row h equal to the matrix product P_i P_h."""
    rng = np.random.default_rng(3)
    n = 4
    checked = 0
    while checked < 300:
        t = orc.Tableau(n)
        x, z, r = t.rows_array()
        x[:, 0] = rng.integers(0, 16, 2 * n).astype(np.uint64)
        z[:, 0] = rng.integers(0, 16, 2 * n).astype(np.uint64)
        r[:] = rng.integers(0, 2, 2 * n).astype(np.uint8)
        t.set_rows(x, z, r)
        h, i = (int(v) for v in rng.choice(2 * n, 2, replace=False))
        ph = sv.row_matrix(x[h], z[h], int(r[h]), n)
        pi = sv.row_matrix(x[i], z[i], int(r[i]), n)
        if not np.allclose(ph @ pi, pi @ ph):
            continue  # CHP only multiplies commuting rows
        assert t.rowsum(h, i) == 0
        x2, z2, r2 = t.rows_array()
        assert np.allclose(sv.row_matrix(x2[h], z2[h], int(r2[h]), n), pi @ ph)
        checked += 1


def test_rowsum_flags_anticommuting_product():
    t = orc.Tableau(1)
    # D_0 = X, S_0 = Z: X*Z is anti-Hermitian, exponent odd
    assert t.rowsum(0, 1) == 1
    assert t.odd_count == 1


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_measurement_update_against_definition(n):
    """Random case: each row h with x_hq = 1 (other than D_p, S_p) becomes the
    matrix product S_p * row_h; D_p becomes the old S_p; S_p becomes
    (-1)^coin Z_q; other rows are unchanged. Checked with matrices."""
    rng = np.random.default_rng(40 + n)
    done = 0
    while done < 25:
        t = orc.Tableau(n)
        t.run(_random_program(rng, n, 30, p_meas=0.1), seed=5)
        q = int(rng.integers(n))
        x, z, r = t.rows_array()
        before = [sv.row_matrix(x[k], z[k], int(r[k]), n) for k in range(2 * n)]
        xq = [sv.bit(x[k], q) for k in range(2 * n)]
        stab_x = [k for k in range(n) if xq[n + k]]
        if not stab_x:
            continue
        p = stab_x[0]
        bits, rnd, _ = t.run(np.array([[orc.MEASURE, q, 0]], dtype=np.uint32), seed=9, shot=1, meas_base=77)
        assert rnd[0] == 1 and bits[0] == orc.coin(9, 1, 77)
        x2, z2, r2 = t.rows_array()
        after = [sv.row_matrix(x2[k], z2[k], int(r2[k]), n) for k in range(2 * n)]
        for k in range(2 * n):
            if k == p:
                want = before[n + p]
            elif k == n + p:
                e = [int(j == q) for j in range(n)]
                want = sv.pauli_matrix([0] * n, e, int(bits[0]))
            elif xq[k]:
                want = before[n + p] @ before[k]
            else:
                want = before[k]
            assert np.allclose(after[k], want), (k, p, q)
        done += 1


# ---------------------------------------------------------------- textbook states
def test_bell_and_ghz_outcomes_agree():
    for seed in range(20):
        t = orc.Tableau(2)
        bits, rnd, _ = t.run(np.array([[orc.H, 0, 0], [orc.CX, 0, 1], meas(0), meas(1)], dtype=np.uint32), seed=seed)
        assert list(rnd) == [1, 0] and bits[0] == bits[1]
        t = orc.Tableau(5)
        prog = [[orc.H, 0, 0]] + [[orc.CX, 0, k] for k in range(1, 5)] + [meas(k) for k in range(5)]
        bits, rnd, _ = t.run(np.array(prog, dtype=np.uint32), seed=seed)
        assert list(rnd) == [1, 0, 0, 0, 0] and len(set(bits.tolist())) == 1


def test_basis_state_outcomes():
    for g, want in [(orc.X, 1), (orc.Y, 1), (orc.Z, 0), (orc.S, 0), (orc.H, None)]:
        t = orc.Tableau(1)
        bits, rnd, _ = t.run(np.array([[g, 0, 0], meas(0)], dtype=np.uint32), seed=3)
        if want is None:
            assert rnd[0] == 1
        else:
            assert rnd[0] == 0 and bits[0] == want


def _tableau_after(n, prog):
    t = orc.Tableau(n)
    t.run(np.array(prog, dtype=np.uint32).reshape(-1, 3))
    return t.rows_array()


def test_gate_identities_on_tableaux():
    rng = np.random.default_rng(11)
    n = 4
    for _ in range(10):
        prefix = _random_program(rng, n, 20, p_meas=0.0).tolist()
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        same = [
            ([[orc.S, a, 0], [orc.S, a, 0]], [[orc.Z, a, 0]]),
            ([[orc.SDG, a, 0]], [[orc.S, a, 0], [orc.S, a, 0], [orc.S, a, 0]]),
            ([[orc.H, a, 0], [orc.S, a, 0]] * 3, []),
            ([[orc.CZ, a, b]], [[orc.H, b, 0], [orc.CX, a, b], [orc.H, b, 0]]),
            ([[orc.CZ, a, b]], [[orc.CZ, b, a]]),
            ([[orc.Y, a, 0]], [[orc.Z, a, 0], [orc.X, a, 0]]),
            # SWAP as three CX; SWAP and iSWAP are symmetric; iSWAP^2 = Z_a Z_b;
            # CY = S_b CX S_b^dagger
            ([[orc.SWAP, a, b]], [[orc.CX, a, b], [orc.CX, b, a], [orc.CX, a, b]]),
            ([[orc.SWAP, a, b]], [[orc.SWAP, b, a]]),
            ([[orc.ISWAP, a, b]], [[orc.ISWAP, b, a]]),
            ([[orc.ISWAP, a, b]] * 2, [[orc.Z, a, 0], [orc.Z, b, 0]]),
            ([[orc.CY, a, b]], [[orc.SDG, b, 0], [orc.CX, a, b], [orc.S, b, 0]]),
        ]
        for lhs, rhs in same:
            ta = _tableau_after(n, prefix + lhs)
            tb = _tableau_after(n, prefix + rhs)
            for u, v in zip(ta, tb):
                assert np.array_equal(u, v)


# ---------------------------------------------------------------- larger n
def test_invariants_and_measure_twice_at_moderate_n():
    """n = 300: symplectic structure after a random circuit with measurements;
    re-measuring a measured qubit is deterministic with the same value."""
    from workload import CircuitConfig, circuit_ops
    cfg = CircuitConfig("t300", 300, 12, 99, cz=True, mid_measure=True)
    ops = circuit_ops(cfg, final_measure=False)
    t = orc.Tableau(300)
    t.run(ops, seed=4)
    qs = [0, 17, 150, 299, 17]
    bits, rnd, _ = t.run(np.array([meas(q) for q in qs] + [meas(q) for q in qs], dtype=np.uint32), seed=4,
                         meas_base=1000)
    assert np.array_equal(bits[:5], bits[5:])
    assert not rnd[5:].any() and rnd[4] == 0
    _check_symplectic(t, 300)
    assert t.odd_count == 0 and t.badscratch_count == 0


def test_row_subset_matches_full_tableau():
    """A handle holding a row subset (with the stabilizer prefix) follows the
    full tableau exactly while the pivots lie in the prefix."""
    from workload import CircuitConfig, circuit_ops
    n = 200
    cfg = CircuitConfig("t200", n, 15, 5, cz=True, mid_measure=False)
    ops = circuit_ops(cfg)
    full = orc.Tableau(n)
    fb, fr, _ = full.run(ops, seed=8, shot=2)
    rows = list(range(n, n + 64)) + [3, 77, 199, 300, 399]
    sub = orc.Tableau(n, rows=rows)
    sb, sr, done = sub.run(ops, seed=8, shot=2)
    assert sb.size >= 5
    assert np.array_equal(sb, fb[:sb.size]) and np.array_equal(sr, fr[:sr.size])
    # replay the full tableau to the same point and compare the held rows
    full2 = orc.Tableau(n)
    full2.run(ops[:done], seed=8, shot=2)
    x, z, r = full2.rows_array()
    xs, zs, rs = sub.rows_array()
    idx = np.array(rows)
    assert np.array_equal(xs, x[idx]) and np.array_equal(zs, z[idx]) and np.array_equal(rs, r[idx])
