"""Pins of the operator-tableau oracle of the paper's CX-injection collapse
(Algorithm alg:stim; oracle/stim_oracle.c), against what the mathematics
fixes rather than against its own arithmetic:

  * its four bit matrices are those of the state tableau (XS[k][q] =
    x_q(S_k) and so on), so after gates alone they equal the CHP oracle's
    rows bit for bit (the CHP oracle being pinned by matrix conjugation);
  * measurement outcomes equal the CHP oracle's under the same coins:
    random outcomes are the coin, deterministic ones are fixed by the state;
  * the post-measurement state is the same: every stabilizer S of the CHP
    oracle's state maps under the operator tableau T = C^dagger to a +Z
    string (T(S) has no x bit and sign +), i.e. S C|0> = C|0>;
  * brute-force state vectors (n <= 5): the outcomes follow the Born rule;
  * textbook cases (GHZ, |+>, X|0>).
Planted mistakes in the collapse each fail one of these.
"""
import os
import tempfile

import numpy as np
import pytest

import statevec as sv
from gpu_util import mixed_program
from oracle import oracle as orc

STIM_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "stim_oracle.c")


def _gates_only(rng, n, layers, extra=False):
    return mixed_program(rng, n, layers, p_meas=0.0, extra=extra)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 65, 130])
def test_gate_bits_equal_the_state_tableau(n):
    rng = np.random.default_rng(n)
    ops = _gates_only(rng, n, 6, extra=n > 1)
    chp = orc.Tableau(n)
    chp.run(ops)
    x, z, _ = chp.rows_array()
    ot = orc.OTableau(n)
    ot.run(ops)
    xs, xd, zs, zd, _, _ = ot.arrays()
    assert np.array_equal(xs, x[n:]) and np.array_equal(xd, x[:n])
    assert np.array_equal(zs, z[n:]) and np.array_equal(zd, z[:n])
    assert ot.odd_count == 0


def _stabilizers_fixed(ot, chp, n):
    """Every CHP stabilizer maps to a +Z string under the operator tableau."""
    x, z, r = chp.rows_array()
    for k in range(n):
        ox, oz, sign, bad = ot.image(x[n + k], z[n + k], int(r[n + k]))
        if bad or ox.any() or sign != 0:
            return False
    return True


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 65, 100])
def test_outcomes_and_state_equal_chp(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(4):
        ops = mixed_program(rng, n, 8, p_meas=0.3, extra=n > 1)
        seed = int(rng.integers(1 << 40))
        chp = orc.Tableau(n)
        cb, cr, _ = chp.run(ops, seed=seed, shot=5, meas_base=3)
        ot = orc.OTableau(n)
        ob, orr = ot.run(ops, seed=seed, shot=5, meas_base=3)
        assert np.array_equal(ob, cb), f"n={n} trial {trial}: outcomes differ from CHP"
        assert np.array_equal(orr, cr), f"n={n} trial {trial}: random flags differ from CHP"
        assert ot.odd_count == 0
        assert _stabilizers_fixed(ot, chp, n), f"n={n} trial {trial}: states differ"


def test_born_rule_small():
    rng = np.random.default_rng(9)
    for n in (2, 3, 4, 5):
        for trial in range(6):
            ops = mixed_program(rng, n, 5, p_meas=0.0, extra=True)
            meas = np.array([[orc.MEASURE, q, 0] for q in rng.permutation(n)], dtype=np.uint32)
            psi = sv.zero_state(n)
            for op in ops:
                psi = sv.apply_gate(psi, n, int(op[0]), int(op[1]), int(op[2]))
            ot = orc.OTableau(n)
            bits, rnd = ot.run(np.concatenate([ops, meas]), seed=trial)
            for (q, b, rr) in zip(meas[:, 1], bits, rnd):
                p1 = sv.prob_one(psi, n, int(q))
                if abs(p1 - 0.5) < 1e-9:
                    assert rr == 1
                else:
                    assert rr == 0 and abs(p1 - b) < 1e-9
                psi = sv.project(psi, int(q), int(b))


def test_textbook_cases():
    n = 6
    ghz = np.array([[orc.H, 0, 0]] + [[orc.CX, 0, q] for q in range(1, n)]
                   + [[orc.MEASURE, q, 0] for q in range(n)], dtype=np.uint32)
    for seed in range(8):
        b, r = orc.OTableau(n).run(ghz, seed=seed)
        assert np.all(b == b[0]) and r[0] == 1 and not r[1:].any()
        assert b[0] == orc.coin(seed, 0, 0)
    plus = np.array([[orc.H, 0, 0], [orc.MEASURE, 0, 0], [orc.MEASURE, 0, 0]], dtype=np.uint32)
    b, r = orc.OTableau(1).run(plus, seed=3)
    assert list(r) == [1, 0] and b[0] == b[1] == orc.coin(3, 0, 0)
    flip = np.array([[orc.X, 0, 0], [orc.Y, 1, 0], [orc.MEASURE, 0, 0], [orc.MEASURE, 1, 0]], dtype=np.uint32)
    b, r = orc.OTableau(2).run(flip)
    assert list(b) == [1, 1] and not r.any()


MUTANTS = {
    "CX injection sign term": ("s[w] ^= xc[w] & zt[w] & ~(zc[w] ^ xt[w]);", "s[w] ^= xc[w] & zt[w] & (zc[w] ^ xt[w]);"),
    "CX injection misses z_c": ("    zc[w] ^= zt[w];\n  }\n}\n\nstatic void inject_invp", "  }\n}\n\nstatic void inject_invp"),
    "swap branch inverted": ("    if (bit(xdp, q)) {\n      inject_invp", "    if (!bit(xdp, q)) {\n      inject_invp"),
    "no X injection": ("    if (bit(t->ss, q) != coin) {", "    if (0) {"),
    "X injection on the x rows": ("      inject_x(t->ss, xdp, W);", "      inject_x(t->ss, xsp, W);"),
    "targets include the pivot row": ("for (uint32_t k = (uint32_t)p + 1; k < n; ++k) {",
                                      "for (uint32_t k = (uint32_t)p; k < n; ++k) {"),
    "S phase sign": ("case OT_S: str_mul(t, str_of(t, a, 0), str_of(t, a, 1), 3); break;",
                     "case OT_S: str_mul(t, str_of(t, a, 0), str_of(t, a, 1), 1); break;"),
    "CZ uses A_b": ("str_mul(t, str_of(t, a, 0), str_of(t, b, 1), 0);  /* A_a <- A_a B_b */",
                    "str_mul(t, str_of(t, a, 0), str_of(t, b, 0), 0);  /* A_a <- A_a B_b */"),
}
# Not listed: flipping InjectInvP's sign term (x & ~z -> x & z). That turns the
# H_YZ rotation into H_YZ followed by a Y at the pivot position, which flips
# SignsS[q] and so the X-injection decision after it; the two together are a
# Z at that position, which fixes |0>, so state and outcomes are unchanged (a
# different sign gauge of the same state, which nothing physical can tell).


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    text = open(STIM_SRC).read()
    assert text.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "stim_mutant.c")
        with open(src, "w") as f:
            f.write(text.replace(old, new))
        lib = orc.load(orc.build_oracle(out=os.path.join(d, "lib.so"), stim_src=src))
        caught = False
        rng = np.random.default_rng(4)
        for n in (2, 3, 5, 17):
            for trial in range(4):
                ops = mixed_program(rng, n, 8, p_meas=0.3, extra=True)
                chp = orc.Tableau(n, lib=lib)
                cb, cr, _ = chp.run(ops, seed=trial)
                ot = orc.OTableau(n, lib=lib)
                ob, orr = ot.run(ops, seed=trial)
                if (not np.array_equal(ob, cb) or not np.array_equal(orr, cr) or ot.odd_count
                        or not _stabilizers_fixed(ot, chp, n)):
                    caught = True
                    break
            if caught:
                break
        assert caught, f"planted mistake '{name}' survived every pin"
