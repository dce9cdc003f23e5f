"""The identity behind the tiled blocked pivot search, on the CPU.

Within a block of measurements, step s's stabilizer-half word is the
column of its qubit XOR the stored rows of the earlier steps s' with
M[s'][s] = 1, with the earlier pivot rows cleared; a stored row also has its
own pivot bit cleared. The tiled search does not keep those rows: it forms
each word from the block's columns through C = (I + M)^-1, built one column
per step (column s is e_s XOR the columns s' < s with M[s'][s] = 1), and it
reads the hits on S_p (which earlier stored rows have a 1 at the new pivot
p) as parities of C's columns against the columns' bits at p. Both forms are
run here on random bit columns (Python integers as bit vectors), random
upper-triangular M and pivots found as the lowest set bit, and must agree at
every step.
"""
import numpy as np
import pytest


def _lowest_bit(v):
    return (v & -v).bit_length() - 1


def _run(rng, nbits, steps, density):
    cols = []
    for _ in range(steps):
        bits = rng.random(nbits) < density
        cols.append(int("".join("1" if b else "0" for b in bits[::-1]) or "0", 2))
    # M[s'][s] for s' < s: arbitrary here (the kernels derive it from the
    # pivots' x bits); the identity holds for any strictly upper M
    M = np.triu(rng.random((steps, steps)) < 0.4, 1)
    stored, pivots, C = [], [], []
    for s in range(steps):
        cleared = 0
        for p in pivots:
            cleared |= 1 << p
        # the recurrence, with stored rows
        v = cols[s]
        for sp in range(s):
            if M[sp, s]:
                v ^= stored[sp]
        v &= ~cleared
        # the closure form
        c = 1 << s
        for sp in range(s):
            if M[sp, s]:
                c ^= C[sp]
        lin = 0
        for t in range(s + 1):
            if (c >> t) & 1:
                lin ^= cols[t]
        assert v == lin & ~cleared, f"step {s}: recurrence and closure differ"
        C.append(c)
        if v == 0:
            return s  # deterministic: the block ends here
        p = _lowest_bit(v)
        assert p not in pivots
        # hits on S_p: stored rows with a 1 at p, against C's parities
        xb = sum(1 << t for t in range(steps) if (cols[t] >> p) & 1)
        for sp in range(s):
            want = (stored[sp] >> p) & 1
            got = bin(C[sp] & xb).count("1") & 1
            assert want == got, f"step {s}: hit of step {sp} differs"
        stored.append(v & ~(1 << p))
        pivots.append(p)
    return steps


@pytest.mark.parametrize("seed", range(12))
def test_closure_form_equals_row_recurrence(seed):
    rng = np.random.default_rng(seed)
    nbits = int(rng.integers(64, 700))
    density = float(rng.choice([0.02, 0.1, 0.5]))
    k = _run(rng, nbits, 32, density)
    assert k >= 1 or density < 0.05


def test_closure_form_with_columns_zero_below_a_bound():
    """Columns whose low bits are zero (the late-sweep shape): the word of
    any step is zero below the smallest first set bit of the columns in its
    sum, and below the prefix minimum over the block's columns."""
    rng = np.random.default_rng(99)
    steps, nbits = 32, 1024
    cols = []
    for _ in range(steps):
        lo = int(rng.integers(0, nbits - 64))
        bits = (rng.random(nbits) < 0.3) & (np.arange(nbits) >= lo)
        cols.append(sum(1 << int(i) for i in np.nonzero(bits)[0]))
    M = np.triu(rng.random((steps, steps)) < 0.4, 1)
    C = []
    prefix = None
    for s in range(steps):
        c = 1 << s
        for sp in range(s):
            if M[sp, s]:
                c ^= C[sp]
        C.append(c)
        lin = 0
        for t in range(s + 1):
            if (c >> t) & 1:
                lin ^= cols[t]
        first = min(_lowest_bit(cols[t]) for t in range(s + 1) if (c >> t) & 1)
        prefix = _lowest_bit(cols[s]) if prefix is None else min(prefix, _lowest_bit(cols[s]))
        assert prefix <= first
        assert lin & ((1 << first) - 1) == 0
