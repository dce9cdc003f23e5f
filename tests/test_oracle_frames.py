"""Pins of the Pauli-frame oracle (many-shot sampling).

The frame sampler draws other bits than per-shot CHP, so it is pinned by what
the mathematics fixes: every sampled outcome string must be possible (its
Born probability is nonzero) and the sample frequencies must match the exact
joint distribution, computed by brute-force state vectors that branch over
every measurement outcome (n <= 5, with measurements in the middle of the
circuit). Its random draws are pinned to numpy's Philox4x64-10.
"""
import itertools

import numpy as np
import pytest

import statevec as sv
from oracle import oracle as orc


def test_frame_bits_are_numpy_philox():
    for seed, s, e in [(0, 0, 0), (7, 5, 3), (123, 64, 9), (2**40 + 3, 200, 1000), (9, 63, 0), (9, 127, 17)]:
        key = np.array([seed, (1 << 63) + (s >> 6)], dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=e - 1 if e else 2**256 - 1)
        word = int(bg.random_raw(1)[0])
        assert orc.frame_bit(seed, s, e) == (word >> (s & 63)) & 1


def _program(rng, n, length, p_meas):
    ops = []
    for _ in range(length):
        if rng.random() < p_meas:
            ops.append([orc.MEASURE, int(rng.integers(n)), 0])
            continue
        t = int(rng.integers(1, 12 if n > 1 else 7))
        if t in orc.TWO_QUBIT:
            a, b = rng.choice(n, 2, replace=False)
            ops.append([t, int(a), int(b)])
        else:
            ops.append([t, int(rng.integers(n)), 0])
    ops.append([orc.MEASURE, int(rng.integers(n)), 0])
    return np.array(ops, dtype=np.uint32)


def exact_distribution(n, ops):
    """Joint distribution of all outcomes: branch the state vector at every
    measurement with its Born probabilities."""
    dist = {}

    def walk(psi, k, prefix, p):
        if p < 1e-12:
            return
        while k < len(ops) and ops[k][0] != orc.MEASURE:
            psi = sv.apply_gate(psi, n, int(ops[k][0]), int(ops[k][1]), int(ops[k][2]))
            k += 1
        if k == len(ops):
            dist[prefix] = dist.get(prefix, 0.0) + p
            return
        q = int(ops[k][1])
        p1 = sv.prob_one(psi, n, q)
        for bit, pb in ((0, 1 - p1), (1, p1)):
            if pb > 1e-12:
                walk(sv.project(psi, q, bit), k + 1, prefix + (bit,), p * pb)

    walk(sv.zero_state(n), 0, (), 1.0)
    return dist


def _strings(words, m):
    return [tuple(int((int(w[i >> 6]) >> (i & 63)) & 1) for i in range(m)) for w in words]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_frame_samples_follow_the_born_distribution(n):
    rng = np.random.default_rng(500 + n)
    shots = 6000
    for trial in range(6):
        ops = _program(rng, n, 14, 0.25)
        m = int(np.count_nonzero(ops[:, 0] == orc.MEASURE))
        dist = exact_distribution(n, ops)
        ref, _, _ = orc.Tableau(n).run(ops, seed=trial, shot=0)
        assert tuple(int(b) for b in ref) in dist, "the CHP reference must be a possible outcome"
        words = orc.frame_sample(n, ops, ref, seed=1000 + trial, shots=shots)
        got = _strings(words, m)
        counts = {}
        for g in got:
            assert g in dist, f"impossible outcome {g} (n={n}, trial {trial})"
            counts[g] = counts.get(g, 0) + 1
        # every outcome has probability 2^-k; its count is binomial: within 5 sigma
        for g, p in dist.items():
            c = counts.get(g, 0)
            sd = np.sqrt(shots * max(p * (1 - p), 0.0))
            assert abs(c - shots * p) <= 5 * sd + 1, (g, c, shots * p)


def test_ghz_frames_agree_within_each_shot():
    n = 6
    ops = np.array([[orc.H, 0, 0]] + [[orc.CX, 0, q] for q in range(1, n)] + [[orc.MEASURE, q, 0] for q in range(n)],
                   dtype=np.uint32)
    ref, _, _ = orc.Tableau(n).run(ops, seed=3)
    words = orc.frame_sample(n, ops, ref, seed=11, shots=2000)
    strings = _strings(words, n)
    assert all(len(set(s)) == 1 for s in strings)
    ones = sum(s[0] for s in strings)
    assert 900 < ones < 1100


def test_deterministic_and_repeated_measurements_equal_reference():
    """X|0> measures 1 in every shot; a qubit measured twice in a row repeats
    its first outcome in every shot."""
    n = 3
    ops = np.array([[orc.X, 0, 0], [orc.H, 1, 0], [orc.MEASURE, 0, 0], [orc.MEASURE, 1, 0], [orc.MEASURE, 1, 0],
                    [orc.S, 2, 0], [orc.MEASURE, 2, 0]], dtype=np.uint32)
    ref, _, _ = orc.Tableau(n).run(ops, seed=5)
    strings = _strings(orc.frame_sample(n, ops, ref, seed=2, shots=500), 4)
    for s in strings:
        assert s[0] == 1 and s[1] == s[2] and s[3] == 0
    assert 180 < sum(s[1] for s in strings) < 320


def test_shot_words_are_independent_of_the_shot_count():
    """Shot s draws the same bits whatever the number of shots requested."""
    rng = np.random.default_rng(8)
    n = 4
    ops = _program(rng, n, 20, 0.2)
    ref, _, _ = orc.Tableau(n).run(ops, seed=1)
    a = orc.frame_sample(n, ops, ref, seed=9, shots=70)
    b = orc.frame_sample(n, ops, ref, seed=9, shots=200)
    assert np.array_equal(a, b[:70])
