"""Helpers shared by the GPU parity tests: seeded circuit drawing and the two
ways of driving each side. Nothing here computes any tableau arithmetic."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc

ONE_Q = np.array([orc.I, orc.H, orc.S, orc.SDG, orc.X, orc.Y, orc.Z], dtype=np.uint32)


def mixed_program(rng, n, layers, p_meas=0.2, cz=True, extra=False):
    """Layers of random one-qubit gates (all types), random disjoint CX/CZ
    pairs (with extra=True also CY, SWAP and iSWAP), then a random (unsorted)
    set of measured qubits."""
    ops = []
    for _ in range(layers):
        kinds = ONE_Q[rng.integers(0, ONE_Q.size, n)]
        for q in np.nonzero(kinds != orc.I)[0]:
            ops.append([int(kinds[q]), int(q), 0])
        perm = rng.permutation(n)
        for k in range(n // 2):
            u = rng.random()
            a, b = int(perm[2 * k]), int(perm[2 * k + 1])
            if extra:
                if u < 0.8:
                    ops.append([[orc.CX, orc.CZ, orc.CY, orc.SWAP, orc.ISWAP][int(u / 0.16)], a, b])
            elif u < 0.45:
                ops.append([orc.CX, a, b])
            elif cz and u < 0.65:
                ops.append([orc.CZ, a, b])
        if p_meas > 0:
            k = int(rng.binomial(n, p_meas))
            for q in rng.choice(n, k, replace=False):
                ops.append([orc.MEASURE, int(q), 0])
    return np.array(ops, dtype=np.uint32).reshape(-1, 3)


def segments(ops):
    """Split a program into ('gates', ops) and ('measure', qubits) runs."""
    a = np.asarray(ops)
    if a.dtype.names:
        a = np.stack([a["type"], a["q0"], a["q1"]], axis=1).astype(np.uint32)
    out = []
    i = 0
    while i < a.shape[0]:
        meas = a[i, 0] == orc.MEASURE
        j = i
        while j < a.shape[0] and (a[j, 0] == orc.MEASURE) == meas:
            j += 1
        out.append(("measure", a[i:j, 1].copy()) if meas else ("gates", a[i:j].copy()))
        i = j
    return out


def oracle_run(n, ops, seed, shot=0, meas_base=0):
    t = orc.Tableau(n)
    bits, rnd, _ = t.run(ops, seed=seed, shot=shot, meas_base=meas_base)
    x, z, r = t.rows_array()
    assert t.odd_count == 0 and t.badscratch_count == 0
    return bits, rnd, x, z, r, t


def gpu_run_calls(t, ops, seed, shot=0, meas_base=0):
    """Drive a GPU tableau through sq_apply_gates / sq_measure calls."""
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


def otableau_state(ot):
    """The operator-tableau oracle's arrays in the library's export order:
    rows i < n the destabilizer half (XD, ZD), rows n + i the stabilizer half
    (XS, ZS); sign byte i < n the image of X_i, n + i the image of Z_i."""
    xs, xd, zs, zd, ss, sd = ot.arrays()
    n = ot.n

    def signs(vec):
        return np.unpackbits(np.ascontiguousarray(vec, dtype="<u8").view(np.uint8), bitorder="little")[:n]

    return (np.concatenate([xd, xs]), np.concatenate([zd, zs]),
            np.concatenate([signs(sd), signs(ss)]).astype(np.uint8))
