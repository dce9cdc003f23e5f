"""Brute-force state-vector and Pauli-matrix helpers used to pin the oracle.

Everything here is plain linear algebra on 2^n complex vectors (n <= 10):
gates are their textbook unitary matrices, Pauli strings are Kronecker
products of the 2x2 Pauli matrices, and measurements follow the Born rule.
Qubit j is bit j of a basis index (little-endian), i.e. the last Kronecker
factor is qubit 0.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
HAD = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
SG = np.array([[1, 0], [0, 1j]], dtype=complex)
SDG = np.array([[1, 0], [0, -1j]], dtype=complex)

ONE_QUBIT = {1: HAD, 2: SG, 3: SDG, 4: PX, 5: PY, 6: PZ}
# |c t> basis with index c + 2 t for (control, target) = (a, b)
CXM = np.zeros((4, 4), dtype=complex)
for _c in (0, 1):
    for _t in (0, 1):
        CXM[_c + 2 * (_t ^ _c), _c + 2 * _t] = 1
CZM = np.diag([1, 1, 1, -1]).astype(complex)
# controlled-Y: Y on the target when the control is 1 (Y|0> = i|1>, Y|1> = -i|0>)
CYM = np.zeros((4, 4), dtype=complex)
CYM[0, 0] = CYM[2, 2] = 1
CYM[3, 1] = 1j
CYM[1, 3] = -1j
# SWAP: |a b> -> |b a>; iSWAP: |01> -> i|10>, |10> -> i|01>
SWAPM = np.zeros((4, 4), dtype=complex)
ISWAPM = np.zeros((4, 4), dtype=complex)
for _a in (0, 1):
    for _b in (0, 1):
        SWAPM[_b + 2 * _a, _a + 2 * _b] = 1
        ISWAPM[_b + 2 * _a, _a + 2 * _b] = 1 if _a == _b else 1j
TWO_QUBIT = {7: CXM, 8: CZM, 9: CYM, 10: SWAPM, 11: ISWAPM}

PAULI_BY_BITS = {(0, 0): I2, (1, 0): PX, (0, 1): PZ, (1, 1): PY}
LETTER_BY_BITS = {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}
BITS_BY_LETTER = {v: k for k, v in LETTER_BY_BITS.items()}


def bit(words: np.ndarray, j: int) -> int:
    return int((int(words[j >> 6]) >> (j & 63)) & 1)


def pauli_matrix(xbits, zbits, sign: int) -> np.ndarray:
    """(-1)^sign * P_{n-1} (x) ... (x) P_0 as a dense matrix."""
    n = len(xbits)
    m = np.array([[1.0 + 0j]])
    for j in reversed(range(n)):
        m = np.kron(m, PAULI_BY_BITS[(int(xbits[j]), int(zbits[j]))])
    return (-1) ** int(sign) * m


def row_matrix(x_row: np.ndarray, z_row: np.ndarray, r: int, n: int) -> np.ndarray:
    xb = [bit(x_row, j) for j in range(n)]
    zb = [bit(z_row, j) for j in range(n)]
    return pauli_matrix(xb, zb, r)


def matrix_to_pauli(m: np.ndarray, n: int):
    """Decompose a matrix that equals +-(Pauli string) into (xbits, zbits, sign).

    Returns None if it is not such a matrix (e.g. a +-i multiple)."""
    for code in range(4 ** n):
        xb, zb = [], []
        c = code
        for _ in range(n):
            x, z = [(0, 0), (1, 0), (0, 1), (1, 1)][c & 3]
            xb.append(x)
            zb.append(z)
            c >>= 2
        p = pauli_matrix(xb, zb, 0)
        coef = np.trace(p.conj().T @ m) / (2 ** n)
        if abs(abs(coef) - 1) < 1e-9:
            if not np.allclose(m, coef * p, atol=1e-9):
                return None
            if abs(coef - 1) < 1e-9:
                return xb, zb, 0
            if abs(coef + 1) < 1e-9:
                return xb, zb, 1
            return None
    return None


def apply_1q(psi: np.ndarray, n: int, u: np.ndarray, q: int) -> np.ndarray:
    t = psi.reshape([2] * n)
    ax = n - 1 - q
    t = np.moveaxis(np.tensordot(u, t, axes=([1], [ax])), 0, ax)
    return t.reshape(-1)


def apply_2q(psi: np.ndarray, n: int, u4: np.ndarray, a: int, b: int) -> np.ndarray:
    """u4 acts on the pair with basis index (bit a) + 2 (bit b)."""
    t = psi.reshape([2] * n)
    ax_a, ax_b = n - 1 - a, n - 1 - b
    u = u4.reshape(2, 2, 2, 2)  # [out_b, out_a, in_b, in_a]
    t = np.tensordot(u, t, axes=([2, 3], [ax_b, ax_a]))
    t = np.moveaxis(t, [0, 1], [ax_b, ax_a])
    return t.reshape(-1)


def gate_unitary(n: int, typ: int, a: int, b: int = 0) -> np.ndarray:
    """Dense 2^n x 2^n unitary of one gate (built column by column)."""
    dim = 2 ** n
    out = np.zeros((dim, dim), dtype=complex)
    for col in range(dim):
        e = np.zeros(dim, dtype=complex)
        e[col] = 1
        out[:, col] = apply_gate(e, n, typ, a, b)
    return out


def apply_gate(psi: np.ndarray, n: int, typ: int, a: int, b: int = 0) -> np.ndarray:
    if typ == 0:
        return psi
    if typ in ONE_QUBIT:
        return apply_1q(psi, n, ONE_QUBIT[typ], a)
    if typ in TWO_QUBIT:
        return apply_2q(psi, n, TWO_QUBIT[typ], a, b)
    raise ValueError(typ)


def prob_one(psi: np.ndarray, n: int, q: int) -> float:
    idx = np.arange(psi.size)
    return float(np.sum(np.abs(psi[((idx >> q) & 1) == 1]) ** 2))


def project(psi: np.ndarray, q: int, outcome: int) -> np.ndarray:
    idx = np.arange(psi.size)
    out = np.where(((idx >> q) & 1) == outcome, psi, 0)
    return out / np.linalg.norm(out)


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = 1
    return psi


def pauli_string(x_row, z_row, r, n) -> str:
    s = "-" if r else "+"
    return s + "".join(LETTER_BY_BITS[(bit(x_row, j), bit(z_row, j))] for j in range(n))


def symplectic_products(x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """GF(2) matrix of anticommutation <P_a, P_b> = x_a.z_b + z_a.x_b for packed rows."""
    # unpack to bits
    xb = np.unpackbits(x.view(np.uint8), axis=1, bitorder="little").astype(np.uint8)
    zb = np.unpackbits(z.view(np.uint8), axis=1, bitorder="little").astype(np.uint8)
    m = (xb.astype(np.int64) @ zb.T.astype(np.int64) + zb.astype(np.int64) @ xb.T.astype(np.int64)) & 1
    return m.astype(np.uint8)
