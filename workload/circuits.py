"""Random layered Clifford circuits with Z-measurements.

The paper evaluates on random circuits of n qubits and depth d drawn from a
Clifford gate set with randomly placed Z-measurements (Experiments, "Setup"
and "Benchmarks"). Those circuit files are not available, so these generators
stand in for their shapes: every layer gives each qubit one uniformly drawn
gate from {I, H, S, X, Z}, then pairs the qubits along a random permutation
and puts a CX (probability 0.5) or, when enabled, a CZ (probability 0.1) on
each pair.

Recipe (fixed draw order, numpy ``Generator(PCG64(seed))``), per layer:

1. ``integers(0, 5, n)``  -> {I, H, S, X, Z} per qubit;
2. ``permutation(n)``     -> consecutive pairs (perm[2i] controls perm[2i+1]);
3. ``random(n // 2)``     -> u < 0.5: CX; 0.5 <= u < 0.6 and CZ enabled: CZ;
   otherwise no two-qubit gate.

Mid-circuit measurement rounds (when enabled) follow layer l (1-based) with
l % 10 == 0 and l < d: ``choice(n, n // 10, replace=False)``, measured in
ascending qubit order. Every circuit ends by measuring all qubits in
ascending order.

Operations are records ``(type, q0, q1)`` of three little-endian uint32.
Identity gates are not emitted.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterator, List, Tuple

import numpy as np

# Gate type codes of an operation record.
GATE_I = 0
GATE_H = 1
GATE_S = 2
GATE_SDG = 3
GATE_X = 4
GATE_Y = 5
GATE_Z = 6
GATE_CX = 7
GATE_CZ = 8
GATE_CY = 9
GATE_SWAP = 10
GATE_ISWAP = 11
OP_MEASURE = 15

OP_DTYPE = np.dtype([("type", "<u4"), ("q0", "<u4"), ("q1", "<u4")])

# {I, H, S, X, Z} in the order the per-qubit draw indexes them.
_ONE_QUBIT_DRAW = np.array([GATE_I, GATE_H, GATE_S, GATE_X, GATE_Z], dtype=np.uint32)


@dataclass(frozen=True)
class CircuitConfig:
    name: str
    n: int
    depth: int
    seed: int
    cz: bool
    mid_measure: bool
    coin_seed: int = 0
    shots: int = 1


CONFIGS = {
    1: CircuitConfig("n64_d10", 64, 10, 0, cz=False, mid_measure=False),
    2: CircuitConfig("n4096_d100_mid", 4096, 100, 1, cz=True, mid_measure=True),
    3: CircuitConfig("n65536_d1000", 65536, 1000, 2, cz=True, mid_measure=False),
    4: CircuitConfig("n180000_d1000", 180000, 1000, 3, cz=True, mid_measure=False),
}


def random_layer(rng: np.random.Generator, n: int, cz: bool) -> np.ndarray:
    """One random layer: single-qubit sublayer, then the pair sublayer."""
    kinds = _ONE_QUBIT_DRAW[rng.integers(0, 5, n)]
    perm = rng.permutation(n).astype(np.uint32)
    u = rng.random(n // 2)
    q = np.nonzero(kinds != GATE_I)[0].astype(np.uint32)
    one = np.empty(q.size, dtype=OP_DTYPE)
    one["type"] = kinds[q]
    one["q0"] = q
    one["q1"] = 0
    first = perm[0:2 * (n // 2):2]
    second = perm[1:2 * (n // 2):2]
    ptype = np.full(n // 2, GATE_I, dtype=np.uint32)
    ptype[u < 0.5] = GATE_CX
    if cz:
        ptype[(u >= 0.5) & (u < 0.6)] = GATE_CZ
    keep = ptype != GATE_I
    two = np.empty(int(keep.sum()), dtype=OP_DTYPE)
    two["type"] = ptype[keep]
    two["q0"] = first[keep]
    two["q1"] = second[keep]
    return np.concatenate([one, two])


def _measure_ops(qubits: np.ndarray) -> np.ndarray:
    ops = np.empty(qubits.size, dtype=OP_DTYPE)
    ops["type"] = OP_MEASURE
    ops["q0"] = qubits
    ops["q1"] = 0
    return ops


def iter_circuit(cfg: CircuitConfig, depth: int | None = None,
                 final_measure: bool = True) -> Iterator[Tuple[str, np.ndarray]]:
    """Yield ('gates', ops) per layer and ('measure', qubits) per round, in program order.

    ``depth`` may truncate the circuit (the draws of the first layers are the
    same as for the full depth); mid-circuit rounds keep their positions.
    """
    d = cfg.depth if depth is None else depth
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    n = cfg.n
    for layer in range(1, d + 1):
        yield "gates", random_layer(rng, n, cfg.cz)
        if cfg.mid_measure and layer % 10 == 0 and layer < cfg.depth:
            sub = np.sort(rng.choice(n, n // 10, replace=False)).astype(np.uint32)
            yield "measure", sub
    if final_measure:
        yield "measure", np.arange(n, dtype=np.uint32)


def circuit_ops(cfg: CircuitConfig, depth: int | None = None,
                final_measure: bool = True) -> np.ndarray:
    """The whole circuit as one flat operation array (measurements as OP_MEASURE)."""
    parts = []
    for kind, arr in iter_circuit(cfg, depth, final_measure):
        parts.append(arr if kind == "gates" else _measure_ops(arr))
    if not parts:
        return np.empty(0, dtype=OP_DTYPE)
    return np.concatenate(parts)


def count_gates(ops: np.ndarray) -> int:
    t = ops["type"]
    return int(np.count_nonzero((t != GATE_I) & (t != OP_MEASURE)))


@dataclass(frozen=True)
class ServedRequest:
    index: int
    n: int
    depth: int
    shots: int
    coin_seed: int
    arrival_s: float

    def config(self) -> CircuitConfig:
        return CircuitConfig(f"served{self.index}", self.n, self.depth, 10_000 + self.index,
                             cz=True, mid_measure=False, coin_seed=self.coin_seed,
                             shots=self.shots)


def served_requests(count: int = 512, seed: int = 4, rate_hz: float = 1.0) -> List[ServedRequest]:
    """The batched/served mix: n log-uniform in [16, 16384], depth uniform in
    [10, 500], shots log-uniform in [1, 4096], Poisson arrivals at ``rate_hz``.

    Draw order: for each request in turn, n, depth, shots, inter-arrival gap.
    Circuit i's layers come from ``PCG64(10000 + i)``; its coin seed is 1000 + i.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(16), math.log(16384)))))
        d = int(rng.integers(10, 501))
        shots = int(round(math.exp(rng.uniform(0.0, math.log(4096)))))
        t += float(rng.exponential(1.0 / rate_hz))
        out.append(ServedRequest(i, n, d, shots, 1000 + i, t))
    return out
