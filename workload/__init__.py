"""Seeded synthetic stabilizer-circuit workloads.

This package only draws random circuits (gate types, qubit pairs, measured
qubit subsets). It holds none of the simulation arithmetic, so both the CPU
oracle and the GPU library may consume its output.
"""
from .circuits import (  # noqa: F401
    GATE_I, GATE_H, GATE_S, GATE_SDG, GATE_X, GATE_Y, GATE_Z, GATE_CX, GATE_CZ, GATE_CY, GATE_SWAP, GATE_ISWAP,
    OP_MEASURE, OP_DTYPE, CONFIGS, CircuitConfig, ServedRequest,
    random_layer, iter_circuit, circuit_ops, served_requests, count_gates, basis_circuit,
)
