"""The seeded circuit generators: fixed draw order, shapes and counts."""
import numpy as np

from workload import (CONFIGS, GATE_CX, GATE_CZ, GATE_I, GATE_Y, GATE_SDG, OP_MEASURE,
                      circuit_ops, count_gates, iter_circuit, served_requests)


def test_deterministic_and_seed_dependent():
    a = circuit_ops(CONFIGS[1])
    b = circuit_ops(CONFIGS[1])
    assert np.array_equal(a, b)
    c = circuit_ops(CONFIGS[2], depth=3, final_measure=False)
    assert not np.array_equal(a[:20], c[:20])


def test_config1_shape():
    ops = circuit_ops(CONFIGS[1])
    t = ops["type"]
    assert not np.any(t == GATE_CZ) and not np.any(t == GATE_I)
    assert not np.any(t == GATE_Y) and not np.any(t == GATE_SDG)
    meas = ops[t == OP_MEASURE]
    assert np.array_equal(meas["q0"], np.arange(64))
    assert ops[-64:]["type"].tolist() == [OP_MEASURE] * 64
    # density: about 0.8 single-qubit + 0.25 CX per qubit-layer
    assert 0.9 < count_gates(ops) / (64 * 10) < 1.2


def test_config2_mid_circuit_rounds():
    rounds = [arr for kind, arr in iter_circuit(CONFIGS[2]) if kind == "measure"]
    assert len(rounds) == 10
    assert all(r.size == 409 for r in rounds[:9]) and rounds[-1].size == 4096
    for r in rounds[:9]:
        assert np.all(np.diff(r.astype(np.int64)) > 0)
    layers = [arr for kind, arr in iter_circuit(CONFIGS[2], depth=5) if kind == "gates"]
    cz = sum(int(np.count_nonzero(l["type"] == GATE_CZ)) for l in layers)
    cx = sum(int(np.count_nonzero(l["type"] == GATE_CX)) for l in layers)
    assert 0.15 < cz / cx < 0.25


def test_pairs_are_disjoint_within_a_layer():
    for kind, arr in iter_circuit(CONFIGS[2], depth=3, final_measure=False):
        two = arr[(arr["type"] == GATE_CX) | (arr["type"] == GATE_CZ)]
        qs = np.concatenate([two["q0"], two["q1"]])
        assert np.unique(qs).size == qs.size


def test_served_mix_ranges():
    reqs = served_requests()
    assert len(reqs) == 512
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 16 and ns.max() <= 16384
    assert 200 < np.median(ns) < 1200
    assert all(10 <= r.depth <= 500 for r in reqs)
    assert all(1 <= r.shots <= 4096 for r in reqs)
    assert all(b.arrival_s > a.arrival_s for a, b in zip(reqs, reqs[1:]))


def test_basis_circuit_planted_bits_match_the_oracle():
    """The planted bit string of basis_circuit is what the CHP oracle measures:
    every qubit deterministic, outcome b_q (and the generator's pairs are
    disjoint within a layer, so layers can be fused)."""
    from oracle import oracle as orc
    from workload import basis_circuit
    n, layers = 257, 40
    ops, bits = basis_circuit(n, layers, seed=11)
    assert set(np.unique(ops["type"])) <= {orc.CX, orc.CZ, orc.SWAP, orc.S, orc.SDG, orc.X, orc.Y, orc.Z}
    assert 0 < bits.sum() < n
    arr = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
    meas = np.stack([np.full(n, orc.MEASURE), np.arange(n), np.zeros(n)], 1).astype(np.uint32)
    t = orc.Tableau(n)
    out, rnd, _ = t.run(np.concatenate([arr, meas]), seed=1)
    assert not rnd.any()
    assert np.array_equal(out, bits)
    # dense products: after 40 layers the destabilizers' X parts are about
    # half full (|A| near n/2 for every qubit)
    x, _, _ = t.rows_array()
    assert np.mean([bin(int(w)).count("1") for w in x[:n].reshape(-1)]) > 16
