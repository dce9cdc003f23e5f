"""Deterministic measurements whose product spans many stabilizers (the CHP
deterministic case with a dense set A), against the CPU oracle bit for bit
and, at full size, against the circuit's planted outcome (needs an MI355X).

The circuits (workload.basis_circuit) use only gates that keep computational
basis states basis states, so from |0...0> every Z measurement afterwards is
deterministic and its outcome is known without any tableau arithmetic; the
CX layers spread the destabilizers' X parts until Z_q is the product of
about n/2 stabilizer generators. Each collapse and layout has its own code
for this case: the column-layout product (k_pivot's list of A's words and
k_post), the blocked sweep (a deterministic measurement ends a block), the
row-layout product (k_row_det) and the CX-injection collapse.
"""
import numpy as np
import pytest

from gpu_util import oracle_run, otableau_state
from oracle import oracle as orc
from workload import basis_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        idx = np.argwhere(got != want)
        raise AssertionError(f"{what}: {idx.shape[0]} mismatches, first at {idx[:5].tolist()}")


def _gates(n, layers, seed):
    ops, bits = basis_circuit(n, layers, seed)
    return np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32), bits


def _meas(qubits):
    q = np.asarray(qubits, dtype=np.uint32)
    return np.stack([np.full(q.size, orc.MEASURE), q, np.zeros(q.size)], 1).astype(np.uint32)


MODES = ["single", "blocked", "rows", "inject", "det_cols_1"]


def _tableau(n, mode):
    from paper_2603_14641_amd import COLLAPSE_INJECT, COLLAPSE_ROWSUM, Tableau
    t = Tableau(n, collapse=COLLAPSE_INJECT if mode == "inject" else COLLAPSE_ROWSUM)
    if mode in ("single", "rows"):
        t.set_tuning(meas_block=1)
    if mode == "det_cols_1":
        t.set_tuning(meas_block=1, det_cols=1)
    return t


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 129, 700, 3000])
def test_dense_deterministic_products_match_oracle(n, mode):
    from paper_2603_14641_amd import LAYOUT_ROWS, Program
    rng = np.random.default_rng(7000 + n)
    gates, planted = _gates(n, 40, seed=n)
    order = rng.permutation(n)
    ops = np.concatenate([gates, _meas(order)])
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed=9)
    assert not rr.any()
    _assert_same(rb, planted[order], "oracle against planted bits")
    t = _tableau(n, mode)
    if gates.size:
        t.apply_gates(gates)
    if mode == "rows":
        t.set_layout(LAYOUT_ROWS)
        bits, rnd = t.measure(order, seed=9)
    else:
        prog = Program(n, _meas(order))
        bits, rnd = t.run_to_host(prog, seed=9)
        prog.close()
    _assert_same(bits, rb, f"{mode} outcomes")
    _assert_same(rnd, rr, f"{mode} flags")
    if mode == "inject":
        # the operator tableau holds the same bits but image signs: compare
        # with the operator-tableau oracle
        ot = orc.OTableau(n)
        ob, orr = ot.run(ops, seed=9)
        _assert_same(ob, rb, "operator-tableau oracle outcomes")
        assert ot.odd_count == 0
        x, z, r = otableau_state(ot)
    ex, ez, er = t.export()
    _assert_same(ex, x, f"{mode} x")
    _assert_same(ez, z, f"{mode} z")
    _assert_same(er, r, f"{mode} signs")
    assert t.error_flags() == 0
    st = t.measure_stats()
    if mode != "inject":
        assert st.n_det == n and st.n_random == 0
    t.close()


@pytest.mark.parametrize("n", [700, 3000])
def test_dense_products_after_random_measurements(n):
    """A random measurement first (the pivot's rowsum rewrites many rows),
    then dense deterministic products on the changed tableau, in columns."""
    from paper_2603_14641_amd import Program
    rng = np.random.default_rng(n)
    gates, _ = _gates(n, 40, seed=3 * n)
    h = np.array([[orc.H, q, 0] for q in rng.choice(n, 5, replace=False)], np.uint32)
    order = rng.permutation(n)
    ops = np.concatenate([gates, h, _meas(order)])
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed=4)
    assert rr.sum() == 5
    t = _tableau(n, "blocked")
    t.apply_gates(np.concatenate([gates, h]))
    prog = Program(n, _meas(order))
    bits, rnd = t.run_to_host(prog, seed=4)
    prog.close()
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "flags")
    ex, ez, er = t.export()
    _assert_same(ex, x, "x")
    _assert_same(ez, z, "z")
    _assert_same(er, r, "signs")
    t.close()


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", ["single", "blocked", "rows"])
def test_full_size_dense_products_equal_planted_outcomes(mode):
    """n = 180,000 after 64 layers: the first 128 qubits (and 128 more spread
    over the register) are deterministic with the planted outcomes; the
    kernels' own product check (the product must be +-Z_q) raises no flag."""
    import torch
    from paper_2603_14641_amd import LAYOUT_ROWS, Program
    n = 180000
    gates, planted = _gates(n, 64, seed=21)
    qs = np.concatenate([np.arange(128), np.linspace(128, n - 1, 128).astype(np.int64)])
    print(f"n={n}, {gates.shape[0]} gates, mode {mode}", flush=True)
    t = _tableau(n, mode)
    prog = Program(n, gates)
    t.run(prog, 1, 0, 0, 0, 0)
    prog.close()
    if mode == "rows":
        t.set_layout(LAYOUT_ROWS)
        bits, rnd = t.measure(qs, seed=1)
    else:
        bits, rnd = t.measure(qs, seed=1)
    assert not rnd.any()
    _assert_same(bits, planted[qs], f"{mode} outcomes")
    assert t.error_flags() == 0
    st = t.measure_stats()
    if mode != "rows":
        # every nonzero word of A is read once per column: dense A means
        # nearly all K words
        K = (n + 63) // 64
        assert st.det_bytes > 0.9 * qs.size * K * 16 * n
    t.close()
    torch.cuda.empty_cache()
