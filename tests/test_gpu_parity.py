"""Bit-exact parity of the HIP path with the CPU oracle (needs an MI355X).

Every comparison is element by element with tolerance 0: tableau x/z bits,
sign bits, measurement outcomes and the random/deterministic flags. The
oracle never sees GPU output; the GPU sometimes starts from an oracle-made
tableau (import).
"""
import numpy as np
import pytest

from gpu_util import gpu_run_calls, mixed_program, oracle_run, segments
from oracle import oracle as orc
from workload import CONFIGS, circuit_ops, iter_circuit

pytestmark = pytest.mark.gpu

SMALL_TILES = dict(layer_block=64, layer_wpt=1, layer_groups=3, rowsum_block=64, rowsum_wpt=1, rowsum_cols=5,
                   det_cols=2, meas_block=1)
SMALL_TILES_W2 = dict(layer_block=64, layer_wpt=2, layer_groups=7, rowsum_block=128, rowsum_wpt=2, rowsum_cols=3,
                      det_cols=3, meas_block=3)
SINGLE = dict(meas_block=1)   # one measurement at a time (the default applies runs of up to 32 in one pass)


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2603_14641_amd as sq
    sq.load()
    yield


def _tab(n, tuning=None):
    from paper_2603_14641_amd import Tableau
    t = Tableau(n)
    if tuning:
        t.set_tuning(**tuning)
    return t


def _assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        idx = np.argwhere(got != want)
        raise AssertionError(f"{what}: {idx.shape[0]} mismatches, first at {idx[:5].tolist()}")


def _compare_full(t, ref):
    x, z, r = t.export()
    rx, rz, rr = ref
    _assert_same(x, rx, "x bits")
    _assert_same(z, rz, "z bits")
    _assert_same(r, rr, "signs")
    assert t.error_flags() == 0


# ------------------------------------------------------------------ configs
@pytest.mark.parametrize("path", ["program", "calls"])
def test_config1_full(path):
    from paper_2603_14641_amd import Program
    cfg = CONFIGS[1]
    ops = circuit_ops(cfg)
    seed = 11
    rb, rr, x, z, r, _ = oracle_run(cfg.n, ops, seed)
    t = _tab(cfg.n)
    if path == "program":
        bits, rnd = t.run_to_host(Program(cfg.n, ops), seed=seed, shot=0)
    else:
        bits, rnd = gpu_run_calls(t, ops, seed)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))


def test_config2_full():
    """n = 4096, depth 100, CZ on, nine mid-circuit rounds of 409 qubits, then all 4096."""
    from paper_2603_14641_amd import Program
    cfg = CONFIGS[2]
    ops = circuit_ops(cfg)
    seed = 2
    rb, rr, x, z, r, _ = oracle_run(cfg.n, ops, seed)
    t = _tab(cfg.n)
    prog = Program(cfg.n, ops)
    assert prog.num_measurements == 9 * 409 + 4096
    bits, rnd = t.run_to_host(prog, seed=seed, shot=0)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))
    st = t.measure_stats()
    assert st.n_random + st.n_det == prog.num_measurements
    assert st.n_random == int(rr.sum())
    assert st.blocks > 0


# ------------------------------------------------------------------ blocked random measurements
def _measure_sequence(rng, n, count):
    """Random qubits with repeats: a repeat inside a run is deterministic and
    ends a block early."""
    qs = rng.integers(0, n, count)
    for k in range(0, count - 1, 7):
        qs[k + 1] = qs[k]
    return qs


@pytest.mark.parametrize("n", [2, 5, 64, 65, 300, 2000])
@pytest.mark.parametrize("mb", [2, 5, 16, 32])
def test_blocked_measurements(n, mb):
    """Runs of random measurements applied up to mb at a time in one pass:
    outcomes, flags and the whole tableau bit-exact with one-at-a-time CHP."""
    rng = np.random.default_rng(n * 100 + mb)
    prep = mixed_program(rng, n, 8, p_meas=0.0)
    qs = _measure_sequence(rng, n, min(3 * n, 80))
    meas = np.array([[orc.MEASURE, int(q), 0] for q in qs], dtype=np.uint32)
    ops = np.concatenate([prep, meas, mixed_program(rng, n, 2, p_meas=0.5)])
    seed = int(rng.integers(1 << 40))
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=2, meas_base=9)
    t = _tab(n, dict(meas_block=mb))
    bits, rnd = gpu_run_calls(t, ops, seed, shot=2, meas_base=9)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))
    st = t.measure_stats()
    assert st.n_random == int(rr.sum()) and st.n_det == int((rr == 0).sum())
    if n >= 64:  # small n can see deterministic measurements first in every block
        assert st.blocks > 0


def _deep_pivot_program(rng, n, lo, hi0, count, qs=None):
    """Superpositions on qubits [0, lo) and [hi0, n) only: measuring a high
    qubit finds its pivot among stabilizer rows >= hi0 (later 64-word tiles),
    a low one in the first word, an untouched one nothing (deterministic,
    which ends a block). The measured qubits mix all three (or are qs)."""
    hi = np.arange(hi0, n)
    ops = [[orc.H, int(q), 0] for q in hi] + [[orc.H, q, 0] for q in range(lo)]
    perm = rng.permutation(hi)
    ops += [[orc.CX, int(a), int(b)] for a, b in zip(perm[::2], perm[1::2])]
    ops += [[orc.S, int(q), 0] for q in rng.choice(hi, hi.size // 4, replace=False)]
    ops += [[orc.CX, a, a + 1] for a in range(0, lo - 1, 2)]
    if qs is not None:
        ops += [[orc.MEASURE, int(q), 0] for q in qs]
        return np.array(ops, dtype=np.uint32)
    qs = []
    for _ in range(count):
        u = rng.random()
        if u < 0.55:
            qs.append(int(rng.choice(hi)))
        elif u < 0.9:
            qs.append(int(rng.integers(0, lo)))
        else:
            qs.append(int(rng.integers(lo, hi0)))
    ops += [[orc.MEASURE, q, 0] for q in qs]
    return np.array(ops, dtype=np.uint32)


@pytest.mark.parametrize("n,hi0", [(5000, 4100), (20000, 16500)])
@pytest.mark.parametrize("pw", ["auto", 1, 2, 16])
def test_blocked_deep_pivots(n, hi0, pw):
    """Pivots spread over several 64-word tiles of the stabilizer half, for
    both pivot searches: registers (automatic at these sizes) and the tiled
    one with 1, 2 or 16 waves (16 runs as 8, its maximum; a wave owning
    several tiles walks them in order, each word formed from the block's
    columns). Outcomes, flags and the whole tableau bit-exact with
    one-at-a-time CHP."""
    rng = np.random.default_rng(n + (0 if pw == "auto" else pw))
    ops = _deep_pivot_program(rng, n, 40, hi0, 96)
    seed = int(rng.integers(1 << 40))
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=1)
    assert rr.sum() >= 40 and (rr == 0).sum() >= 8
    tun = dict(meas_block=32)
    if pw != "auto":
        tun["pivot_waves"] = pw
    t = _tab(n, tun)
    bits, rnd = gpu_run_calls(t, ops, seed, shot=1)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))
    assert t.measure_stats().blocks > 0


@pytest.mark.parametrize("n,hi0", [(5000, 4100), (20000, 16500)])
@pytest.mark.parametrize("pw", [1, 2, 16])
def test_tiled_search_starts_at_first_nonzero_bound(n, hi0, pw):
    """The tiled search starts step s at the smallest first-nonzero
    stabilizer word of the block's columns so far. Blocks here open with
    high qubits (columns zero below word hi0 / 64) and then drop to low ones,
    so later steps start below where earlier rows were written (those rows
    are stale there and must read as zero). Other blocks are all high, or
    hold an untouched qubit (a column with no nonzero word) first or in the
    middle. Outcomes, flags and the whole tableau bit-exact with CHP."""
    rng = np.random.default_rng(77 * n + pw)
    lo = 40
    hi = np.arange(hi0, n)
    mid = np.arange(lo, hi0)
    pick = lambda a, m: [int(x) for x in rng.choice(a, m, replace=False)]
    qs = (pick(hi, 1) + pick(range(lo), 31)          # bound drops after step 0
          + pick(hi, 32)                              # bound stays high
          + pick(mid, 1) + pick(hi, 4)                # deterministic first
          + pick(hi, 3) + pick(range(lo), 4) + pick(mid, 1) + pick(hi, 8)
          + pick(hi, 2) + pick(range(lo), 30))
    ops = _deep_pivot_program(rng, n, lo, hi0, 0, qs=qs)
    seed = int(rng.integers(1 << 40))
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=1)
    assert rr.sum() >= 40 and (rr == 0).sum() >= 2
    t = _tab(n, dict(meas_block=32, pivot_waves=pw))
    bits, rnd = gpu_run_calls(t, ops, seed, shot=1)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))
    assert t.measure_stats().blocks > 0


@pytest.mark.parametrize("n", [32768, 32769])
def test_blocked_pivots_at_register_limit(n):
    """The register pivot search at its largest size (8 tiles of 64
    stabilizer words, 512 threads) and one qubit more (9 tiles: the tiled
    search), with pivots in the last tiles: outcomes, flags and 1,024 rows
    (the pivots' stabilizer and destabilizer rows among them) bit-exact with
    one-at-a-time CHP."""
    rng = np.random.default_rng(n)
    ops = _deep_pivot_program(rng, n, 40, n - 3000, 96)
    seed = 7
    ref = orc.Tableau(n)
    rb, rr, _ = ref.run(ops, seed=seed, shot=1)
    assert ref.odd_count == 0 and ref.badscratch_count == 0
    x, z, r = ref.rows_array()
    t = _tab(n)
    bits, rnd = gpu_run_calls(t, ops, seed, shot=1)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    rows = np.concatenate([np.arange(n - 3000, n - 2700), np.arange(2 * n - 3000, 2 * n - 2700),
                           np.arange(n, n + 40), np.arange(0, 40)])
    rows = np.unique(np.concatenate([rows, rng.choice(2 * n, 1024 - rows.size, replace=False)]))
    gx, gz, gr = t.export_rows(rows)
    _assert_same(gx, x[rows], "sampled x rows")
    _assert_same(gz, z[rows], "sampled z rows")
    _assert_same(gr, r[rows], "sampled signs")
    assert t.measure_stats().blocks > 0 and t.error_flags() == 0


def test_blocked_pivots_share_words():
    """n = 40 (one word of rows per half): every pivot of a block sits in the
    same 64-row word, as do the D rows they overwrite."""
    n = 40
    rng = np.random.default_rng(41)
    ops = np.concatenate([mixed_program(rng, n, 10, p_meas=0.0),
                          np.array([[orc.MEASURE, q, 0] for q in rng.permutation(n)], dtype=np.uint32)])
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed=3)
    assert rr[:16].sum() >= 8
    t = _tab(n)
    bits, rnd = gpu_run_calls(t, ops, seed=3)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))


# ------------------------------------------------------------------ tiles, ragged tails, all gate types
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 130, 700, 2500])
@pytest.mark.parametrize("tuning", [None, SINGLE, SMALL_TILES, SMALL_TILES_W2],
                         ids=["default", "single", "small", "small_w2"])
def test_mixed_circuits(n, tuning):
    rng = np.random.default_rng(1000 + n)
    layers = 6 if n >= 700 else 12
    ops = mixed_program(rng, n, layers, p_meas=0.15 if n > 3 else 0.4)
    seed = int(rng.integers(1 << 40))
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=3, meas_base=5)
    t = _tab(n, tuning)
    bits, rnd = gpu_run_calls(t, ops, seed, shot=3, meas_base=5)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))


@pytest.mark.parametrize("n", [2, 5, 64, 65, 300, 1500])
@pytest.mark.parametrize("tuning", [None, SMALL_TILES], ids=["default", "small"])
def test_all_gate_types(n, tuning):
    """CY, SWAP and iSWAP beside the other gates (the GPU applies them as
    products of its micro-ops, the oracle by its own rules)."""
    rng = np.random.default_rng(5000 + n)
    ops = mixed_program(rng, n, 8 if n >= 300 else 14, p_meas=0.15 if n > 2 else 0.4, extra=True)
    assert np.isin(ops[:, 0], [orc.CY, orc.SWAP, orc.ISWAP]).any() or n < 4
    seed = int(rng.integers(1 << 40))
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed, shot=1, meas_base=3)
    t = _tab(n, tuning)
    bits, rnd = gpu_run_calls(t, ops, seed, shot=1, meas_base=3)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, (x, z, r))


def test_program_and_calls_agree_with_oracle_many_small():
    """200 small circuits with dense measurement (many deterministic outcomes)."""
    from paper_2603_14641_amd import Program
    rng = np.random.default_rng(77)
    det = 0
    for k in range(200):
        n = int(rng.integers(2, 20))
        ops = mixed_program(rng, n, 8, p_meas=0.3)
        rb, rr, x, z, r, _ = oracle_run(n, ops, seed=k, shot=k)
        t = _tab(n)
        bits, rnd = t.run_to_host(Program(n, ops), seed=k, shot=k)
        _assert_same(bits, rb, f"outcomes circuit {k}")
        _assert_same(rnd, rr, f"flags circuit {k}")
        _compare_full(t, (x, z, r))
        det += int((rr == 0).sum())
    assert det > 200


# ------------------------------------------------------------------ deterministic phase with mixed generators
def _scrambled_state(n, rng, seed):
    """An oracle tableau where half the qubits have been measured (so Z_q is in
    the stabilizer group for those), then re-expressed in a random other
    generator basis by symplectic row operations S_i <- S_j S_i, D_j <- D_i D_j."""
    t = orc.Tableau(n)
    t.run(mixed_program(rng, n, 10, p_meas=0.0), seed=seed)
    meas = [[orc.MEASURE, q, 0] for q in range(0, n, 2)]
    t.run(np.array(meas, dtype=np.uint32), seed=seed, shot=0, meas_base=0)
    for _ in range(4 * n):
        i, j = (int(v) for v in rng.choice(n, 2, replace=False))
        assert t.rowsum(n + i, n + j) == 0
        assert t.rowsum(j, i) == 0
    return t


@pytest.mark.parametrize("n", [12, 40, 200, 1000])
def test_deterministic_phase_after_basis_scramble(n):
    from paper_2603_14641_amd import Program
    rng = np.random.default_rng(n * 10 + 1)
    ref = _scrambled_state(n, rng, seed=n)
    x0, z0, r0 = ref.rows_array()
    t = _tab(n, SMALL_TILES if n == 200 else None)
    t.import_(x0, z0, r0)
    _compare_full(t, (x0, z0, r0))
    qs = list(range(0, n, 2)) + list(rng.permutation(n)[: n // 2])
    prog_ops = np.array([[orc.MEASURE, int(q), 0] for q in qs], dtype=np.uint32)
    rb, rr, _ = ref.run(prog_ops, seed=9, shot=1, meas_base=100)
    assert ref.det_phase2_count > 0, "the scramble should give nonzero deterministic phase sums"
    bits, rnd = t.run_to_host(Program(n, prog_ops), seed=9, shot=1, meas_base=100)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    _compare_full(t, ref.rows_array())


# ------------------------------------------------------------------ edge cases
def test_empty_calls_and_errors_leave_state_unchanged():
    from paper_2603_14641_amd import SqError
    n = 70
    rng = np.random.default_rng(5)
    ops = mixed_program(rng, n, 3, p_meas=0.0)
    t = _tab(n)
    t.apply_gates(ops)
    before = t.export()
    t.apply_gates(np.zeros((0, 3), np.uint32))
    b, r = t.measure([])
    assert b.size == 0 and r.size == 0
    for bad in ([[orc.H, n, 0]], [[orc.CX, 3, 3]], [[orc.CZ, 1, n + 5]], [[12, 0, 0]], [[orc.MEASURE, 0, 0]]):
        with pytest.raises(SqError):
            t.apply_gates(np.array(bad, dtype=np.uint32))
    with pytest.raises(SqError):
        t.measure([0, n])
    for bad in (dict(pivot_waves=17), dict(meas_block=33), dict(layer_block=96)):
        with pytest.raises(SqError):
            t.set_tuning(**bad)
    assert t.tuning().pivot_waves == 255   # automatic, unchanged by the rejected calls
    after = t.export()
    for u, v in zip(before, after):
        _assert_same(u, v, "state after rejected calls")


def test_reset_import_export_roundtrip():
    n = 300
    rng = np.random.default_rng(6)
    ops = mixed_program(rng, n, 5, p_meas=0.1)
    rb, rr, x, z, r, _ = oracle_run(n, ops, seed=4)
    t = _tab(n)
    t.import_(x, z, r)
    _compare_full(t, (x, z, r))
    t.reset()
    fresh = orc.Tableau(n).rows_array()
    _compare_full(t, fresh)
    rows = rng.choice(2 * n, 37, replace=False)
    t.import_(x, z, r)
    ex, ez, er = t.export_rows(rows)
    _assert_same(ex, x[rows], "export_rows x")
    _assert_same(ez, z[rows], "export_rows z")
    _assert_same(er, r[rows], "export_rows r")


def test_measure_twice_and_program_mismatch():
    from paper_2603_14641_amd import Program, SqError
    n = 129
    rng = np.random.default_rng(8)
    t = _tab(n)
    t.apply_gates(mixed_program(rng, n, 8, p_meas=0.0))
    qs = rng.permutation(n)[:40]
    b1, r1 = t.measure(qs, seed=1, meas_base=0)
    b2, r2 = t.measure(qs, seed=2, meas_base=40)
    _assert_same(b2, b1, "re-measured outcomes")
    assert not r2.any()
    with pytest.raises(SqError):
        t.run(Program(n + 1, np.array([[orc.H, 0, 0]], dtype=np.uint32)), 0, 0, 0, 0)


# ------------------------------------------------------------------ full sizes, sampled rows
def _sampled_rows(n, rng, k_prefix=64, k_rand=32):
    rows = list(range(n, n + k_prefix)) + list(range(0, 16))
    extra = rng.choice(np.arange(16, 2 * n), k_rand, replace=False)
    rows += [int(v) for v in extra if not (n <= v < n + k_prefix)]
    return rows


@pytest.mark.parametrize("cfg_id,depth,nmeas", [(3, 40, 16), (4, 100, 40)])
def test_full_size_sampled_rows(cfg_id, depth, nmeas):
    """n = 65,536 and 180,000 in the default launch configuration: after
    `depth` generator layers and the first `nmeas` measurements of the final
    sweep, the oracle (holding only a sample of rows, which evolve
    independently under gates, and the stabilizer prefix that contains every
    pivot) must agree on the outcomes and on every sampled row."""
    from paper_2603_14641_amd import Program
    cfg = CONFIGS[cfg_id]
    n = cfg.n
    rng = np.random.default_rng(cfg_id)
    rows = _sampled_rows(n, rng)
    ops = circuit_ops(cfg, depth=depth, final_measure=False)
    meas = np.array([[orc.MEASURE, q, 0] for q in range(nmeas)], dtype=np.uint32)
    allops = np.concatenate([np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32), meas])
    sub = orc.Tableau(n, rows=rows)
    rb, rr, done = sub.run(allops, seed=cfg.seed, shot=0)
    assert rb.size == nmeas, "a pivot fell outside the sampled stabilizer prefix"
    t = _tab(n)
    prog = Program(n, allops)
    bits, rnd = t.run_to_host(prog, seed=cfg.seed, shot=0)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    x, z, r = t.export_rows(rows)
    sx, sz, sr = sub.rows_array()
    _assert_same(x, sx, "sampled x rows")
    _assert_same(z, sz, "sampled z rows")
    _assert_same(r, sr, "sampled signs")
    assert t.error_flags() == 0
    # measuring the same qubits again is deterministic and repeats the outcomes
    b2, r2 = t.measure(np.arange(nmeas), seed=5, meas_base=nmeas)
    _assert_same(b2, bits, "re-measured outcomes")
    assert not r2.any()


@pytest.mark.slow
def test_config3_full_depth_sampled_rows():
    """n = 65,536 at its full depth (1000 generator layers, 72 M gates, in
    the default launch configuration), then the first 16 measurements of the
    final sweep: outcomes and 56 sampled rows against the row-subset oracle."""
    from paper_2603_14641_amd import Program
    cfg = CONFIGS[3]
    n, nmeas = cfg.n, 16
    rng = np.random.default_rng(33)
    rows = sorted(set(list(range(n, n + 32)) + list(range(0, 8))
                      + [int(v) for v in rng.choice(np.arange(8, 2 * n), 16, replace=False)]))
    ops = circuit_ops(cfg, final_measure=False)
    assert int(np.count_nonzero(ops["type"] == orc.MEASURE)) == 0
    meas = np.array([[orc.MEASURE, q, 0] for q in range(nmeas)], dtype=np.uint32)
    allops = np.concatenate([np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32), meas])
    sub = orc.Tableau(n, rows=rows)
    rb, rr, _ = sub.run(allops, seed=cfg.seed, shot=0)
    assert rb.size == nmeas, "a pivot fell outside the sampled stabilizer prefix"
    t = _tab(n)
    bits, rnd = t.run_to_host(Program(n, allops), seed=cfg.seed, shot=0)
    _assert_same(bits, rb, "outcomes")
    _assert_same(rnd, rr, "random flags")
    x, z, r = t.export_rows(rows)
    sx, sz, sr = sub.rows_array()
    _assert_same(x, sx, "sampled x rows")
    _assert_same(z, sz, "sampled z rows")
    _assert_same(r, sr, "sampled signs")
    assert t.error_flags() == 0


def test_long_gate_list_compiled_in_chunks():
    """2^20 + 777 gates of every type through sq_apply_gates, which compiles
    lists this long in chunks on helper threads: 96 sampled rows against the
    oracle holding only those rows, and the whole tableau against the same
    gates run as a program (one builder)."""
    from paper_2603_14641_amd import Program
    n = 3000
    rng = np.random.default_rng(123)
    count = (1 << 20) + 777
    t = rng.integers(0, 12, count)
    a = rng.integers(0, n, count)
    b = (a + 1 + rng.integers(0, n - 1, count)) % n
    ops = np.stack([t, a, np.where(np.isin(t, orc.TWO_QUBIT), b, 0)], 1).astype(np.uint32)
    rows = sorted(int(v) for v in rng.choice(2 * n, 96, replace=False))
    sub = orc.Tableau(n, rows=rows)
    sub.run(ops)
    t1 = _tab(n)
    t1.apply_gates(ops)
    x, z, r = t1.export_rows(rows)
    sx, sz, sr = sub.rows_array()
    _assert_same(x, sx, "sampled x rows")
    _assert_same(z, sz, "sampled z rows")
    _assert_same(r, sr, "sampled signs")
    t2 = _tab(n)
    t2.run_to_host(Program(n, ops), seed=0, shot=0)
    for u, v, what in zip(t1.export(), t2.export(), ("x", "z", "signs")):
        _assert_same(u, v, f"{what}: chunked list vs program")


def test_layer_then_inverse_is_identity_at_180k():
    """Any size: a generator layer followed by its inverse restores |0...0> exactly, signs included."""
    cfg = CONFIGS[4]
    n = cfg.n
    layer = next(iter_circuit(cfg, depth=1, final_measure=False))[1]
    a = np.stack([layer["type"], layer["q0"], layer["q1"]], 1).astype(np.uint32)
    inv = a[::-1].copy()
    inv[inv[:, 0] == orc.S, 0] = 99
    inv[inv[:, 0] == orc.SDG, 0] = orc.S
    inv[inv[:, 0] == 99, 0] = orc.SDG
    t = _tab(n)
    t.apply_gates(a)
    rng = np.random.default_rng(0)
    rows = rng.choice(2 * n, 512, replace=False)
    x1, z1, _ = t.export_rows(rows)
    assert x1.any() or z1.any()
    t.apply_gates(inv)
    x, z, r = t.export_rows(rows)
    fresh = orc.Tableau(n, rows=rows).rows_array()
    _assert_same(x, fresh[0], "x after inverse")
    _assert_same(z, fresh[1], "z after inverse")
    _assert_same(r, fresh[2], "signs after inverse")
