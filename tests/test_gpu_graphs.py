"""Program gate segments replayed as HIP graphs (needs an MI355X).

From the second run of a program on a tableau, each gate segment is launched
as one graph captured on that run. Every replay is checked against the oracle
and against a tableau that launches kernel by kernel, with other eager work on
the tableau (gate lists, measurements, resets) between the replays.
"""
import numpy as np
import pytest

from gpu_util import mixed_program
from oracle import oracle as orc

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


def _same(got, want, what):
    for u, v, part in zip(got, want, ("x", "z", "signs")):
        assert u.shape == v.shape and np.array_equal(u, v), f"{what}: {part} differ"


def test_gate_program_replays_match_oracle():
    """A gates-only program run five times, an eager gate list applied
    between the runs: after every run the tableau equals the oracle's and
    that of a tableau with graphs off."""
    from paper_2603_14641_amd import Program, Tableau
    n = 300
    rng = np.random.default_rng(11)
    ops = mixed_program(rng, n, 8, p_meas=0.0, extra=True)
    prog = Program(n, ops)
    tg, te = Tableau(n), Tableau(n)
    te.set_graphs(False)
    ref = orc.Tableau(n)
    for rep in range(5):
        tg.run_to_host(prog)
        te.run_to_host(prog)
        ref.run(ops)
        want = ref.rows_array()
        _same(tg.export(), want, f"graph tableau after run {rep}")
        _same(te.export(), want, f"eager tableau after run {rep}")
        extra = mixed_program(rng, n, 1, p_meas=0.0)
        tg.apply_gates(extra)
        te.apply_gates(extra)
        ref.run(extra)
    captures, replays = tg.graph_stats()
    assert captures >= 1 and replays >= 4 * captures, (captures, replays)
    assert te.graph_stats() == (0, 0)


def test_program_with_measurements_replays():
    """Gate segments between mid-circuit measurements: four runs from
    |0...0> with different seeds give the oracle's outcomes and tableau each
    time, the measurement segments running eagerly between replayed gate
    segments."""
    from paper_2603_14641_amd import Program, Tableau
    n = 200
    rng = np.random.default_rng(12)
    ops = mixed_program(rng, n, 6, p_meas=0.05)
    nseg = int(np.count_nonzero(ops[:, 0] == orc.MEASURE))
    assert nseg > 0
    prog = Program(n, ops)
    t = Tableau(n)
    for seed in (3, 4, 5, 6):
        t.reset()
        bits, rnd = t.run_to_host(prog, seed=seed, shot=1)
        ref = orc.Tableau(n)
        rb, rr, _ = ref.run(ops, seed=seed, shot=1)
        assert np.array_equal(bits, rb) and np.array_equal(rnd, rr), f"outcomes, seed {seed}"
        _same(t.export(), ref.rows_array(), f"tableau, seed {seed}")
    captures, replays = t.graph_stats()
    assert captures >= 1 and replays >= 3 * captures


def test_new_launch_geometry_captures_again():
    """A tuning change between runs gives a new capture for the new launch
    geometry (on the second run under it); the results do not change. Runs:
    default (first), default (capture), A (first), A (capture), B (first),
    B (capture)."""
    from paper_2603_14641_amd import Program, Tableau
    n = 130
    rng = np.random.default_rng(13)
    ops = mixed_program(rng, n, 5, p_meas=0.0)
    prog = Program(n, ops)
    t = Tableau(n)
    ref = orc.Tableau(n)
    for rep, tun in enumerate([None, None, dict(layer_block=64, layer_wpt=1, layer_groups=3), None,
                               dict(layer_block=128, layer_wpt=2, layer_groups=5), None]):
        if tun:
            t.set_tuning(**tun)
        t.run_to_host(prog)
        ref.run(ops)
        _same(t.export(), ref.rows_array(), f"run {rep}")
    captures, replays = t.graph_stats()
    assert captures == 3 and replays == 3, (captures, replays)


def test_destroyed_program_graph_is_not_reused():
    """Graphs are keyed by a unique program id: a new program (possibly at
    the freed program's address) runs its own gates."""
    from paper_2603_14641_amd import Program, Tableau
    n = 100
    rng = np.random.default_rng(14)
    t = Tableau(n)
    ref = orc.Tableau(n)
    for k in range(4):
        ops = mixed_program(rng, n, 3, p_meas=0.0)
        prog = Program(n, ops)
        for _ in range(2):
            t.run_to_host(prog)
            ref.run(ops)
        prog.close()
        _same(t.export(), ref.rows_array(), f"program {k}")
    assert t.graph_stats() == (4, 4)


def test_cache_eviction_keeps_results():
    """More distinct segments than the cache holds (32): the oldest graphs are
    dropped (after the stream drains) and their programs, run again, start
    over kernel by kernel; every tableau state matches the oracle."""
    from paper_2603_14641_amd import Program, Tableau
    n = 40
    rng = np.random.default_rng(15)
    t = Tableau(n)
    ref = orc.Tableau(n)
    progs = []
    for k in range(36):
        ops = mixed_program(rng, n, 2, p_meas=0.0)
        progs.append((Program(n, ops), ops))
        for _ in range(2):
            t.run_to_host(progs[-1][0])
            ref.run(ops)
    _same(t.export(), ref.rows_array(), "after 36 programs")
    assert t.graph_stats() == (36, 36)
    for prog, ops in progs[:3]:  # evicted: first run again, then a new capture
        for _ in range(2):
            t.run_to_host(prog)
            ref.run(ops)
    _same(t.export(), ref.rows_array(), "after re-running evicted programs")
    assert t.graph_stats() == (39, 39)
    for prog, _ in progs:
        prog.close()
