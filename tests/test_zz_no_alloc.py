"""sq_measure_noalloc (staging in the library's fixed device array, no
device allocation) against sq_measure on identical tableaux, through the C
ABI: outcomes, random flags and the whole exported tableau, bit for bit, on
two calls in a row (the second with a shorter list), in both collapse modes;
and the size limit (needs an MI355X)."""
import ctypes

import numpy as np
import pytest

from gpu_util import mixed_program

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


def _pair(n, gates, collapse):
    from paper_2603_14641_amd import Tableau
    a = Tableau(n, collapse=collapse)
    b = Tableau(n, collapse=collapse)
    a.apply_gates(gates)
    b.apply_gates(gates)
    return a, b


def _noalloc(t, qubits, seed, shot, base):
    from paper_2603_14641_amd import binding
    q = np.ascontiguousarray(qubits, dtype=np.uint32)
    bits = np.zeros(q.size, dtype=np.uint8)
    rnd = np.zeros(q.size, dtype=np.uint8)
    st = t.lib.sq_measure_noalloc(t.h, q.ctypes.data, q.size, seed, shot, base, bits.ctypes.data, rnd.ctypes.data)
    binding._check(st)
    return bits, rnd


@pytest.mark.parametrize("collapse", [0, 1])
@pytest.mark.parametrize("n", [5, 300, 4100])
def test_noalloc_equals_measure(n, collapse):
    rng = np.random.default_rng(60 + n + collapse)
    gates = mixed_program(rng, n, 8, p_meas=0.0, extra=True)
    a, b = _pair(n, gates, collapse)
    first = rng.permutation(n).astype(np.uint32)
    first = np.concatenate([first, first[: n // 3]])        # repeats: deterministic re-measurements
    second = rng.choice(n, max(1, n // 4), replace=False).astype(np.uint32)
    base = 0
    for k, qs in enumerate((first, second)):
        wb, wr = a.measure(qs, seed=77, shot=k, meas_base=base)
        gb, gr = _noalloc(b, qs, 77, k, base)
        assert np.array_equal(gb, wb), f"call {k}: outcomes differ"
        assert np.array_equal(gr, wr), f"call {k}: random flags differ"
        xa, za, ra = a.export()
        xb, zb, rb = b.export()
        assert np.array_equal(xa, xb) and np.array_equal(za, zb) and np.array_equal(ra, rb), f"call {k}: tableau"
        base += qs.size
    assert a.error_flags() == 0 and b.error_flags() == 0


def test_noalloc_limits():
    from paper_2603_14641_amd import Tableau, binding
    t = Tableau(8)
    assert t.lib.sq_measure_noalloc(t.h, None, 0, 0, 0, 0, None, None) == binding.SQ_OK
    big = np.zeros(1048577, dtype=np.uint32)
    out = np.zeros(big.size, dtype=np.uint8)
    st = t.lib.sq_measure_noalloc(t.h, big.ctypes.data, big.size, 0, 0, 0, out.ctypes.data, None)
    assert st == binding.SQ_ERANGE
    bad = np.array([8], dtype=np.uint32)
    st = t.lib.sq_measure_noalloc(t.h, bad.ctypes.data, 1, 0, 0, 0, out.ctypes.data, None)
    assert st == binding.SQ_ERANGE
    b, r = _noalloc(t, np.arange(8), 1, 0, 0)   # the tableau is still usable after rejected calls
    assert not r.any() and not b.any()
