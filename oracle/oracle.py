"""ctypes binding of the CPU CHP oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import this module. It shares no code with the GPU library:
it loads ``oracle/libsq_oracle.so``, built from ``oracle/chp_oracle.c`` by
``build_oracle`` (plain gcc with OpenMP).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chp_oracle.c")
_STIM_SRC = os.path.join(_HERE, "stim_oracle.c")
_LIB = os.path.join(_HERE, "libsq_oracle.so")

# Operation type codes (records of three uint32: type, q0, q1).
I, H, S, SDG, X, Y, Z, CX, CZ, CY, SWAP, ISWAP, MEASURE = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 15
TWO_QUBIT = (CX, CZ, CY, SWAP, ISWAP)


def build_oracle(src: str = _SRC, out: str = _LIB, extra_flags: Sequence[str] = (), stim_src: str = _STIM_SRC) -> str:
    """Compile the oracle (the CHP tableau and the operator-tableau collapse) with gcc (always recompiles)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", *extra_flags, src, stim_src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def _bind(lib):
    u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    vp = ctypes.c_void_p
    lib.sqo_create.restype = vp
    lib.sqo_create.argtypes = [u32, vp, u32]
    lib.sqo_destroy.restype = None
    lib.sqo_destroy.argtypes = [vp]
    lib.sqo_words.restype = u32
    lib.sqo_words.argtypes = [vp]
    lib.sqo_nrows.restype = u32
    lib.sqo_nrows.argtypes = [vp]
    lib.sqo_odd_count.restype = u64
    lib.sqo_odd_count.argtypes = [vp]
    lib.sqo_badscratch_count.restype = u64
    lib.sqo_badscratch_count.argtypes = [vp]
    lib.sqo_det_phase2_count.restype = u64
    lib.sqo_det_phase2_count.argtypes = [vp]
    lib.sqo_get_rows.restype = None
    lib.sqo_get_rows.argtypes = [vp, vp, vp, vp]
    lib.sqo_set_rows.restype = None
    lib.sqo_set_rows.argtypes = [vp, vp, vp, vp]
    lib.sqo_rowsum.restype = ctypes.c_int
    lib.sqo_rowsum.argtypes = [vp, u32, u32]
    lib.sqo_run.restype = i64
    lib.sqo_run.argtypes = [vp, vp, u64, u64, u64, u64, vp, vp, ctypes.POINTER(u64)]
    lib.sqo_philox4x64_10.restype = None
    lib.sqo_philox4x64_10.argtypes = [vp, vp, vp]
    lib.sqo_coin.restype = ctypes.c_int
    lib.sqo_coin.argtypes = [u64, u64, u64]
    lib.sqo_frame_bit.restype = ctypes.c_int
    lib.sqo_frame_bit.argtypes = [u64, u64, u64]
    lib.sqo_frame_sample.restype = i64
    lib.sqo_frame_sample.argtypes = [u32, vp, u64, vp, u64, u32, vp]
    lib.sqo_g.restype = ctypes.c_int
    lib.sqo_g.argtypes = [ctypes.c_int] * 4
    lib.sqo_gsum_word.restype = ctypes.c_int
    lib.sqo_gsum_word.argtypes = [u64, u64, u64, u64]
    lib.sqo_num_threads.restype = ctypes.c_int
    lib.sqo_num_threads.argtypes = []
    lib.sqo_otab_create.restype = vp
    lib.sqo_otab_create.argtypes = [u32]
    lib.sqo_otab_destroy.restype = None
    lib.sqo_otab_destroy.argtypes = [vp]
    lib.sqo_otab_odd_count.restype = u64
    lib.sqo_otab_odd_count.argtypes = [vp]
    lib.sqo_otab_run.restype = i64
    lib.sqo_otab_run.argtypes = [vp, vp, u64, u64, u64, u64, vp, vp]
    lib.sqo_otab_get.restype = None
    lib.sqo_otab_get.argtypes = [vp] * 7
    lib.sqo_otab_set.restype = None
    lib.sqo_otab_set.argtypes = [vp] * 7
    lib.sqo_otab_image.restype = ctypes.c_int
    lib.sqo_otab_image.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp]
    del i32
    return lib


def load(path: Optional[str] = None):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ops_array(ops) -> np.ndarray:
    a = np.ascontiguousarray(ops)
    if a.dtype.names:
        a = np.ascontiguousarray(
            np.stack([a["type"], a["q0"], a["q1"]], axis=1).astype(np.uint32))
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32).reshape(-1, 3))
    return a


class Tableau:
    """A CHP tableau (or a subset of its rows) held by the oracle."""

    def __init__(self, n: int, rows: Optional[Sequence[int]] = None, lib=None):
        self.lib = lib if lib is not None else load()
        self.n = int(n)
        if rows is None:
            self._rows = None
            h = self.lib.sqo_create(self.n, None, 0)
            self.rows = np.arange(2 * self.n, dtype=np.uint32)
        else:
            self.rows = np.ascontiguousarray(np.asarray(rows, dtype=np.uint32))
            h = self.lib.sqo_create(self.n, self.rows.ctypes.data, int(self.rows.size))
        if not h:
            raise ValueError("oracle: bad tableau arguments")
        self.h = ctypes.c_void_p(h)
        self.W = int(self.lib.sqo_words(self.h))

    def close(self):
        if self.h:
            self.lib.sqo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, ops, seed: int = 0, shot: int = 0, meas_base: int = 0
            ) -> Tuple[np.ndarray, np.ndarray, int]:
        """Run operations in order. Returns (outcomes, was_random, ops_done)."""
        a = _ops_array(ops)
        nmeas = int(np.count_nonzero(a[:, 0] == MEASURE))
        bits = np.zeros(max(nmeas, 1), dtype=np.uint8)
        rnd = np.zeros(max(nmeas, 1), dtype=np.uint8)
        done = ctypes.c_uint64(0)
        m = self.lib.sqo_run(self.h, a.ctypes.data, a.shape[0], seed, shot, meas_base,
                             bits.ctypes.data, rnd.ctypes.data, ctypes.byref(done))
        return bits[:m].copy(), rnd[:m].copy(), int(done.value)

    def rows_array(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(x, z, r): x and z are (rows, W) uint64, row-major, LSB-first."""
        nr = int(self.rows.size)
        x = np.zeros((nr, self.W), dtype=np.uint64)
        z = np.zeros((nr, self.W), dtype=np.uint64)
        r = np.zeros(nr, dtype=np.uint8)
        self.lib.sqo_get_rows(self.h, x.ctypes.data, z.ctypes.data, r.ctypes.data)
        return x, z, r

    def set_rows(self, x: np.ndarray, z: np.ndarray, r: np.ndarray):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        r = np.ascontiguousarray(r, dtype=np.uint8)
        assert x.shape == (self.rows.size, self.W) and z.shape == x.shape and r.shape == (self.rows.size,)
        self.lib.sqo_set_rows(self.h, x.ctypes.data, z.ctypes.data, r.ctypes.data)

    def rowsum(self, h: int, i: int) -> int:
        return int(self.lib.sqo_rowsum(self.h, h, i))

    @property
    def odd_count(self) -> int:
        return int(self.lib.sqo_odd_count(self.h))

    @property
    def det_phase2_count(self) -> int:
        """Deterministic outcomes whose summed phase exponents were 2 (mod 4)."""
        return int(self.lib.sqo_det_phase2_count(self.h))

    @property
    def badscratch_count(self) -> int:
        return int(self.lib.sqo_badscratch_count(self.h))


class OTableau:
    """The operator tableau T = C^dagger of the paper's CX-injection collapse
    (Algorithm alg:stim), held by the oracle: matrices XS, XD, ZS, ZD
    [generator k, qubit q] and sign vectors SignsS, SignsD over qubits."""

    def __init__(self, n: int, lib=None):
        self.lib = lib if lib is not None else load()
        self.n = int(n)
        h = self.lib.sqo_otab_create(self.n)
        if not h:
            raise ValueError("oracle: bad operator tableau size")
        self.h = ctypes.c_void_p(h)
        self.W = (self.n + 63) // 64

    def close(self):
        if self.h:
            self.lib.sqo_otab_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, ops, seed: int = 0, shot: int = 0, meas_base: int = 0) -> Tuple[np.ndarray, np.ndarray]:
        """Run operations in order; returns (outcomes, was_random)."""
        a = _ops_array(ops)
        nmeas = int(np.count_nonzero(a[:, 0] == MEASURE))
        bits = np.zeros(max(nmeas, 1), dtype=np.uint8)
        rnd = np.zeros(max(nmeas, 1), dtype=np.uint8)
        m = self.lib.sqo_otab_run(self.h, a.ctypes.data, a.shape[0], seed, shot, meas_base,
                                  bits.ctypes.data, rnd.ctypes.data)
        return bits[:m].copy(), rnd[:m].copy()

    def arrays(self):
        """(xs, xd, zs, zd, ss, sd): four (n, W) uint64 matrices and two (W,) sign vectors."""
        mats = [np.zeros((self.n, self.W), dtype=np.uint64) for _ in range(4)]
        sv = [np.zeros(self.W, dtype=np.uint64) for _ in range(2)]
        self.lib.sqo_otab_get(self.h, *[m.ctypes.data for m in mats], *[v.ctypes.data for v in sv])
        return (*mats, *sv)

    def set_arrays(self, xs, xd, zs, zd, ss, sd):
        arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (xs, xd, zs, zd, ss, sd)]
        for a in arrs[:4]:
            assert a.shape == (self.n, self.W)
        for a in arrs[4:]:
            assert a.shape == (self.W,)
        self.lib.sqo_otab_set(self.h, *[a.ctypes.data for a in arrs])

    def image(self, x, z, r: int):
        """T(P) of the Pauli (x, z, r) in the CHP encoding: (ox, oz, sign, phase_not_real)."""
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        ox = np.zeros(self.W, dtype=np.uint64)
        oz = np.zeros(self.W, dtype=np.uint64)
        sg = np.zeros(1, dtype=np.uint8)
        bad = self.lib.sqo_otab_image(self.h, x.ctypes.data, z.ctypes.data, int(r), ox.ctypes.data,
                                      oz.ctypes.data, sg.ctypes.data)
        return ox, oz, int(sg[0]), bool(bad)

    @property
    def odd_count(self) -> int:
        return int(self.lib.sqo_otab_odd_count(self.h))


def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    lib = load()
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.sqo_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def coin(seed: int, shot: int, m: int) -> int:
    return int(load().sqo_coin(seed, shot, m))


def frame_bit(seed: int, shot: int, event: int, lib=None) -> int:
    """Random bit of a shot for one frame event (see sqo_frame_sample)."""
    return int((lib or load()).sqo_frame_bit(seed, shot, event))


def frame_sample(n: int, ops, ref, seed: int, shots: int, lib=None) -> np.ndarray:
    """Pauli-frame samples (shots x ceil(M/64) words) of a program against a
    reference outcome vector ref (one 0/1 per measurement)."""
    lib = lib or load()
    a = np.ascontiguousarray(np.asarray(ops, dtype=np.uint32).reshape(-1, 3))
    m = int(np.count_nonzero(a[:, 0] == MEASURE))
    r = np.ascontiguousarray(np.asarray(ref, dtype=np.uint8).reshape(-1))
    if r.size != m:
        raise ValueError(f"reference has {r.size} outcomes, program measures {m}")
    W = max((m + 63) // 64, 1)
    out = np.zeros((max(shots, 1), W), dtype=np.uint64)
    got = lib.sqo_frame_sample(n, a.ctypes.data, a.shape[0], r.ctypes.data, seed, shots, out.ctypes.data)
    if got < 0:
        raise ValueError("bad program")
    return out[:shots, :(m + 63) // 64]


def num_threads() -> int:
    return int(load().sqo_num_threads())
