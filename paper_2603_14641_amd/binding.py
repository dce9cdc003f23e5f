"""ctypes binding of libsq.so: argument marshalling only.

Every step of the simulation runs in the HIP kernels behind the C ABI
(include/sq.h). There is no CPU fallback: if the library is missing, or a
call fails, this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsq.so")

# status codes and op types (include/sq.h)
SQ_OK, SQ_EINVAL, SQ_ENOMEM, SQ_EDEVICE, SQ_ERANGE, SQ_ESTATE = 0, -1, -2, -3, -5, -6
I, H, S, SDG, X, Y, Z, CX, CZ, CY, SWAP, ISWAP, MEASURE = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 15
(K_LAYER, K_SIGNS, K_PIVOT, K_GATHER, K_ROWSUM, K_POST, K_BPIVOT, K_BPREP, K_BPASS, K_BFINAL,
 K_IPIVOT, K_IAPPLY, K_TRANSPOSE, K_RPREP, K_RROWSUM, K_RDET, K_RFINISH) = range(17)
KERNEL_NAMES = ["layer", "signs", "pivot", "gather", "rowsum", "post",
                "block_pivot", "block_prep", "block_pass", "block_final", "inject_pivot", "inject_apply",
                "transpose", "row_prep", "row_rowsum", "row_det", "row_finish"]
LAYOUT_COLUMNS, LAYOUT_ROWS = 0, 1  # sq_set_layout
COLLAPSE_ROWSUM, COLLAPSE_INJECT = 0, 1  # sq_set_collapse modes
MAX_MEAS_BLOCK = 32
PIVOT_AUTO = 255         # sq_tuning.pivot_waves: choose the pivot search automatically

EXPORTED = [
    "sq_last_error", "sq_version", "sq_bytes_required", "sq_create", "sq_destroy", "sq_reset", "sq_sync",
    "sq_num_qubits", "sq_apply_gates", "sq_measure", "sq_sample", "sq_batch_sample", "sq_program_create",
    "sq_program_destroy",
    "sq_program_num_measurements", "sq_program_num_gates", "sq_program_num_passes", "sq_program_gate_bytes",
    "sq_plan_gates",
    "sq_run", "sq_export_rows", "sq_export", "sq_import", "sq_measure_stats", "sq_error_flags",
    "sq_get_tuning", "sq_set_tuning", "sq_profile_enable", "sq_profile_read", "sq_profile_reset",
    "sq_qasm_parse", "sq_frame_sample", "sq_set_graphs", "sq_graph_stats",
    "sq_create_in", "sq_layout", "sq_batch_item_bytes", "sq_sample_many", "sq_sample_bytes",
    "sq_set_collapse", "sq_get_collapse", "sq_measure_noalloc", "sq_set_layout", "sq_get_layout",
]


class SqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sq error {status}: {msg}")
        self.status = status


class Tuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in (
        "layer_block", "layer_wpt", "layer_groups", "rowsum_block", "rowsum_wpt", "rowsum_cols",
        "det_cols", "meas_block", "pivot_waves")]


class BatchItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("ops", ctypes.c_void_p), ("nops", ctypes.c_uint64),
                ("qubits", ctypes.c_void_p), ("count", ctypes.c_uint32), ("shots", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("shot_begin", ctypes.c_uint64), ("meas_base", ctypes.c_uint64),
                ("out", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("max_batch_n", ctypes.c_uint32),
                ("streams", ctypes.c_uint32)]


class LayoutInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("K", ctypes.c_uint32), ("L", ctypes.c_uint32), ("Ls", ctypes.c_uint32),
                ("x_offset", ctypes.c_uint64), ("z_offset", ctypes.c_uint64), ("r_offset", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64)]


class ShotSet(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("shot_begin", ctypes.c_uint64), ("meas_base", ctypes.c_uint64),
                ("shots", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("out", ctypes.c_void_p)]


class MeasStats(ctypes.Structure):
    _fields_ = [("n_random", ctypes.c_uint64), ("n_det", ctypes.c_uint64),
                ("rowsum_bytes", ctypes.c_uint64), ("det_bytes", ctypes.c_uint64),
                ("blocks", ctypes.c_uint64), ("block_bytes", ctypes.c_uint64),
                ("inject_bytes", ctypes.c_uint64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libsq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    # torch ships its own HIP runtime under the same soname as the system one;
    # importing torch first makes libsq.so bind to that already-loaded copy, so
    # the process holds a single HIP runtime and both see the same devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    pvp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "sq_last_error": (ctypes.c_char_p, []),
        "sq_version": (ctypes.c_char_p, []),
        "sq_bytes_required": (ctypes.c_size_t, [u32]),
        "sq_create": (i32, [u32, vp, pvp]),
        "sq_create_in": (i32, [u32, vp, ctypes.c_size_t, vp, pvp]),
        "sq_layout": (i32, [u32, ctypes.POINTER(LayoutInfo)]),
        "sq_batch_item_bytes": (ctypes.c_size_t, [u32, u64, u32, u32, ctypes.POINTER(BatchOpts)]),
        "sq_sample_many": (i32, [vp, vp, u32, ctypes.POINTER(ShotSet), u32]),
        "sq_sample_bytes": (ctypes.c_size_t, [u32, u32, u32]),
        "sq_destroy": (i32, [vp]),
        "sq_reset": (i32, [vp]),
        "sq_sync": (i32, [vp]),
        "sq_set_collapse": (i32, [vp, u32]),
        "sq_get_collapse": (u32, [vp]),
        "sq_set_layout": (i32, [vp, u32]),
        "sq_get_layout": (u32, [vp]),
        "sq_num_qubits": (u32, [vp]),
        "sq_apply_gates": (i32, [vp, vp, u64]),
        "sq_measure": (i32, [vp, vp, u32, u64, u64, u64, vp, vp]),
        "sq_measure_noalloc": (i32, [vp, vp, u32, u64, u64, u64, vp, vp]),
        "sq_sample": (i32, [vp, vp, u32, u64, u64, u32, u64, vp]),
        "sq_batch_sample": (i32, [ctypes.POINTER(BatchItem), u32, ctypes.POINTER(BatchOpts), vp]),
        "sq_program_create": (i32, [u32, vp, u64, pvp]),
        "sq_program_destroy": (i32, [vp]),
        "sq_program_num_measurements": (u64, [vp]),
        "sq_program_num_gates": (u64, [vp]),
        "sq_program_num_passes": (u64, [vp]),
        "sq_program_gate_bytes": (u64, [vp]),
        "sq_plan_gates": (i32, [u32, vp, u64, vp, u64, ctypes.POINTER(u64)]),
        "sq_qasm_parse": (i32, [ctypes.c_char_p, ctypes.c_size_t, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u32)]),
        "sq_frame_sample": (i32, [vp, vp, u64, u32, vp, vp]),
        "sq_run": (i32, [vp, vp, u64, u64, u64, vp, vp]),
        "sq_export_rows": (i32, [vp, vp, u32, vp, vp, vp]),
        "sq_export": (i32, [vp, vp, vp, vp]),
        "sq_import": (i32, [vp, vp, vp, vp]),
        "sq_measure_stats": (i32, [vp, ctypes.POINTER(MeasStats)]),
        "sq_error_flags": (i32, [vp, ctypes.POINTER(u32)]),
        "sq_get_tuning": (i32, [vp, ctypes.POINTER(Tuning)]),
        "sq_set_tuning": (i32, [vp, ctypes.POINTER(Tuning)]),
        "sq_profile_enable": (i32, [vp, i32]),
        "sq_set_graphs": (i32, [vp, i32]),
        "sq_graph_stats": (i32, [vp, vp, vp]),
        "sq_profile_read": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]),
        "sq_profile_reset": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != SQ_OK:
        raise SqError(status, load().sq_last_error().decode())


def ops_array(ops) -> np.ndarray:
    """(count, 3) uint32 records (type, q0, q1) from a structured or plain array."""
    a = np.asarray(ops)
    if a.dtype.names:
        a = np.stack([a["type"], a["q0"], a["q1"]], axis=1)
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32).reshape(-1, 3))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Program:
    """A compiled circuit resident on the device (sq_program)."""

    def __init__(self, n: int, ops):
        self.lib = load()
        self._ops = ops_array(ops)
        h = ctypes.c_void_p()
        _check(self.lib.sq_program_create(int(n), self._ops.ctypes.data, self._ops.shape[0], ctypes.byref(h)))
        self.h = h
        self.n = int(n)
        self.num_measurements = int(self.lib.sq_program_num_measurements(h))
        self.num_gates = int(self.lib.sq_program_num_gates(h))
        self.num_passes = int(self.lib.sq_program_num_passes(h))
        self.gate_bytes = int(self.lib.sq_program_gate_bytes(h))

    def frame_sample(self, shots: int, seed: int = 0, ref=None, ref_seed: Optional[int] = None,
                     stream=None) -> np.ndarray:
        """Pauli-frame samples (shots x ceil(M/64) uint64 words, sq_frame_sample).
        ref: one 0/1 per measurement; by default the program's CHP outcomes
        for (ref_seed or seed, shot 0) on a fresh tableau."""
        m = self.num_measurements
        if ref is None:
            t = Tableau(self.n, stream=stream)
            try:
                ref, _ = t.run_to_host(self, seed=seed if ref_seed is None else ref_seed, shot=0)
            finally:
                t.close()
        r = np.ascontiguousarray(np.asarray(ref, dtype=np.uint8).reshape(-1))
        if r.size != m:
            raise ValueError(f"reference has {r.size} outcomes, program measures {m}")
        W = (m + 63) // 64
        out = np.zeros((max(int(shots), 1), max(W, 1)), dtype=np.uint64)
        _check(self.lib.sq_frame_sample(self.h, r.ctypes.data, int(seed), int(shots), out.ctypes.data,
                                        _stream_ptr(stream)))
        return out[:int(shots), :W]

    def close(self):
        if getattr(self, "h", None):
            self.lib.sq_program_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tableau:
    """A CHP tableau of n qubits resident on the current HIP device.

    buffer: optional device tensor (e.g. ``torch.empty(bytes_required(n),
    dtype=torch.uint8, device="cuda")``) whose storage holds the tableau
    (sq_create_in); the tableau keeps a reference to it."""

    def __init__(self, n: int, stream=None, buffer=None, collapse: int = COLLAPSE_ROWSUM):
        self.lib = load()
        h = ctypes.c_void_p()
        self.buffer = buffer
        if buffer is None:
            _check(self.lib.sq_create(int(n), _stream_ptr(stream), ctypes.byref(h)))
        else:
            nbytes = int(buffer.numel() * buffer.element_size())
            _check(self.lib.sq_create_in(int(n), int(buffer.data_ptr()), nbytes, _stream_ptr(stream),
                                         ctypes.byref(h)))
        self.h = h
        self.n = int(n)
        self.W = (self.n + 63) // 64
        if collapse != COLLAPSE_ROWSUM:
            self.set_collapse(collapse)

    def close(self):
        if getattr(self, "h", None):
            self.lib.sq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- evolution -----------------------------------------------------------
    def reset(self):
        _check(self.lib.sq_reset(self.h))

    def sync(self):
        _check(self.lib.sq_sync(self.h))

    def set_collapse(self, mode: int):
        """COLLAPSE_ROWSUM (generator signs, CHP rowsum) or COLLAPSE_INJECT
        (image signs, CX-injection collapse); resets to |0...0>."""
        _check(self.lib.sq_set_collapse(self.h, int(mode)))

    @property
    def collapse(self) -> int:
        return int(self.lib.sq_get_collapse(self.h))

    def set_layout(self, layout: int):
        """LAYOUT_COLUMNS or LAYOUT_ROWS (queues the in-place transpose)."""
        _check(self.lib.sq_set_layout(self.h, int(layout)))

    @property
    def layout(self) -> int:
        return int(self.lib.sq_get_layout(self.h))

    def apply_gates(self, ops):
        a = ops_array(ops)
        _check(self.lib.sq_apply_gates(self.h, a.ctypes.data, a.shape[0]))

    def measure(self, qubits: Sequence[int], seed: int = 0, shot: int = 0, meas_base: int = 0
                ) -> Tuple[np.ndarray, np.ndarray]:
        q = np.ascontiguousarray(np.asarray(qubits, dtype=np.uint32).reshape(-1))
        bits = np.zeros(max(q.size, 1), dtype=np.uint8)
        rnd = np.zeros(max(q.size, 1), dtype=np.uint8)
        _check(self.lib.sq_measure(self.h, q.ctypes.data, q.size, seed, shot, meas_base,
                                   bits.ctypes.data, rnd.ctypes.data))
        return bits[:q.size], rnd[:q.size]

    def sample(self, qubits: Sequence[int], shots: int, seed: int = 0, shot_begin: int = 0,
               meas_base: int = 0) -> np.ndarray:
        """(shots, ceil(count/64)) uint64 words: bit i%64 of word i/64 = outcome i of that shot."""
        q = np.ascontiguousarray(np.asarray(qubits, dtype=np.uint32).reshape(-1))
        W = (q.size + 63) // 64
        out = np.zeros((max(int(shots), 1), max(W, 1)), dtype=np.uint64)
        _check(self.lib.sq_sample(self.h, q.ctypes.data, q.size, seed, shot_begin, int(shots), meas_base,
                                  out.ctypes.data))
        return out[:int(shots), :W]

    def sample_many(self, qubits: Sequence[int], sets) -> list:
        """Several shot sets (dicts with shots and optional seed, shot_begin,
        meas_base) of one measured list, sharing one sweep (sq_sample_many).
        Returns one (shots, ceil(count/64)) uint64 array per set."""
        q = np.ascontiguousarray(np.asarray(qubits, dtype=np.uint32).reshape(-1))
        W = (q.size + 63) // 64
        arr = (ShotSet * max(len(sets), 1))()
        outs = []
        for k, e in enumerate(sets):
            shots = int(e["shots"])
            out = np.zeros((max(shots, 1), max(W, 1)), dtype=np.uint64)
            outs.append(out)
            arr[k].seed = int(e.get("seed", 0))
            arr[k].shot_begin = int(e.get("shot_begin", 0))
            arr[k].meas_base = int(e.get("meas_base", 0))
            arr[k].shots = shots
            arr[k].out = out.ctypes.data
        _check(self.lib.sq_sample_many(self.h, q.ctypes.data, q.size, arr, len(sets)))
        return [o[:int(e["shots"]), :W] for o, e in zip(outs, sets)]

    def sample_bits(self, qubits: Sequence[int], shots: int, seed: int = 0, shot_begin: int = 0,
                    meas_base: int = 0) -> np.ndarray:
        """(shots, count) uint8 outcome bits."""
        words = self.sample(qubits, shots, seed, shot_begin, meas_base)
        count = len(np.asarray(qubits).reshape(-1))
        bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")
        return bits[:, :count]

    def run(self, program: Program, seed: int, shot: int, meas_base: int, dev_bits_ptr: int,
            dev_rand_ptr: Optional[int] = None):
        """Queue a program; outcomes land in device buffers (e.g. torch uint8 tensors' data_ptr())."""
        _check(self.lib.sq_run(self.h, program.h, seed, shot, meas_base, dev_bits_ptr, dev_rand_ptr))

    def run_to_host(self, program: Program, seed: int = 0, shot: int = 0, meas_base: int = 0
                    ) -> Tuple[np.ndarray, np.ndarray]:
        """Run a program and copy its outcomes back (uses torch for the device buffers)."""
        import torch
        m = max(program.num_measurements, 1)
        bits = torch.zeros(m, dtype=torch.uint8, device="cuda")
        rnd = torch.zeros(m, dtype=torch.uint8, device="cuda")
        torch.cuda.current_stream().synchronize()
        self.run(program, seed, shot, meas_base, bits.data_ptr(), rnd.data_ptr())
        self.sync()
        k = program.num_measurements
        return bits.cpu().numpy()[:k], rnd.cpu().numpy()[:k]

    # -- state access --------------------------------------------------------
    def export_rows(self, rows: Sequence[int]) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint32).reshape(-1))
        x = np.zeros((r.size, self.W), dtype=np.uint64)
        z = np.zeros((r.size, self.W), dtype=np.uint64)
        s = np.zeros(r.size, dtype=np.uint8)
        _check(self.lib.sq_export_rows(self.h, r.ctypes.data, r.size, x.ctypes.data, z.ctypes.data, s.ctypes.data))
        return x, z, s

    def export(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        rows = 2 * self.n
        x = np.zeros((rows, self.W), dtype=np.uint64)
        z = np.zeros((rows, self.W), dtype=np.uint64)
        s = np.zeros(rows, dtype=np.uint8)
        _check(self.lib.sq_export(self.h, x.ctypes.data, z.ctypes.data, s.ctypes.data))
        return x, z, s

    def import_(self, x: np.ndarray, z: np.ndarray, r: np.ndarray):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        r = np.ascontiguousarray(r, dtype=np.uint8)
        assert x.shape == (2 * self.n, self.W) and z.shape == x.shape and r.shape == (2 * self.n,)
        _check(self.lib.sq_import(self.h, x.ctypes.data, z.ctypes.data, r.ctypes.data))

    def error_flags(self) -> int:
        f = ctypes.c_uint32(0)
        _check(self.lib.sq_error_flags(self.h, ctypes.byref(f)))
        return int(f.value)

    def measure_stats(self) -> MeasStats:
        s = MeasStats()
        _check(self.lib.sq_measure_stats(self.h, ctypes.byref(s)))
        return s

    # -- tuning and profiling ------------------------------------------------
    def tuning(self) -> Tuning:
        t = Tuning()
        _check(self.lib.sq_get_tuning(self.h, ctypes.byref(t)))
        return t

    def set_tuning(self, **kw):
        t = Tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(self.lib.sq_set_tuning(self.h, ctypes.byref(t)))

    def set_graphs(self, on: bool = True):
        """Replay program gate segments as HIP graphs from their second run (default on)."""
        _check(self.lib.sq_set_graphs(self.h, 1 if on else 0))

    def graph_stats(self) -> Tuple[int, int]:
        """(segments captured as graphs, graph launches) since creation."""
        c, r = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(self.lib.sq_graph_stats(self.h, ctypes.byref(c), ctypes.byref(r)))
        return int(c.value), int(r.value)

    def profile(self, on: bool = True):
        _check(self.lib.sq_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(self.lib.sq_profile_reset(self.h))

    def profile_read(self, kernel: int) -> Tuple[float, int]:
        ms = ctypes.c_double(0)
        n = ctypes.c_uint64(0)
        _check(self.lib.sq_profile_read(self.h, kernel, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


def batch_sample(requests, block: int = 0, grid: int = 0, max_batch_n: int = 0, streams: int = 0, stream=None):
    """Run many independent circuits in one batched launch (sq_batch_sample).

    Each request is a dict with n, ops (gates), qubits, shots and optional
    seed, shot_begin, meas_base. Returns a list of (shots, ceil(count/64))
    uint64 outcome-word arrays."""
    lib = load()
    keep, outs = [], []
    arr = (BatchItem * max(len(requests), 1))()
    for k, r in enumerate(requests):
        ops = ops_array(r["ops"])
        q = np.ascontiguousarray(np.asarray(r["qubits"], dtype=np.uint32).reshape(-1))
        W = (q.size + 63) // 64
        out = np.zeros((max(int(r["shots"]), 1), max(W, 1)), dtype=np.uint64)
        keep += [ops, q]
        outs.append(out)
        it = arr[k]
        it.n = int(r["n"])
        it.ops = ops.ctypes.data if ops.size else None
        it.nops = ops.shape[0]
        it.qubits = q.ctypes.data if q.size else None
        it.count = q.size
        it.shots = int(r["shots"])
        it.seed = int(r.get("seed", 0))
        it.shot_begin = int(r.get("shot_begin", 0))
        it.meas_base = int(r.get("meas_base", 0))
        it.out = out.ctypes.data
    opts = BatchOpts(block, grid, max_batch_n, streams)
    _check(lib.sq_batch_sample(arr, len(requests), ctypes.byref(opts), _stream_ptr(stream)))
    res = []
    for r, out in zip(requests, outs):
        W = (len(np.asarray(r["qubits"]).reshape(-1)) + 63) // 64
        res.append(out[:int(r["shots"]), :W])
    return res


def words_to_bits(words: np.ndarray, count: int) -> np.ndarray:
    bits = np.unpackbits(np.ascontiguousarray(words).view(np.uint8), axis=1, bitorder="little")
    return bits[:, :count]


def plan_gates(n: int, ops) -> list:
    """Host-only: the pass plan of a gate sequence, as a list of passes, each a
    list of groups (header, qubits, micro-ops); see sq_plan_gates."""
    lib = load()
    a = ops_array(ops)
    need = ctypes.c_uint64(0)
    _check(lib.sq_plan_gates(int(n), a.ctypes.data, a.shape[0], None, 0, ctypes.byref(need)))
    buf = np.zeros(max(int(need.value), 1), dtype=np.uint64)
    _check(lib.sq_plan_gates(int(n), a.ctypes.data, a.shape[0], buf.ctypes.data, buf.size, ctypes.byref(need)))
    passes, k = [], 0
    while k < int(need.value):
        cnt = int(buf[k])
        k += 1
        groups = []
        for _ in range(cnt):
            hdr = int(buf[k])
            nq, nops = hdr & 15, (hdr >> 4) & 63
            qubits = [int(v) for v in buf[k + 1:k + 1 + nq]]
            uops = [int(v) for v in buf[k + 1 + nq:k + 1 + nq + nops]]
            groups.append((hdr, qubits, uops))
            k += 1 + nq + nops
        passes.append(groups)
    return passes


def parse_qasm(text) -> Tuple[int, np.ndarray]:
    """Host-only: an OpenQASM 2.0 circuit as (qubit count, (k, 3) uint32 op records)."""
    lib = load()
    data = text.encode() if isinstance(text, str) else bytes(text)
    count, n = ctypes.c_uint64(0), ctypes.c_uint32(0)
    _check(lib.sq_qasm_parse(data, len(data), None, 0, ctypes.byref(count), ctypes.byref(n)))
    out = np.zeros((max(int(count.value), 1), 3), dtype=np.uint32)
    _check(lib.sq_qasm_parse(data, len(data), out.ctypes.data, int(count.value), ctypes.byref(count),
                             ctypes.byref(n)))
    return int(n.value), out[:int(count.value)]


def bytes_required(n: int) -> int:
    return int(load().sq_bytes_required(int(n)))


def layout(n: int) -> dict:
    """Where X, Z and the signs sit in a tableau's device block (sq_layout)."""
    info = LayoutInfo()
    _check(load().sq_layout(int(n), ctypes.byref(info)))
    return {name: int(getattr(info, name)) for name, _ in LayoutInfo._fields_}


def sample_bytes(n: int, count: int, shots: int) -> int:
    """Device scratch bytes of sq_sample / sq_sample_many (sq_sample_bytes)."""
    return int(load().sq_sample_bytes(int(n), int(count), int(shots)))


def batch_item_bytes(n: int, nops: int, count: int, shots: int, block: int = 0, max_batch_n: int = 0) -> int:
    """Device bytes sq_batch_sample holds for such an item (sq_batch_item_bytes)."""
    opts = BatchOpts(block, 0, max_batch_n, 0)
    return int(load().sq_batch_item_bytes(int(n), int(nops), int(count), int(shots), ctypes.byref(opts)))


def version() -> str:
    return load().sq_version().decode()
