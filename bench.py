#!/usr/bin/env python3
"""Throughput of the stabilizer-tableau hot path on one MI355X.

Timed step (the 180,000-qubit, depth-1000 generator circuit): reset to
|0...0>, apply all 1000 random layers (about 198 million non-identity gates,
fused into passes), then the first M Z measurements (qubits 0..M-1 in order)
of the circuit's final all-qubit measurement. Inputs (the compiled gate
passes and the measured list) are resident in HBM before timing starts;
outcomes stay on the device.

After the timed steps (not part of `value`):
  * full_sweep: the same circuit once more with all 180,000 final
    measurements (measurements/s over the whole sweep);
  * deterministic: the first 1000 qubits measured again on the swept
    tableau, every outcome deterministic;
  * dense_deterministic: deterministic measurements whose product spans
    about n/2 stabilizers (a basis-state-preserving circuit with planted
    outcomes), in columns and on rows;
  * batched_served: the 512-request batched/served mix, all of it, on the
    plain per-circuit path, the batched path, the serving loop (Poisson
    arrivals) and the Pauli-frame path, plus sampling requests against
    resident tableaux (sessions);
  * cpu_baseline: the CPU oracle on a bounded sample of the timed workload.

Every roofline entry gives the kernel's bandwidth two ways: `achieved` =
the per-unit bytes of the method's cost model (a gate layer reads and writes
the X and Z columns of every qubit it touches, plus the sign column; a
random measurement reads and writes X and Z of every row word; a
deterministic one reads n columns of the stabilizer half twice) times the
units one launch processes, over the launch's average duration (HIP events
on the library's stream); and `achieved_moved` = the bytes the launch
actually streams (counted by the library) over the same duration. The two
differ because a pass fuses about 2.4 generator layers and a blocked pass
applies up to 32 measurements, so `frac` (cost-model bytes) can exceed 1;
`frac_moved` is the physical fraction of HBM peak.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD public specification
HBM_SUMMARY = "hbm_counters_n180000_bench.md"  # profiles/ summary of FETCH_SIZE / WRITE_SIZE on this workload
HBM_SUMMARY_IR = "hbm_counters_n180000_inject_rows.md"  # the same for the CX-injection and row-layout sections
METRIC = "gates/s & measurements/s at n=180k (HBM % of peak); batched vs plain shots/s"


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def build_ops(cfg, layers: int):
    from workload import OP_DTYPE, iter_circuit
    parts = []
    t0 = time.time()
    for k, (kind, arr) in enumerate(iter_circuit(cfg, depth=layers, final_measure=False)):
        parts.append(arr)
        if (k + 1) % 200 == 0:
            log(f"generated {k + 1}/{layers} layers ({time.time() - t0:.1f} s)")
    gates = np.concatenate(parts) if parts else np.empty(0, dtype=OP_DTYPE)
    return gates, parts


def meas_ops(qubits):
    q = np.asarray(qubits, dtype=np.uint32)
    return np.stack([np.full(q.size, 15, np.uint32), q, np.zeros(q.size, np.uint32)], 1)


def layer_model_bytes(parts, n: int, L: int) -> int:
    """Cost-model bytes of the gate layers: per layer, 4 column reads and
    writes (X and Z) of every distinct qubit it touches plus the sign column
    read and written, a column being L words of 8 bytes."""
    C = 8 * L
    total = 0
    for arr in parts:
        two = arr["type"] >= 7
        touched = np.unique(np.concatenate([arr["q0"], arr["q1"][two]]))
        total += touched.size * 4 * C + 2 * C
    return total


def roof(name, ms, launches, model_bytes, moved_bytes, unit_desc, traffic=None):
    """A roofline entry from the total kernel time and launches (all timed
    steps) and the bytes of those launches."""
    launches = max(launches, 1)
    avg_s = ms / launches * 1e-3
    per_model = model_bytes / launches
    per_moved = moved_bytes / launches
    ach = per_model / avg_s / 1e9 if avg_s > 0 else 0.0
    mov = per_moved / avg_s / 1e9 if avg_s > 0 else 0.0
    return {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "achieved_moved": round(mov, 1), "frac_moved": round(mov / HBM_PEAK_GBS, 4),
            "bytes_per_launch": int(per_model), "moved_bytes_per_launch": int(per_moved),
            "traffic_over_moved": round(traffic / per_moved, 3) if traffic and per_moved else None,
            "model_unit": unit_desc, "avg_launch_ms": round(ms / launches, 4), "launches": int(launches)}


def cpu_baseline(cfg, layer_parts, seconds: float, nrows: int = 64):
    """The oracle evolving a sample of rows (rows evolve independently under
    gates) through as many layers as fit in about `seconds`; scaled to gates/s
    of the whole 2n-row tableau."""
    from oracle import oracle as orc
    n = cfg.n
    rows = list(range(n, n + nrows // 2)) + list(range(0, nrows // 2))
    sub = orc.Tableau(n, rows=rows)
    t0 = time.time()
    gates_done = 0
    layers_done = 0
    for arr in layer_parts:
        sub.run(arr)
        gates_done += int(arr.size)
        layers_done += 1
        if time.time() - t0 > seconds:
            break
    dt = time.time() - t0
    row_gate_rate = gates_done * nrows / dt
    return {
        "value": row_gate_rate / (2 * n),
        "unit": "gates/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": f"{nrows} of the {2 * n} tableau rows through the first {layers_done} layers "
                  f"({gates_done} gates, {dt:.1f} s); rate scaled by {nrows}/{2 * n}",
    }


# ---------------------------------------------------------------- the 180,000-qubit circuit
def main_steps(args, sq, sqb, profsum, cfg, pg, pm, parts, L):
    import torch
    n = cfg.n
    stream = torch.cuda.current_stream()
    t = sq.Tableau(n, stream=stream)
    out_bits = torch.zeros(max(args.meas, 1), dtype=torch.uint8, device="cuda")
    out_rand = torch.zeros(max(args.meas, 1), dtype=torch.uint8, device="cuda")

    def step(record=None):
        t.reset()
        if record:
            record[0].record(stream)
        t.run(pg, cfg.seed, 0, 0, out_bits.data_ptr(), out_rand.data_ptr())
        if record:
            record[1].record(stream)
        if pm is not None:
            t.run(pm, cfg.seed, 0, 0, out_bits.data_ptr(), out_rand.data_ptr())
        if record:
            record[2].record(stream)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    t.profile_reset()
    t.profile(True)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
        if k + 1 < args.steps:
            torch.cuda.synchronize()
            log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t.profile(False)
    log(f"timed {args.steps} steps in {wall:.2f} s")
    st1 = t.measure_stats()  # each step starts from reset, which clears the counters: one step
    gate_ms = sum(e[0].elapsed_time(e[1]) for e in events)
    meas_ms = sum(e[1].elapsed_time(e[2]) for e in events)
    assert t.error_flags() == 0
    kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    layer_ms, layer_n = kern["layer"]
    assert layer_n > 0
    C = 8 * L
    model_gate = layer_model_bytes(parts, n, L)
    traffic = profsum.traffic_per_dispatch("k_layer", HBM_SUMMARY)
    roofs = [roof("k_layer", layer_ms, layer_n, model_gate * args.steps, pg.gate_bytes * args.steps,
                  f"gate layer: 4 C per distinct qubit touched + 2 C (C = {C} B); "
                  f"{len(parts) / max(pg.num_passes, 1):.2f} layers per launch", traffic)]
    if kern["block_pass"][1]:
        nb = max(st1.blocks, 1)
        roofs.append(roof("k_blk_pass", *kern["block_pass"], st1.n_random * 4 * n * C * args.steps,
                          st1.block_bytes * args.steps,
                          f"random measurement: 4 n C = {4 * n * C / 1e9:.1f} GB (every row word read and "
                          f"written in X and Z); {st1.n_random / nb:.1f} measurements per launch",
                          profsum.traffic_per_dispatch("k_blk_pass", HBM_SUMMARY)))
    roofs.sort(key=lambda r: -r["avg_launch_ms"] * r["launches"])
    res = {
        "value": pg.num_gates * args.steps / (gate_ms * 1e-3),
        "ms_per_step": wall * 1e3 / args.steps,
        "measurements_per_s": args.meas * args.steps / (meas_ms * 1e-3) if args.meas else None,
        "gate_phase_ms_per_step": gate_ms / args.steps,
        "meas_phase_ms_per_step": meas_ms / args.steps,
        "random_measurements_per_step": int(st1.n_random),
        "measurement_blocks_per_step": int(st1.blocks),
        "gate_model_bytes_per_step": int(model_gate),
        "gate_moved_bytes_per_step": int(pg.gate_bytes),
        "roofline": roofs[0],
        "roofline_other": roofs[1:],
        "kernel_ms": {k: round(v[0], 3) for k, v in kern.items()},
        "kernel_launches": {k: v[1] for k, v in kern.items()},
    }
    t.last_bits = out_bits
    return t, res


def full_sweep(t, cfg, pg, sqb, L):
    """All n final measurements once (after the gates), then the first 1000
    again (deterministic)."""
    import torch
    n = cfg.n
    C = 8 * L
    stream = torch.cuda.current_stream()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    rnd = torch.zeros(n, dtype=torch.uint8, device="cuda")
    sweep = sqb.Program(n, meas_ops(np.arange(n)))
    t.reset()
    t.run(pg, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    torch.cuda.synchronize()
    log("full sweep: gates done; measuring all qubits")
    t.profile_reset()
    t.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t.run(sweep, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    t.profile(False)
    ms = e0.elapsed_time(e1)
    st = t.measure_stats()
    kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    assert t.error_flags() == 0
    sweep.close()
    log(f"full sweep: {n} measurements in {ms / 1e3:.2f} s")
    res = {
        "workload": f"all {n} final Z measurements of the n={n} depth-1000 circuit after its gates",
        "measurements": n, "seconds": ms / 1e3, "measurements_per_s": n / (ms * 1e-3),
        "random": int(st.n_random), "deterministic": int(st.n_det), "blocks": int(st.blocks),
        "roofline": roof("k_blk_pass", *kern["block_pass"], st.n_random * 4 * n * C, st.block_bytes,
                         f"random measurement: 4 n C = {4 * n * C / 1e9:.1f} GB; "
                         f"{st.n_random / max(st.blocks, 1):.1f} measurements per launch"),
        "kernel_ms": {k: round(v[0], 1) for k, v in kern.items()},
    }
    # deterministic: the first 1000 qubits again
    k = min(1000, n)
    again = sqb.Program(n, meas_ops(np.arange(k)))
    out2 = torch.zeros(k, dtype=torch.uint8, device="cuda")
    rnd2 = torch.zeros(k, dtype=torch.uint8, device="cuda")
    st0 = t.measure_stats()
    t.profile_reset()
    t.profile(True)
    e0.record(stream)
    t.run(again, cfg.seed, 0, n, out2.data_ptr(), rnd2.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    t.profile(False)
    dms = e0.elapsed_time(e1)
    st1 = t.measure_stats()
    kern2 = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    same = bool(torch.equal(out2, out[:k])) and not bool(rnd2.any())
    assert same and t.error_flags() == 0, "re-measured outcomes differ or were random"
    again.close()
    ndet = st1.n_det - st0.n_det
    det_moved = st1.det_bytes - st0.det_bytes
    log(f"deterministic: {k} measurements in {dms / 1e3:.2f} s")
    det = {
        "workload": f"qubits 0..{k - 1} measured again after the full sweep (all deterministic)",
        "measurements": k, "seconds": dms / 1e3, "measurements_per_s": k / (dms * 1e-3),
        "deterministic": int(ndet), "outcomes_repeat": same,
        "roofline": roof("k_post (deterministic)", *kern2["post"], ndet * n * C, det_moved,
                         f"deterministic measurement: n C = {n * C / 1e9:.1f} GB (x and z of the stabilizer "
                         f"half of every column read once)"),
        "kernel_ms": {kk: round(v[0], 1) for kk, v in kern2.items()},
    }
    return res, det


def inject_collapse(sq, sqb, cfg, pg, L, ref_bits, meas: int):
    """The paper's own collapse (CX injection on the operator tableau) on the
    same circuit: the gate passes in that mode (image signs), then the first
    `meas` final measurements, then the same qubits again (deterministic).
    Outcomes must equal the rowsum collapse's (`ref_bits`, same coins)."""
    import torch
    from paper_2603_14641_amd import profsum
    n = cfg.n
    C = 8 * L
    stream = torch.cuda.current_stream()
    t = sq.Tableau(n, stream=stream, collapse=sqb.COLLAPSE_INJECT)
    out = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    rnd = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    pm = sqb.Program(n, meas_ops(np.arange(meas)))
    e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    t.run(pg, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())  # first run: kernel by kernel, graphs captured next
    torch.cuda.synchronize()
    t.reset()
    t.profile_reset()
    t.profile(True)
    e[0].record(stream)
    t.run(pg, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    e[1].record(stream)
    t.run(pm, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    e[2].record(stream)
    torch.cuda.synchronize()
    st = t.measure_stats()
    out2 = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    rnd2 = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    e[3].record(stream)
    t.run(pm, cfg.seed + 1, 1, meas, out2.data_ptr(), rnd2.data_ptr())
    e[4].record(stream)
    torch.cuda.synchronize()
    t.profile(False)
    kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    assert t.error_flags() == 0
    same = bool(torch.equal(out, ref_bits[:meas].to(out.device)))
    repeat = bool(torch.equal(out2, out)) and not bool(rnd2.any())
    assert same and repeat, "CX-injection outcomes differ from the rowsum collapse's, or did not repeat"
    gms, mms, dms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[3].elapsed_time(e[4])
    ia_ms, ia_n = kern["inject_apply"]
    nr = int(st.n_random)
    res = {
        "workload": f"n={n} depth-1000 circuit on the operator tableau: gate passes with image signs, then the "
                    f"first {meas} final Z measurements (CX-injection collapse), then the same {meas} again",
        "gates_per_s": pg.num_gates / (gms * 1e-3), "gate_phase_ms": gms,
        "measurements_per_s": meas / (mms * 1e-3), "random": nr,
        "deterministic_measurements_per_s": meas / (dms * 1e-3),
        "outcomes_equal_rowsum_collapse": same, "remeasured_deterministic": repeat,
        "roofline_gates": roof("k_layer_op", *kern["layer"], pg.gate_bytes * kern["layer"][1] // max(pg.num_passes, 1),
                               pg.gate_bytes * kern["layer"][1] // max(pg.num_passes, 1),
                               "bytes the pass moves (column reads + changed-column writes), same plans as k_layer",
                               profsum.traffic_per_dispatch("k_layer_op", HBM_SUMMARY_IR)),
        "roofline": roof("k_inj_apply", ia_ms, ia_n, st.inject_bytes, st.inject_bytes,
                         f"per column: read x, z of the destabilizer word of every target word and read+write "
                         f"the stabilizer word where the pivot has x (z); random measurement with B_word = "
                         f"{4 * n * C / 1e9:.1f} GB for comparison",
                         profsum.traffic_per_dispatch("k_inj_apply", HBM_SUMMARY_IR)),
        "kernel_ms": {k: round(v[0], 2) for k, v in kern.items() if v[1]},
        "kernel_launches": {k: v[1] for k, v in kern.items() if v[1]},
    }
    log(f"inject collapse: gates {res['gates_per_s']:.3g}/s, {meas} measurements {res['measurements_per_s']:.3g}/s")
    pm.close()
    t.close()
    return res


def row_layout(sq, sqb, cfg, pg, L, ref_bits, meas: int):
    """The dual layout: after the gates, transpose to rows, the first `meas`
    final measurements one at a time on whole rows, the same qubits again
    (deterministic), transpose back, the same qubits again in columns
    (deterministic, column kernels); then, from the same post-gate state,
    the first `meas` measurements one at a time in columns (no blocks): the
    row-granular and word-granular costs of the same measurements."""
    import torch
    from paper_2603_14641_amd import profsum
    n = cfg.n
    C = 8 * L
    stream = torch.cuda.current_stream()
    t = sq.Tableau(n, stream=stream)
    out = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    rnd = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    out2, rnd2 = torch.zeros_like(out), torch.zeros_like(rnd)
    out3, rnd3 = torch.zeros_like(out), torch.zeros_like(rnd)
    pm = sqb.Program(n, meas_ops(np.arange(meas)))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    t.run(pg, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    torch.cuda.synchronize()
    t.profile_reset()
    t.profile(True)
    ev[0].record(stream)
    t.set_layout(sqb.LAYOUT_ROWS)
    ev[1].record(stream)
    t.run(pm, cfg.seed, 0, 0, out.data_ptr(), rnd.data_ptr())
    ev[2].record(stream)
    torch.cuda.synchronize()
    st_r = t.measure_stats()
    ev[3].record(stream)
    t.run(pm, cfg.seed + 1, 1, meas, out2.data_ptr(), rnd2.data_ptr())
    ev[4].record(stream)
    torch.cuda.synchronize()
    st_d = t.measure_stats()
    ev[5].record(stream)
    t.set_layout(sqb.LAYOUT_COLUMNS)
    ev[6].record(stream)
    t.run(pm, cfg.seed + 2, 2, 2 * meas, out3.data_ptr(), rnd3.data_ptr())
    ev[7].record(stream)
    torch.cuda.synchronize()
    t.profile(False)
    st_c = t.measure_stats()
    kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    assert t.error_flags() == 0
    same = bool(torch.equal(out, ref_bits[:meas].to(out.device)))
    repeat = bool(torch.equal(out2, out)) and bool(torch.equal(out3, out)) and not bool(rnd2.any() or rnd3.any())
    assert same and repeat, "row-layout outcomes differ from the column layout's, or did not repeat"
    # the same measurements one at a time in columns, from the same state
    t.reset()
    t.run(pg, cfg.seed, 0, 0, out2.data_ptr(), rnd2.data_ptr())
    t.set_tuning(meas_block=1)
    torch.cuda.synchronize()
    st0 = t.measure_stats()
    t.profile_reset()
    t.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t.run(pm, cfg.seed, 0, 0, out3.data_ptr(), rnd3.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    t.profile(False)
    st1 = t.measure_stats()
    kc = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    assert bool(torch.equal(out3, out)) and t.error_flags() == 0
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(7)]
    det_rows_moved = st_d.det_bytes - st_r.det_bytes
    det_cols_moved = st_c.det_bytes - st_d.det_bytes
    nr = int(st_r.n_random)
    tr_bytes = 2 * 2 * 64 * sqb.layout(n)["K"] * 2 * sqb.layout(n)["K"] * 8  # X and Z, read and written
    res = {
        "workload": f"n={n} depth-1000 circuit: transpose to rows, the first {meas} final measurements one at a "
                    f"time on rows, the same qubits again (deterministic) on rows, transpose back, again on "
                    f"columns; then from the same post-gate state the {meas} measurements one at a time on columns",
        "transpose_ms": [round(ms[0], 3), round(ms[5], 3)],
        "measurements_per_s_rows": meas / (ms[1] * 1e-3), "random": nr,
        "measurements_per_s_columns_single": meas / (e0.elapsed_time(e1) * 1e-3),
        "deterministic_per_s_rows": meas / (ms[3] * 1e-3),
        "deterministic_per_s_columns": meas / (ms[6] * 1e-3),
        "rowsum_bytes_per_measurement_rows": int(st_r.rowsum_bytes / max(nr, 1)),
        "rowsum_bytes_per_measurement_columns": int((st1.rowsum_bytes - st0.rowsum_bytes) / max(nr, 1)),
        "det_bytes_per_measurement_rows": int(det_rows_moved / meas),
        "det_bytes_per_measurement_columns": int(det_cols_moved / meas),
        "outcomes_equal_blocked_columns": same,
        "roofline_transpose": roof("k_transpose", *kern["transpose"], tr_bytes * kern["transpose"][1],
                                   tr_bytes * kern["transpose"][1],
                                   "X and Z, both halves, every word read and written once",
                                   profsum.traffic_per_dispatch("k_transpose", HBM_SUMMARY_IR)),
        "roofline": roof("k_row_rowsum", *kern["row_rowsum"], nr * n * 4 * (L // 2) * 8, st_r.rowsum_bytes,
                         f"random measurement, row granular: the rows with x_q = 1 (about n of 2n) read and "
                         f"written in x and z; cost model n rows x 4 x {L // 2} words; B_word = "
                         f"{4 * n * C / 1e9:.1f} GB for comparison",
                         profsum.traffic_per_dispatch("k_row_rowsum<true>", HBM_SUMMARY_IR)),
        "roofline_det": roof("k_row_det", *kern["row_det"], det_rows_moved, det_rows_moved,
                             "deterministic: x and z of every stabilizer row in the product, read once"),
        "roofline_columns_single": roof("k_rowsum", *kc["rowsum"], nr * 4 * n * C,
                                        st1.rowsum_bytes - st0.rowsum_bytes,
                                        f"random measurement, word granular: B_word = {4 * n * C / 1e9:.1f} GB"),
        "kernel_ms": {k: round(v[0], 2) for k, v in kern.items() if v[1]},
        "kernel_ms_columns_single": {k: round(v[0], 2) for k, v in kc.items() if v[1]},
    }
    log(f"row layout: transposes {ms[0]:.1f} / {ms[5]:.1f} ms, {meas} measurements "
        f"{res['measurements_per_s_rows']:.3g}/s on rows vs {res['measurements_per_s_columns_single']:.3g}/s "
        f"single on columns; deterministic {res['deterministic_per_s_rows']:.3g}/s rows vs "
        f"{res['deterministic_per_s_columns']:.3g}/s columns")
    pm.close()
    t.close()
    return res


# ---------------------------------------------------------------- the batched/served mix
def dense_deterministic(sq, sqb, meas: int, layers: int = 64):
    """Deterministic measurements whose product spans about n/2 stabilizers:
    n = 180,000 after `layers` layers of basis-state-preserving gates
    (workload.basis_circuit: CX, CZ, SWAP, S, SDG, X, Y, Z), then qubits
    0..meas-1, every one deterministic with the circuit's planted outcome.
    Here the set A of the CHP deterministic case is dense, so each
    measurement reads x and z of nearly every stabilizer word of every
    column, the n C bytes of the cost model. Timed in columns (k_pivot +
    k_post), then the same qubits again on rows (k_row_det)."""
    import torch
    from workload import basis_circuit
    n = 180000
    L = sqb.layout(n)["L"]
    C = 8 * L
    log(f"dense deterministic: generating {layers} basis-preserving layers")
    ops, planted = basis_circuit(n, layers, seed=21)
    gates = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
    pg = sq.Program(n, gates)
    pm = sq.Program(n, meas_ops(np.arange(meas)))
    t = sq.Tableau(n)
    stream = torch.cuda.current_stream()
    out = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    rnd = torch.zeros(meas, dtype=torch.uint8, device="cuda")
    t.run(pg, 1, 0, 0, 0, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(tag):
        st0 = t.measure_stats()
        t.profile_reset()
        t.profile(True)
        e0.record(stream)
        t.run(pm, 1, 0, 0, out.data_ptr(), rnd.data_ptr())
        e1.record(stream)
        torch.cuda.synchronize()
        t.profile(False)
        st1 = t.measure_stats()
        ok = bool(np.array_equal(out.cpu().numpy(), planted[:meas])) and not bool(rnd.any())
        assert ok and t.error_flags() == 0, f"dense deterministic ({tag}): outcomes differ from the planted bits"
        kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
        return e0.elapsed_time(e1), st1.n_det - st0.n_det, st1.det_bytes - st0.det_bytes, kern

    ms_c, nd_c, moved_c, kc = timed("columns")
    t.set_layout(sqb.LAYOUT_ROWS)
    torch.cuda.synchronize()
    ms_r, nd_r, moved_r, kr = timed("rows")
    t.close()
    pg.close()
    pm.close()
    log(f"dense deterministic: {meas / (ms_c * 1e-3):.3g}/s columns, {meas / (ms_r * 1e-3):.3g}/s rows")
    return {
        "workload": f"n={n}: {layers} layers of CX/CZ/SWAP/S/SDG/X/Y/Z from |0...0> ({gates.shape[0]} gates), "
                    f"then qubits 0..{meas - 1} (all deterministic, dense products, planted outcomes)",
        "measurements": meas, "outcomes_equal_planted": True,
        "measurements_per_s_columns": meas / (ms_c * 1e-3),
        "measurements_per_s_rows": meas / (ms_r * 1e-3),
        "avg_rows_in_product": round(moved_r / max(nd_r, 1) / (16 * (L // 2)), 1),
        "roofline": roof("k_post (deterministic, dense A)", *kc["post"], nd_c * n * C, moved_c,
                         f"deterministic measurement: n C = {n * C / 1e9:.1f} GB (x and z of the stabilizer half "
                         f"of every column read once); moved = the nonzero words of A in every column"),
        "roofline_rows": roof("k_row_det", *kr["row_det"], moved_r, moved_r,
                              "x and z of every stabilizer row in the product, read once"),
        "kernel_ms_columns": {k: round(v[0], 2) for k, v in kc.items() if v[1]},
        "kernel_ms_rows": {k: round(v[0], 2) for k, v in kr.items() if v[1]},
    }


def served_mix(nreq: int, budget_bytes: int, session_requests: int):
    import torch
    import paper_2603_14641_amd as sq
    from paper_2603_14641_amd import autotune, serving
    from workload import circuit_ops, served_requests

    log(f"served mix: drawing {nreq} circuits")
    base = served_requests()[:nreq]
    reqs = []
    for r in base:
        ops = circuit_ops(r.config(), final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(dict(n=r.n, ops=ops, qubits=np.arange(r.n, dtype=np.uint32), shots=r.shots, seed=r.coin_seed))
    shots = sum(r["shots"] for r in reqs)
    log(f"served mix: {nreq} requests, {shots} shots; plain path")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_out = []
    for r in reqs:
        t = sq.Tableau(r["n"])
        t.apply_gates(r["ops"])
        plain_out.append(t.sample(r["qubits"], r["shots"], seed=r["seed"]))
        t.close()
    plain_s = time.perf_counter() - t0
    log(f"plain {plain_s:.2f} s; Pauli frames")
    progs = [sq.Program(r["n"], np.concatenate([r["ops"], meas_ops(r["qubits"])])) for r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, pg in zip(reqs, progs):
        pg.frame_sample(r["shots"], seed=r["seed"])
    frame_s = time.perf_counter() - t0
    for pg in progs:
        pg.close()
    log(f"frames {frame_s:.2f} s; tuning the batch schedule")
    # the autotuner picks (block, persistent-launch size limit, streams) on a
    # stratified sample of the requests; not part of any timed region
    cands = [dict(block=256, max_batch_n=m, streams=st) for m in (256, 512, 1024, 2048) for st in (4, 8)]
    tuned = autotune.tune_batch(reqs, sample=12, candidates=cands, use_cache=False)
    kw = {k: int(tuned[k]) for k in ("block", "max_batch_n", "streams")}
    log(f"schedule {kw}; batched")
    t0 = time.perf_counter()
    batch_out = sq.batch_sample(reqs, **kw)
    batch_s = time.perf_counter() - t0
    same = all(np.array_equal(a, b) for a, b in zip(plain_out, batch_out))
    res = {
        "workload": f"all {nreq} batched/served requests (n log-uniform 16..16384, depth 10..500, 1..4096 shots, "
                    f"final all-qubit Z measurement)",
        "requests": nreq, "shots": shots,
        "plain_s": plain_s, "plain_shots_per_s": shots / plain_s,
        "batched_s": batch_s, "batched_shots_per_s": shots / batch_s,
        "batched_vs_plain": plain_s / batch_s,
        "frame_s": frame_s, "frame_shots_per_s": shots / frame_s,
        "frame_note": "Pauli frames: reference CHP run plus frames per request, same distribution, other bits",
        "batch_schedule": dict(kw, tuned_on_requests=int(tuned["sample"])),
        "served": [],
    }
    # the serving loop with Poisson arrivals: at 0.8 x the plain path's request
    # rate (latency), and at 4 x (arrivals outpace service, so batches form)
    for mult in (0.8, 4.0):
        rate = mult * nreq / plain_s
        rng = np.random.Generator(np.random.PCG64(4))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
        sreqs = [serving.CircuitRequest(n=r["n"], ops=r["ops"], qubits=r["qubits"], shots=r["shots"], seed=r["seed"],
                                        arrival=float(a)) for r, a in zip(reqs, arrivals)]
        log(f"serving at {rate:.2f} requests/s")
        st = serving.Server(budget_bytes=budget_bytes, workers=2, batch_kwargs=kw).run(sreqs)
        ok = all(r.ok for r in sreqs) and all(np.array_equal(r.result, b) for r, b in zip(sreqs, batch_out))
        same = same and ok
        log(f"served makespan {st.makespan_s:.2f} s, p50 {st.latency_p50_s:.3f} s, p99 {st.latency_p99_s:.3f} s, "
            f"mean batch {st.mean_batch:.2f}")
        res["served"].append({"arrival_rate_per_s": rate, "rate_over_plain": mult, "shots_per_s": st.shots_per_s,
                              "makespan_s": st.makespan_s, "latency_p50_s": st.latency_p50_s,
                              "latency_p99_s": st.latency_p99_s, "batches": st.batches,
                              "mean_batch": st.mean_batch, "max_in_flight_bytes": st.max_in_flight_bytes,
                              "budget_bytes": budget_bytes, "completed": st.completed})
    if session_requests > 0:
        res["sessions"] = sessions_run(reqs, session_requests, budget_bytes)
        same = same and res["sessions"]["served_equals_alone"]
    res["outputs_identical_across_paths"] = bool(same)
    return res


def served_kernels_single_thread(nreq: int):
    """The kernels of the batched/served paths driven from one host thread
    (for a kernel trace): the plain per-circuit sampling of every request
    (gates, symbolic sweep, per-shot evaluation), the Pauli-frame path, and
    the persistent batched launch on the requests it takes (n <= 1024, so no
    worker threads start)."""
    import torch
    import paper_2603_14641_amd as sq
    from workload import circuit_ops, served_requests

    reqs = []
    for r in served_requests()[:nreq]:
        ops = circuit_ops(r.config(), final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(dict(n=r.n, ops=ops, qubits=np.arange(r.n, dtype=np.uint32), shots=r.shots, seed=r.coin_seed))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        t = sq.Tableau(r["n"])
        t.apply_gates(r["ops"])
        t.sample(r["qubits"], r["shots"], seed=r["seed"])
        t.close()
    plain_s = time.perf_counter() - t0
    small = [r for r in reqs if r["n"] <= 1024]
    t0 = time.perf_counter()
    sq.batch_sample(small, block=256, max_batch_n=1024, streams=1)
    batch_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    for r in reqs[:64]:
        pg = sq.Program(r["n"], np.concatenate([r["ops"], meas_ops(r["qubits"])]))
        pg.frame_sample(r["shots"], seed=r["seed"])
        pg.close()
    frame_s = time.perf_counter() - t0
    log(f"single-thread served kernels: plain {plain_s:.2f} s, batched ({len(small)} small) {batch_s:.2f} s, "
        f"frames (64) {frame_s:.2f} s")
    return {"requests": nreq, "plain_s": plain_s, "batched_small_requests": len(small), "batched_s": batch_s,
            "frame_requests": 64, "frame_s": frame_s}


def sessions_run(reqs, nsample: int, budget_bytes: int):
    """Resident tableaux: 16 of the mix's circuits opened as sessions, then
    `nsample` sampling requests (Poisson, each on a random session, shots
    log-uniform 1..4096) served with per-session batching (queued requests
    on one session share one measurement sweep), against the same requests
    run one by one on the same resident tableaux."""
    import torch
    import paper_2603_14641_amd as sq
    from paper_2603_14641_amd import serving

    pick = [r for r in reqs if 1024 <= r["n"] <= 8192][:16]
    rng = np.random.Generator(np.random.PCG64(44))
    draws = [(int(rng.integers(len(pick))), int(round(np.exp(rng.uniform(0, np.log(4096))))), int(rng.integers(1 << 30)))
             for _ in range(nsample)]
    # alone: every request by itself on the resident tableau
    tabs = []
    for r in pick:
        t = sq.Tableau(r["n"])
        t.apply_gates(r["ops"])
        tabs.append(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [tabs[k].sample(pick[k]["qubits"], s, seed=seed) for k, s, seed in draws]
    alone_s = time.perf_counter() - t0
    for t in tabs:
        t.close()
    shots = sum(s for _, s, _ in draws)
    log(f"sessions: {nsample} sampling requests alone in {alone_s:.2f} s; serving")
    # served: open the sessions, then the requests at 2 x the alone rate
    rate = 2.0 * nsample / alone_s
    arr = np.cumsum(rng.exponential(1.0 / rate, nsample))
    srv = serving.Server(budget_bytes=budget_bytes, workers=2)
    srv.start()
    opens = [srv.submit(serving.OpenSession(session=f"s{k}", n=r["n"], ops=r["ops"])) for k, r in enumerate(pick)]
    while any(o.state not in ("done", "failed") for o in opens):
        time.sleep(0.01)
    base = srv._now()
    sreqs = [serving.SampleRequest(session=f"s{k}", qubits=pick[k]["qubits"], shots=s, seed=seed, arrival=base + a)
             for (k, s, seed), a in zip(draws, arr)]
    for r in sreqs:
        delay = r.arrival - srv._now()
        if delay > 0:
            time.sleep(delay)
        srv.submit(r)
    for k in range(len(pick)):
        srv.submit(serving.CloseSession(session=f"s{k}"))
    srv.stop()
    st = srv.stats(sreqs)
    equal = all(r.ok for r in sreqs) and all(np.array_equal(r.result, a) for r, a in zip(sreqs, alone))
    sweeps = srv.batch_sizes("sample")
    log(f"sessions served: {st.shots_per_s:.3g} shots/s vs alone {shots / alone_s:.3g}, "
        f"{len(sweeps)} sweeps for {nsample} requests")
    return {"sessions": len(pick), "session_n": [r["n"] for r in pick], "sampling_requests": nsample, "shots": shots,
            "alone_s": alone_s, "alone_shots_per_s": shots / alone_s, "arrival_rate_per_s": rate,
            "served_shots_per_s": st.shots_per_s, "served_makespan_s": st.makespan_s,
            "latency_p50_s": st.latency_p50_s, "latency_p99_s": st.latency_p99_s,
            "requests_per_sweep_mean": float(np.mean(sweeps)) if sweeps else 0.0, "sweeps": len(sweeps),
            "served_equals_alone": bool(equal)}


def stream_ceiling():
    """Measured HBM ceiling of plain torch kernels on 4 GiB buffers (GB/s)."""
    import torch
    n = 1 << 29
    a = torch.ones(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)

    def tm(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    nb = 8 * n
    res = {"copy_read_write": 2 * nb / tm(lambda: b.copy_(a)) / 1e6,
           "read_only": nb / tm(lambda: a.sum()) / 1e6,
           "write_only": nb / tm(lambda: b.fill_(7)) / 1e6}
    del a, b
    torch.cuda.empty_cache()
    return {k: round(v, 1) for k, v in res.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--layers", type=int, default=1000)
    ap.add_argument("--meas", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-sweep", action="store_true", help="skip the full 180,000-measurement sweep")
    ap.add_argument("--served-requests", type=int, default=512,
                    help="requests of the batched/served mix to run (0 skips that part)")
    ap.add_argument("--session-requests", type=int, default=96,
                    help="sampling requests against resident tableaux (0 skips)")
    ap.add_argument("--inject-meas", type=int, default=256,
                    help="final measurements run with the CX-injection collapse (0 skips that part)")
    ap.add_argument("--row-meas", type=int, default=256,
                    help="final measurements run one at a time in the row layout (0 skips that part)")
    ap.add_argument("--det-meas", type=int, default=256,
                    help="deterministic measurements with dense products (0 skips that part)")
    ap.add_argument("--served-single-thread", action="store_true",
                    help="run only the batched/served paths' kernels from one host thread (for kernel traces)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-sharded design is not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_14641_amd as sq
    from paper_2603_14641_amd import binding as sqb
    from paper_2603_14641_amd import profsum
    from workload import CONFIGS

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sq.load()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 copies of 1 GiB done")
    cfg = CONFIGS[4]
    n = cfg.n
    L = sqb.layout(n)["L"]
    log(f"generating {args.layers} layers of n={n}")
    gates, parts = build_ops(cfg, args.layers)
    log(f"{gates.size} gates; compiling")
    pg = sq.Program(n, gates)
    pm = sq.Program(n, meas_ops(np.arange(args.meas))) if args.meas else None
    log(f"{pg.num_passes} gate passes, {pg.gate_bytes / 1e9:.1f} GB moved per step")
    t, res = main_steps(args, sq, sqb, profsum, cfg, pg, pm, parts, L)
    result = {
        "metric": METRIC,
        "value": res.pop("value"),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"n=180000 generator circuit (seed {cfg.seed}): {args.layers} layers + first "
                        f"{args.meas} of the final 180000 Z-measurements per step",
            "n": n, "layers": args.layers, "gates_per_step": int(pg.num_gates), "passes_per_step": pg.num_passes,
            "measurements_per_step": args.meas,
        },
    }
    result.update(res)
    res_bits = None
    if max(args.inject_meas, args.row_meas) and args.meas >= max(args.inject_meas, args.row_meas):
        res_bits = t.last_bits.clone()
    if not args.no_full_sweep and args.layers == 1000:
        result["full_sweep"], result["deterministic"] = full_sweep(t, cfg, pg, sqb, L)
    t.close()
    torch.cuda.empty_cache()
    if res_bits is not None and args.inject_meas:
        result["inject_collapse"] = inject_collapse(sq, sqb, cfg, pg, L, res_bits, args.inject_meas)
        torch.cuda.empty_cache()
    if res_bits is not None and args.row_meas:
        result["row_layout"] = row_layout(sq, sqb, cfg, pg, L, res_bits, args.row_meas)
    pg.close()
    if pm is not None:
        pm.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.det_meas:
        result["dense_deterministic"] = dense_deterministic(sq, sqb, args.det_meas)
        torch.cuda.empty_cache()
    result["hbm_stream_ceiling_gbs"] = stream_ceiling()
    if args.served_requests > 0 and args.served_single_thread:
        result["served_single_thread"] = served_kernels_single_thread(args.served_requests)
    elif args.served_requests > 0:
        result["batched_served"] = served_mix(args.served_requests, 8 << 30, args.session_requests)
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(cfg, parts, args.cpu_seconds)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
