#!/usr/bin/env python3
"""Throughput of the stabilizer-tableau hot path on one MI355X.

Workload (the 180,000-qubit, depth-1000 generator circuit): each step resets
the tableau to |0...0>, applies all 1000 random layers (about 198 million
non-identity gates, fused into passes) and then performs the first M Z
measurements (qubits 0..M-1 in order) of the circuit's final all-qubit
measurement. Inputs (the compiled gate passes) are resident in HBM before
timing starts; outcomes stay on the device.

Prints one JSON line: gates/s of the gate phase as `value`, measurements/s of
the measurement phase, the roofline of the dominant kernel (algorithmic bytes
per launch / average launch duration, both measured here with HIP events on
the library's stream) and the CPU oracle timed on a bounded sample.
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


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def build_ops(cfg, layers: int, nmeas: int):
    from workload import OP_DTYPE, OP_MEASURE, iter_circuit
    parts = []
    t0 = time.time()
    for k, (kind, arr) in enumerate(iter_circuit(cfg, depth=layers, final_measure=False)):
        parts.append(arr)
        if (k + 1) % 200 == 0:
            log(f"generated {k + 1}/{layers} layers ({time.time() - t0:.1f} s)")
    gates = np.concatenate(parts) if parts else np.empty(0, dtype=OP_DTYPE)
    meas = np.empty(nmeas, dtype=OP_DTYPE)
    meas["type"] = OP_MEASURE
    meas["q0"] = np.arange(nmeas, dtype=np.uint32)
    meas["q1"] = 0
    return gates, meas, parts


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


def served_mix(nreq: int, budget_bytes: int):
    """The batched/served workload on its first `nreq` requests: the plain
    per-circuit path (one tableau at a time: create, gates, sq_sample), one
    batched call over all of them, and the serving loop with Poisson arrivals
    at 0.8 x the plain path's request rate. Returns shots/s of each and the
    served p50/p99 latency."""
    import torch
    import paper_2603_14641_amd as sq
    from paper_2603_14641_amd import autotune, serving
    from workload import circuit_ops, served_requests

    base = served_requests()[:nreq]
    reqs = []
    for r in base:
        cfg = r.config()
        ops = circuit_ops(cfg, final_measure=False)
        ops = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        reqs.append(dict(n=cfg.n, ops=ops, qubits=np.arange(cfg.n, dtype=np.uint32), shots=r.shots,
                         seed=r.coin_seed))
    shots = sum(r["shots"] for r in reqs)
    log(f"served mix: {nreq} requests, {shots} shots; plain path")
    t0 = time.perf_counter()
    plain_out = []
    for r in reqs:
        t = sq.Tableau(r["n"])
        t.apply_gates(r["ops"])
        plain_out.append(t.sample(r["qubits"], r["shots"], seed=r["seed"]))
        t.close()
    plain_s = time.perf_counter() - t0
    # Pauli-frame path (the paper's sampling mode): per request, one CHP run
    # of the circuit with its final measurement for the reference sample, then
    # the frames; same distribution as the per-shot CHP outcomes, other bits
    log(f"plain {plain_s:.2f} s; Pauli frames")
    progs = []
    for r in reqs:
        meas = np.stack([np.full(r["n"], sq.MEASURE, np.uint32), r["qubits"], np.zeros(r["n"], np.uint32)], 1)
        progs.append(sq.Program(r["n"], np.concatenate([r["ops"], meas])))
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
    rate = 0.8 * nreq / plain_s
    rng = np.random.Generator(np.random.PCG64(4))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    sreqs = [serving.Request(rid=k, n=r["n"], ops=r["ops"], qubits=r["qubits"], shots=r["shots"], seed=r["seed"],
                             arrival=float(a)) for k, (r, a) in enumerate(zip(reqs, arrivals))]
    log(f"batched {batch_s:.2f} s; serving at {rate:.2f} requests/s")
    st = serving.Server(budget_bytes=budget_bytes, workers=2, batch_kwargs=kw).run(sreqs)
    same = same and all(np.array_equal(r.result, b) for r, b in zip(sreqs, batch_out))
    log(f"served makespan {st.makespan_s:.2f} s, p50 {st.latency_p50_s:.3f} s, p99 {st.latency_p99_s:.3f} s")
    return {
        "workload": f"first {nreq} of the 512 batched/served requests (n log-uniform 16..16384, depth 10..500, "
                    f"1..4096 shots, final all-qubit Z measurement)",
        "requests": nreq, "shots": shots,
        "plain_shots_per_s": shots / plain_s,
        "batched_shots_per_s": shots / batch_s,
        "served_shots_per_s": st.shots_per_s,
        "batched_vs_plain": plain_s / batch_s,
        "frame_shots_per_s": shots / frame_s,
        "frame_note": "Pauli frames: reference CHP run plus frames per request, same distribution, other bits",
        "served_arrival_rate_per_s": rate,
        "served_latency_p50_s": st.latency_p50_s,
        "served_latency_p99_s": st.latency_p99_s,
        "served_batches": st.batches,
        "served_mean_batch": st.mean_batch,
        "served_budget_bytes": budget_bytes,
        "batch_schedule": dict(kw, tuned_on_requests=int(tuned["sample"])),
        "outputs_identical_across_paths": bool(same),
    }


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
    ap.add_argument("--served-requests", type=int, default=48,
                    help="requests of the batched/served mix to time (0 skips that part)")
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
    log(f"generating {args.layers} layers of n={n}")
    gates, meas, layer_parts = build_ops(cfg, args.layers, args.meas)
    log(f"{gates.size} gates; compiling")
    pg = sq.Program(n, gates)
    pm = sq.Program(n, meas)
    log(f"{pg.num_passes} gate passes, {pg.gate_bytes / 1e9:.1f} GB algorithmic per step")
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
    # Each step starts from reset (which also clears the byte accounting) and
    # does identical work, so the counters now hold exactly one step.
    st1 = t.measure_stats()
    gate_ms = sum(e[0].elapsed_time(e[1]) for e in events)
    meas_ms = sum(e[1].elapsed_time(e[2]) for e in events)
    assert t.error_flags() == 0

    kern = {name: t.profile_read(i) for i, name in enumerate(sqb.KERNEL_NAMES)}
    assert kern["layer"][1] > 0
    layer_ms, layer_n = kern["layer"]
    n_random = st1.n_random

    def roof(name, ms, launches, total_bytes):
        per = total_bytes / max(launches, 1)
        gbs = per / (ms / launches * 1e-3) / 1e9 if launches else 0.0
        # HBM bytes per launch from the committed rocprofv3 counter summary of
        # this workload (its first layers and measurements), or None if that
        # kernel's source changed since or the run measures far beyond the
        # start of the sweep, where a block's bytes differ
        traffic = profsum.traffic_per_dispatch(name, HBM_SUMMARY) if args.meas <= 1000 else None
        return {"kernel": name, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes per launch",
                "traffic_over_algorithmic": round(traffic / per, 3) if traffic and per else None,
                "bytes_per_launch": int(per),
                "avg_launch_ms": round(ms / max(launches, 1), 4), "launches_per_step": launches // args.steps,
                "ms_per_step": round(ms / args.steps, 3)}

    # The library's byte counters hold one step (each step starts from reset);
    # the profile holds all timed steps.
    roofs = [roof("k_layer", layer_ms, layer_n, pg.gate_bytes * args.steps)]
    if kern["block_pass"][1]:
        roofs.append(roof("k_blk_pass", *kern["block_pass"], st1.block_bytes * args.steps))
    if kern["rowsum"][1]:
        roofs.append(roof("k_rowsum", *kern["rowsum"], st1.rowsum_bytes * args.steps))
    roofs.sort(key=lambda r: -r["ms_per_step"])
    dominant, others = roofs[0], roofs[1:]

    gates_per_step = int(pg.num_gates)
    result = {
        "metric": "gates/s & measurements/s at n=180k (HBM % of peak); batched vs plain shots/s",
        "value": gates_per_step * args.steps / (gate_ms * 1e-3),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"n=180000 generator circuit (seed {cfg.seed}): {args.layers} layers + first "
                        f"{args.meas} of the final 180000 Z-measurements per step",
            "n": n, "layers": args.layers, "gates_per_step": gates_per_step, "passes_per_step": pg.num_passes,
            "measurements_per_step": args.meas,
        },
        "measurements_per_s": args.meas * args.steps / (meas_ms * 1e-3),
        "gate_phase_ms_per_step": gate_ms / args.steps,
        "meas_phase_ms_per_step": meas_ms / args.steps,
        "random_measurements_per_step": int(n_random),
        "measurement_blocks_per_step": int(st1.blocks),
        "roofline": dominant,
        "roofline_other": others,
        "kernel_ms": {k: round(v[0], 3) for k, v in kern.items()},
        "kernel_launches": {k: v[1] for k, v in kern.items()},
    }
    t.close()
    result["hbm_stream_ceiling_gbs"] = stream_ceiling()
    if args.served_requests > 0:
        result["batched_served"] = served_mix(args.served_requests, budget_bytes=8 << 30)
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(cfg, layer_parts, args.cpu_seconds)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
