#!/usr/bin/env python3
"""Write tests/golden/served_mix_oracle.json: the CPU oracle's per-shot CHP
outcomes on the batched/served mix (512 generator circuits, n log-uniform in
[16, 16384], depth uniform in [10, 500], 1..4096 shots of measuring every
qubit in order, coin seed 1000 + i).

Per request it stores the checked shot indices and a SHA-256 of their
outcome words (shot-major, ceil(n/64) little-endian uint64 words per shot,
bit i of word i/64 = outcome of qubit i), the layout sq_sample returns:
  * n <= 256: every shot;
  * 256 < n <= 2048: shots {0, 1, S-1} and 5 more drawn from
    numpy Generator(PCG64(5000 + i));
  * 2048 < n <= 8192: 8 requests drawn with numpy Generator(PCG64(77))
    among them, shots {0, S-1} (a per-shot CHP sweep costs ~n^3 bit
    operations, so the largest requests are left to the batched-vs-plain
    comparison of the GPU test).

Shot s is, by definition, the CHP measurement sequence run on a copy of the
circuit's final state with coins keyed (coin seed, shot s, measurement index).
This script calls only oracle/ and workload/; it takes about an hour on
8 cores and saves after every request, so an interrupted run resumes where
it stopped. Command (from the repository root):
    python tests/golden/make_served_mix_fixtures.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from workload import circuit_ops, served_requests  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "served_mix_oracle.json")
LARGE_PICKS = 8
LARGE_MAX_N = 8192


def checked_shots(i: int, n: int, shots: int, large: set) -> list:
    if n <= 256:
        return list(range(shots))
    if n <= 2048:
        rng = np.random.Generator(np.random.PCG64(5000 + i))
        return sorted({0, 1 % shots, shots - 1} | {int(v) for v in rng.integers(0, shots, 5)})
    if i in large:
        return sorted({0, shots - 1})
    return []


def oracle_words(n, gates, seed, shot_list):
    ref = orc.Tableau(n)
    ref.run(gates)
    x, z, r = ref.rows_array()
    meas = np.stack([np.full(n, orc.MEASURE, np.uint32), np.arange(n, dtype=np.uint32),
                     np.zeros(n, np.uint32)], 1)
    W = (n + 63) // 64
    out = np.zeros((len(shot_list), W), dtype=np.uint64)
    for k, s in enumerate(shot_list):
        t = orc.Tableau(n)
        t.set_rows(x, z, r)
        bits, _, _ = t.run(meas, seed=seed, shot=s, meas_base=0)
        assert bits.size == n and t.odd_count == 0 and t.badscratch_count == 0
        padded = np.zeros(W * 64, dtype=np.uint8)
        padded[:n] = bits
        out[k] = np.packbits(padded.reshape(W, 64), axis=1, bitorder="little").view(np.uint64)[:, 0]
    return out


def main():
    reqs = served_requests()
    big = [r.index for r in reqs if 2048 < r.n <= LARGE_MAX_N]
    pick = np.random.Generator(np.random.PCG64(77)).choice(len(big), LARGE_PICKS, replace=False)
    large = {big[int(k)] for k in pick}
    res = {}
    if os.path.exists(OUT):  # resume: keep entries made with the same rule
        res = json.load(open(OUT)).get("requests", {})
        want = {str(r.index) for r in reqs if checked_shots(r.index, r.n, r.shots, large)}
        res = {k: v for k, v in res.items() if k in want}
    t0 = time.time()
    for r in reqs:
        shots = checked_shots(r.index, r.n, r.shots, large)
        if not shots:
            continue
        old = res.get(str(r.index))
        if old and old["shots"] == shots and old["n"] == r.n and old["shots_total"] == r.shots:
            continue
        cfg = r.config()
        ops = circuit_ops(cfg, final_measure=False)
        gates = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
        words = oracle_words(r.n, gates, r.coin_seed, shots)
        res[str(r.index)] = {"n": r.n, "depth": r.depth, "shots_total": r.shots, "shots": shots,
                             "sha256": hashlib.sha256(np.ascontiguousarray(words).tobytes()).hexdigest()}
        print(f"[{time.time() - t0:7.1f} s] request {r.index}: n={r.n} d={r.depth} {len(shots)} shots",
              flush=True)
        save(res, partial=True)
    save(res, partial=False)
    print(f"wrote {OUT}: {len(res)} requests, {sum(len(v['shots']) for v in res.values())} shots")


def save(res, partial):
    doc = {"what": "oracle per-shot CHP outcomes of the batched/served mix, checked shots and SHA-256 of their "
                   "outcome words (shot-major, ceil(n/64) little-endian uint64 per shot)",
           "command": "python tests/golden/make_served_mix_fixtures.py",
           "complete": not partial,
           "requests": res}
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=0, sort_keys=True)
    os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
