#!/usr/bin/env python3
"""Write tests/golden/full_size_oracle.json: the CPU oracle's result on a
sample of rows of the two full-size generator circuits (n = 65,536 and
n = 180,000, depth 1000, seeds 2 and 3), after every gate layer and the first
M measurements of the final all-qubit Z measurement (qubits 0..M-1 in order,
coin seed = circuit seed, shot 0, measurement indices 0..M-1).

Rows evolve independently under gates, and the random-case update of a row
needs only that row and the pivot row S_p, so an oracle tableau holding a
subset of rows that contains every pivot reproduces those rows and the
outcomes exactly (the oracle stops early if a pivot falls outside the
subset, which this script turns into an error). The subset is the first
`prefix` stabilizer rows, the first 64 destabilizer rows and `extra` rows
drawn with numpy Generator(PCG64(row_seed)).

Per circuit it stores the rows, the outcomes and random flags of the M
measurements, and one SHA-256 per row of the row's x words, z words
(ceil(n/64) little-endian uint64 each, bit j of word j/64 = qubit j) and
sign byte, concatenated in that order.

This script calls only oracle/ and workload/; it takes about 20 minutes on
8 cores. Command (from the repository root):
    python tests/golden/make_full_size_fixtures.py
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
from workload import CONFIGS, iter_circuit  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_oracle.json")
PLAN = {3: dict(meas=128, prefix=256, extra=64, row_seed=303),
        4: dict(meas=128, prefix=256, extra=64, row_seed=404)}


def sample_rows(n: int, prefix: int, extra: int, row_seed: int) -> list:
    rng = np.random.Generator(np.random.PCG64(row_seed))
    pool = np.setdiff1d(np.arange(64, 2 * n), np.arange(n, n + prefix))
    drawn = rng.choice(pool, extra, replace=False)
    return sorted(set(range(n, n + prefix)) | set(range(64)) | {int(v) for v in drawn})


def row_digest(x: np.ndarray, z: np.ndarray, r: int) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(z, dtype="<u8").tobytes())
    h.update(bytes([int(r)]))
    return h.hexdigest()


def one(cfg_id: int, plan: dict) -> dict:
    cfg = CONFIGS[cfg_id]
    n = cfg.n
    rows = sample_rows(n, plan["prefix"], plan["extra"], plan["row_seed"])
    sub = orc.Tableau(n, rows=rows)
    t0 = time.time()
    ngates = 0
    for k, (kind, arr) in enumerate(iter_circuit(cfg, final_measure=False)):
        sub.run(arr)
        ngates += int(arr.size)
        if (k + 1) % 50 == 0:
            print(f"[config {cfg_id}] {k + 1}/{cfg.depth} layers, {ngates} gates, {time.time() - t0:.0f} s",
                  flush=True)
    m = plan["meas"]
    meas = np.stack([np.full(m, orc.MEASURE, np.uint32), np.arange(m, dtype=np.uint32),
                     np.zeros(m, np.uint32)], 1)
    bits, rnd, _ = sub.run(meas, seed=cfg.seed, shot=0, meas_base=0)
    if bits.size != m:
        raise RuntimeError(f"config {cfg_id}: a pivot fell outside the sampled rows after {bits.size} measurements")
    assert sub.odd_count == 0 and sub.badscratch_count == 0
    x, z, r = sub.rows_array()
    W = (n + 63) // 64
    assert x.shape == (len(rows), W)
    return {"n": n, "depth": cfg.depth, "seed": cfg.seed, "gates": ngates, "measurements": m,
            "rows": rows, "outcomes": "".join(str(int(b)) for b in bits),
            "random": "".join(str(int(b)) for b in rnd),
            "row_sha256": [row_digest(x[i], z[i], r[i]) for i in range(len(rows))]}


def main():
    which = [int(a) for a in sys.argv[1:]] or sorted(PLAN)
    doc = {"what": "oracle rows (per-row SHA-256 of x words, z words, sign byte) and outcomes of the full-size "
                   "generator circuits after all layers and the first M final measurements",
           "command": "python tests/golden/make_full_size_fixtures.py", "configs": {}}
    if os.path.exists(OUT):
        doc["configs"] = json.load(open(OUT))["configs"]
    for c in which:
        doc["configs"][str(c)] = one(c, PLAN[c])
        with open(OUT, "w") as f:
            json.dump(doc, f, indent=0, sort_keys=True)
        print(f"wrote config {c} to {OUT}", flush=True)


if __name__ == "__main__":
    main()
