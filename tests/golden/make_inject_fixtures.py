#!/usr/bin/env python3
"""Write tests/golden/inject_oracle.json: the operator-tableau oracle's
result (the paper's CX-injection collapse, Algorithm alg:stim) on the whole
of configs 1 and 2 (n = 64, depth 10; n = 4,096, depth 100 with nine
mid-circuit rounds; every qubit measured at the end), coin seed 1000 + the
circuit seed, shot 0, measurement indices from 0.

Per config it stores the outcomes, the random flags and one SHA-256 of the
final tableau in the library's export layout: x rows then z rows (2n rows
each: the destabilizer half XD / ZD, then the stabilizer half XS / ZS, as
ceil(n/64) little-endian uint64 words per row, bit j of word j/64 = qubit
j), then 2n sign bytes (SignsD[0..n), then SignsS[0..n)).

This script calls only oracle/ and workload/; it takes about a minute.
Command (from the repository root):
    python tests/golden/make_inject_fixtures.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from workload import CONFIGS, circuit_ops  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "inject_oracle.json")


def signs(vec, n):
    return np.unpackbits(np.ascontiguousarray(vec, dtype="<u8").view(np.uint8), bitorder="little")[:n]


def one(cfg_id: int) -> dict:
    cfg = CONFIGS[cfg_id]
    seed = 1000 + cfg.seed
    ops = circuit_ops(cfg)
    a = np.stack([ops["type"], ops["q0"], ops["q1"]], 1).astype(np.uint32)
    ot = orc.OTableau(cfg.n)
    bits, rnd = ot.run(a, seed=seed, shot=0, meas_base=0)
    assert ot.odd_count == 0
    xs, xd, zs, zd, ss, sd = ot.arrays()
    h = hashlib.sha256()
    for m in (np.concatenate([xd, xs]), np.concatenate([zd, zs])):
        h.update(np.ascontiguousarray(m, dtype="<u8").tobytes())
    h.update(np.concatenate([signs(sd, cfg.n), signs(ss, cfg.n)]).astype(np.uint8).tobytes())
    print(f"config {cfg_id}: {bits.size} measurements, {int(rnd.sum())} random", flush=True)
    return {"n": cfg.n, "depth": cfg.depth, "seed": seed, "outcomes": "".join(str(int(b)) for b in bits),
            "random": "".join(str(int(b)) for b in rnd), "state_sha256": h.hexdigest()}


def main():
    doc = {"what": "operator-tableau oracle (CX-injection collapse): outcomes, random flags and SHA-256 of the "
                   "final tableau (x rows, z rows, sign bytes in the library's export layout)",
           "command": "python tests/golden/make_inject_fixtures.py",
           "configs": {str(c): one(c) for c in (1, 2)}}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0, sort_keys=True)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
