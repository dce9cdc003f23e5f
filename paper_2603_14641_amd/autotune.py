"""Autotuner for launch geometry.

* Tableau kernels: for an n bucket (next power of two), time candidate
  (block, words per thread, chunk) shapes of the gate-pass kernel and of the
  rowsum kernel on a synthetic generator circuit, with the library's own HIP
  event timing, and keep the fastest of each.
* Batched sampling: time candidate (block, size threshold for the persistent
  launch, concurrent streams for larger circuits) on a stratified sample of the
  requests and keep the fastest.

Winners are cached per device in a JSON file (``SQ_TUNE_CACHE`` or
``~/.cache/sq_autotune.json``). Tuning changes only launch shapes, never
results: every shape is bit-exact (the parity tests run several shapes).
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import binding

LAYER_CANDIDATES = [
    dict(layer_block=b, layer_wpt=w, layer_groups=g)
    for b in (64, 256, 512) for w in (1, 2) for g in (0, 64, 256)
]
ROWSUM_CANDIDATES = [
    dict(rowsum_block=b, rowsum_wpt=w, rowsum_cols=c)
    for b in (64, 256, 512) for w in (1, 2) for c in (0, 128, 512)
]
BATCH_CANDIDATES = [
    dict(block=b, max_batch_n=m, streams=s)
    for b in (128, 256) for m in (256, 512, 1024, 2048) for s in (4, 8)
]


def cache_path() -> str:
    return os.environ.get("SQ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sq_autotune.json"))


def _load_cache(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, data: Dict):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}/{getattr(p, 'gcnArchName', '')}/{p.multi_processor_count}"


def n_bucket(n: int) -> int:
    return 1 << max(0, int(n - 1).bit_length())


def pick_best(candidates: Sequence[Dict], timer: Callable[[Dict], float]) -> Dict:
    """Time every candidate (seconds, lower is better) and return the fastest,
    with its time, and the table of all times."""
    times = []
    for c in candidates:
        times.append(float(timer(c)))
    k = int(np.argmin(times))
    return dict(best=dict(candidates[k]), seconds=times[k],
                table=[dict(c, seconds=t) for c, t in zip(candidates, times)])


# ---------------------------------------------------------------- tableau kernels
def _timers_for_tableau(n: int, layers: int, meas: int, seed: int):
    from workload import CircuitConfig, iter_circuit
    cfg = CircuitConfig(f"tune{n}", n, layers + 20, seed, cz=True, mid_measure=False)
    parts = [arr for kind, arr in iter_circuit(cfg, final_measure=False)]
    warm = np.concatenate(parts[:20]) if len(parts) > 20 else np.concatenate(parts)
    test = np.concatenate(parts[20:]) if len(parts) > 20 else parts[-1]
    t = binding.Tableau(n)
    t.apply_gates(warm)
    t.sync()
    qubits = iter(range(10 ** 9))

    def layer_timer(c: Dict) -> float:
        t.set_tuning(**c)
        t.profile_reset()
        t.profile(True)
        t.apply_gates(test)
        ms, k = t.profile_read(binding.K_LAYER)
        t.profile(False)
        return ms / max(k, 1) * 1e-3

    def rowsum_timer(c: Dict) -> float:
        t.set_tuning(**c)
        t.profile_reset()
        t.profile(True)
        qs = [next(qubits) % n for _ in range(meas)]
        t.measure(qs, seed=seed)
        ms, k = t.profile_read(binding.K_ROWSUM)
        t.profile(False)
        return ms / max(k, 1) * 1e-3

    return t, layer_timer, rowsum_timer


def tune_tableau(n: int, layers: int = 4, meas: int = 4, seed: int = 0, use_cache: bool = True) -> Dict:
    """Best launch shapes for a tableau of n qubits (cached per device and n bucket)."""
    path = cache_path()
    key = f"{device_key()}/tableau/{n_bucket(n)}"
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        return cache[key]
    nb = n_bucket(n) if n_bucket(n) <= 262144 else n
    t, layer_timer, rowsum_timer = _timers_for_tableau(nb, layers, meas, seed)
    try:
        lay = pick_best(LAYER_CANDIDATES, layer_timer)
        row = pick_best(ROWSUM_CANDIDATES, rowsum_timer)
    finally:
        t.close()
    res = dict(lay["best"], **row["best"], layer_seconds=lay["seconds"], rowsum_seconds=row["seconds"],
               tuned_at=time.strftime("%Y-%m-%d %H:%M:%S"))
    if use_cache:
        cache = _load_cache(path)
        cache[key] = res
        _store_cache(path, cache)
    return res


def tuned_tableau(n: int, stream=None, tune_if_missing: bool = True) -> binding.Tableau:
    """A Tableau with the cached (or freshly tuned) launch shapes applied."""
    key = f"{device_key()}/tableau/{n_bucket(n)}"
    cfg = _load_cache(cache_path()).get(key)
    if cfg is None and tune_if_missing:
        cfg = tune_tableau(n)
    t = binding.Tableau(n, stream=stream)
    if cfg:
        t.set_tuning(**{k: v for k, v in cfg.items() if k in {f for f, _ in binding.Tuning._fields_}})
    return t


# ---------------------------------------------------------------- batched sampling
def stratified_sample(requests: List[Dict], k: int, seed: int = 0) -> List[Dict]:
    """k requests spread over the size range (sorted by n, evenly spaced)."""
    if len(requests) <= k:
        return list(requests)
    order = sorted(range(len(requests)), key=lambda i: requests[i]["n"])
    idx = np.linspace(0, len(order) - 1, k).round().astype(int)
    return [requests[order[i]] for i in sorted(set(idx.tolist()))]


def tune_batch(requests: List[Dict], sample: int = 24, candidates: Optional[Iterable[Dict]] = None,
               use_cache: bool = True, cache_tag: str = "default") -> Dict:
    """Best (block, max_batch_n, streams) for batched sampling of a request mix."""
    path = cache_path()
    key = f"{device_key()}/batch/{cache_tag}"
    if use_cache:
        cache = _load_cache(path)
        if key in cache:
            return cache[key]
    sub = stratified_sample(requests, sample)
    cands = list(candidates or BATCH_CANDIDATES)

    def timer(c: Dict) -> float:
        t0 = time.perf_counter()
        binding.batch_sample(sub, **c)
        return time.perf_counter() - t0

    res = pick_best(cands, timer)
    out = dict(res["best"], seconds=res["seconds"], sample=len(sub), tuned_at=time.strftime("%Y-%m-%d %H:%M:%S"))
    if use_cache:
        cache = _load_cache(path)
        cache[key] = out
        _store_cache(path, cache)
    return out
