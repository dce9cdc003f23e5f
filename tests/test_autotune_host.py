"""Autotuner host logic (no GPU): candidate selection, stratified sampling and
the per-device cache."""
import json

import numpy as np

from paper_2603_14641_amd import autotune


def test_pick_best_takes_the_fastest():
    cands = [dict(a=1), dict(a=2), dict(a=3)]
    res = autotune.pick_best(cands, lambda c: {1: 0.3, 2: 0.1, 3: 0.2}[c["a"]])
    assert res["best"] == dict(a=2) and abs(res["seconds"] - 0.1) < 1e-12
    assert [r["seconds"] for r in res["table"]] == [0.3, 0.1, 0.2]


def test_stratified_sample_spans_sizes():
    reqs = [dict(n=int(n)) for n in np.random.default_rng(0).integers(16, 16384, 200)]
    sub = autotune.stratified_sample(reqs, 10)
    ns = sorted(r["n"] for r in sub)
    assert len(sub) == 10
    assert ns[0] == min(r["n"] for r in reqs) and ns[-1] == max(r["n"] for r in reqs)


def test_n_bucket():
    assert autotune.n_bucket(1) == 1 and autotune.n_bucket(64) == 64 and autotune.n_bucket(65) == 128
    assert autotune.n_bucket(180000) == 262144


def test_batch_tuning_is_cached(monkeypatch, tmp_path):
    monkeypatch.setenv("SQ_TUNE_CACHE", str(tmp_path / "c.json"))
    monkeypatch.setattr(autotune, "device_key", lambda: "fake-gpu")
    calls = []

    def fake_batch(reqs, **kw):
        calls.append(kw)
        return []

    monkeypatch.setattr(autotune.binding, "batch_sample", fake_batch)
    reqs = [dict(n=n) for n in range(16, 400, 7)]
    cands = [dict(block=128, max_batch_n=1024, streams=4), dict(block=256, max_batch_n=2048, streams=4)]
    first = autotune.tune_batch(reqs, sample=5, candidates=cands)
    assert len(calls) == 2 and first["block"] in (128, 256)
    again = autotune.tune_batch(reqs, sample=5, candidates=cands)
    assert len(calls) == 2 and again == first
    data = json.load(open(tmp_path / "c.json"))
    assert "fake-gpu/batch/default" in data
