"""Autotuner for the batched launch: measures candidate (path, chunk length) pairs on the
caller's own device-resident batch with HIP-event timing and keeps the fastest.

Results are cached in a JSON file (FV_TUNE_CACHE, default ~/.cache/fv_tune.json) under a key
made of the GPU architecture, K, D, the arithmetic form and the batch size bucket
(log2 of total rows), so later processes can apply them without measuring.
"""
from __future__ import annotations

import json
import math
import os

from . import fv as _fv

CHUNKS = (256, 512, 1024, 2048, 4096)
PATHS = (1, 2)  # fused single pass, two-pass


def cache_path() -> str:
    return os.environ.get("FV_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fv_tune.json"))


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def key(g: _fv.Gmm, precision: int, rows: int) -> str:
    return f"{_arch()}|K{g.K}|D{g.D}|p{precision}|r2^{int(math.log2(max(rows, 1)))}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(k: str, cfg: dict):
    c = _load_cache()
    c[k] = cfg
    os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
    tmp = cache_path() + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path())


def measure(g, Xd, offsets, out, precision, stream, reps=5) -> float:
    """Median milliseconds of fv_encode_batch (events on `stream`)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    _fv.encode_batch(g, Xd, offsets, out=out, precision=precision, flags=_fv.ASYNC, stream=stream)
    for a, b in ev:
        a.record(stream)
        _fv.encode_batch(g, Xd, offsets, out=out, precision=precision, flags=_fv.ASYNC, stream=stream)
        b.record(stream)
    stream.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    return ts[len(ts) // 2]


def tune_batch(g: _fv.Gmm, Xd, offsets, precision: int = 0, stream=None, chunks=CHUNKS,
               paths=PATHS, reps=5, use_cache=True) -> dict:
    """Pick the fastest (path, chunk) for this batch shape; applies and caches it."""
    import torch
    rows = int(offsets[-1])
    k = key(g, precision, rows)
    if use_cache:
        hit = _load_cache().get(k)
        if hit:
            _fv.set_tuning(g, hit["batch_chunk"], hit["batch_path"], hit.get("single_split_below", 0))
            return dict(hit, cached=True)
    stream = stream or torch.cuda.Stream()
    out = torch.empty(len(offsets) - 1, g.out_len, dtype=torch.float32, device=Xd.device)
    saved = _fv.get_tuning(g)
    trials = []
    for p in paths:
        if p == 1 and g.K > 256:
            continue
        for ch in chunks:
            _fv.set_tuning(g, ch, p, saved["single_split_below"])
            trials.append({"batch_path": p, "batch_chunk": ch,
                           "ms": measure(g, Xd, offsets, out, precision, stream, reps)})
    best = min(trials, key=lambda t: t["ms"])
    cfg = {"batch_chunk": best["batch_chunk"], "batch_path": best["batch_path"],
           "single_split_below": saved["single_split_below"], "ms": best["ms"], "trials": trials}
    _fv.set_tuning(g, cfg["batch_chunk"], cfg["batch_path"], cfg["single_split_below"])
    if use_cache:
        _store(k, cfg)
    return dict(cfg, cached=False)


def apply(g: _fv.Gmm, precision: int, rows: int) -> bool:
    """Apply a cached result for this handle and batch size, if any."""
    hit = _load_cache().get(key(g, precision, rows))
    if not hit:
        return False
    _fv.set_tuning(g, hit["batch_chunk"], hit["batch_path"], hit.get("single_split_below", 0))
    return True
