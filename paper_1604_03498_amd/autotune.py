"""Autotuner for the batched launch: measures candidate launch settings on the caller's own
device-resident batch with HIP-event timing and keeps the fastest, axis by axis: first every
(path, chunk length) pair, then, for the best pair, the statistics grid (resident workgroups,
half or twice as many), then, for a fused 16-bit batch at 256 components, the kernel variant
(wave-specialised or single-role).

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
GRIDS = (0.5, 2.0)  # statistics grid as a multiple of the resident workgroups (1 = automatic)
VARIANTS = (3, 1, 2)  # fused 16-bit kernel: pipelined, wave-specialised, single-role


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


def measure(g, Xd, offsets, out, precision, stream, reps=5, warmup=3) -> float:
    """Milliseconds per fv_encode_batch over `reps` back-to-back calls (events on `stream`
    around the whole run, as in steady use, so the host's table building overlaps the device's
    work), after `warmup` untimed calls (a new setting captures its graphs in the first ones)."""
    import torch
    for _ in range(warmup):
        _fv.encode_batch(g, Xd, offsets, out=out, precision=precision, flags=_fv.ASYNC, stream=stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        _fv.encode_batch(g, Xd, offsets, out=out, precision=precision, flags=_fv.ASYNC, stream=stream)
    b.record(stream)
    stream.synchronize()
    return a.elapsed_time(b) / reps


def _set(g, cfg):
    _fv.set_tuning(g, cfg["batch_chunk"], cfg["batch_path"], cfg.get("single_split_below", 0),
                   cfg.get("batch_grid", 0), cfg.get("fused16_variant", 0))


def _resident(g) -> int:
    import torch
    cu = torch.cuda.get_device_properties(g.device).multi_processor_count
    waves = max(1, min(8, (g.K + 31) // 32 if g.K <= 256 else 8))
    return cu * max(1, 8 // (1 << (waves - 1).bit_length()))


def tune_batch(g: _fv.Gmm, Xd, offsets, precision: int = 0, stream=None, chunks=CHUNKS,
               paths=PATHS, reps=5, use_cache=True, grids=GRIDS, variants=VARIANTS) -> dict:
    """Pick the fastest launch settings for this batch shape; applies and caches them."""
    import torch
    rows = int(offsets[-1])
    k = key(g, precision, rows)
    if use_cache:
        hit = _load_cache().get(k)
        if hit:
            _set(g, hit)
            return dict(hit, cached=True)
    stream = stream or torch.cuda.Stream()
    out = torch.empty(len(offsets) - 1, g.out_len, dtype=torch.float32, device=Xd.device)
    saved = _fv.get_tuning(g)
    base = {"single_split_below": saved["single_split_below"], "batch_grid": 0, "fused16_variant": 0}
    trials = []
    # the device first runs the batch for a while at the starting setting, so that the first
    # trials do not run at a lower clock than the later ones
    p0 = next((p for p in paths if not (p == 1 and g.K > 256)), paths[0])
    _set(g, dict(base, batch_path=p0, batch_chunk=chunks[0]))
    measure(g, Xd, offsets, out, precision, stream, reps=20, warmup=3)

    def trial(cfg):
        _set(g, cfg)
        t = dict(cfg, ms=measure(g, Xd, offsets, out, precision, stream, reps))
        trials.append(t)
        return t

    # axis 1: path x chunk
    for p in paths:
        if p == 1 and g.K > 256:
            continue
        for ch in chunks:
            trial(dict(base, batch_path=p, batch_chunk=ch))
    best = min(trials, key=lambda t: t["ms"])
    # axis 2: the statistics grid, around the resident workgroup count
    res = _resident(g)
    for m in grids:
        n = max(8, int(round(res * m)))
        t = trial(dict(best, batch_grid=n))
        if t["ms"] < best["ms"]:
            best = t
    # axis 3: the fused 16-bit kernel variant (one group of 256 components, D <= 64)
    if precision in (1, 2, 3) and best["batch_path"] == 1 and 224 < g.K <= 256 and g.D <= 64:
        for v in variants:
            t = trial(dict(best, fused16_variant=v))
            if t["ms"] < best["ms"]:
                best = t
    cfg = {k2: best[k2] for k2 in ("batch_chunk", "batch_path", "single_split_below",
                                   "batch_grid", "fused16_variant")}
    cfg["ms"] = best["ms"]
    cfg["trials"] = trials
    _set(g, cfg)
    if use_cache:
        _store(k, cfg)
    return dict(cfg, cached=False)


def apply(g: _fv.Gmm, precision: int, rows: int) -> bool:
    """Apply a cached result for this handle and batch size, if any."""
    hit = _load_cache().get(key(g, precision, rows))
    if not hit:
        return False
    _set(g, hit)
    return True
