"""Autotuner for the kernel choices of single frames and batches.

Every choice (``sb_tune``: vote pixels per thread, tile rows and uniform-window
split, levels per gather round and blocks per wave; for batches also the
persistent grid's blocks per compute unit) computes the same bits, so the tuner may pick any of them.  It times
each candidate on the caller's own work with HIP events, keeps only
candidates whose outputs equal the default choice's bit for bit, and caches
the winner in a JSON file keyed by the device name and a signature of the
work (sizes, guide formats, parameters).  Timing and launching go through the
C ABI like every other call; nothing here computes pixels.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import TUNES, Batch, FrameJob, SbParams, Style, _torch, stylize

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "styleblit_gfx950", "tune.json")
BATCH_BLOCKS_PER_CU = (2, 4, 8, 16)


def _device_name(torch) -> str:
    # the tag changes whenever the set of kernel choices does, so cached
    # winners of an older set are never read back
    return torch.cuda.get_device_name(0) + "|choices5"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, cache: Dict[str, dict]):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _tkey(tune) -> str:
    return ",".join(str(int(v)) for v in tune)


def _tparse(key: str) -> List[int]:
    return [int(v) for v in key.split(",")]


def _params_key(p: SbParams) -> str:
    return f"L{p.levels}f{p.finest}t{p.threshold}r{p.radius}"


def frame_signature(style: Style, w: int, h: int, p: SbParams) -> str:
    return f"frame:{w}x{h}:src{style.sw}x{style.sh}:fmt{style.fmt}:{_params_key(p)}"


def batch_signature(jobs: Sequence[FrameJob]) -> str:
    """Signature of a batch by its shape mix (order-insensitive)."""
    parts = sorted(f"{j.w}x{j.h}:fmt{j.style.fmt}:{_params_key(j.params)}" for j in jobs)
    px = sum(j.w * j.h for j in jobs)
    return f"batch:{len(jobs)}:{px}:" + ",".join(sorted(set(parts)))


def _time_events(torch, fn, reps: int) -> float:
    """Median milliseconds of fn over reps runs (HIP events on the current
    stream, after one warm-up run)."""
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune_frame(style: Style, guide, jitter, p: SbParams, candidates: Iterable[Tuple] = TUNES,
               reps: int = 10, cache_path: Optional[str] = DEFAULT_CACHE,
               refresh: bool = False) -> dict:
    """Fastest bit-exact kernel choice for frames like this one.  Returns
    {"tune": (ppt, rows, group), "ms": ..., "candidates": {...}, "cached": bool}."""
    torch = _torch()
    h, w = (int(guide.shape[0]), int(guide.shape[1]))
    key = f"{_device_name(torch)}|{frame_signature(style, w, h, p)}"
    cache = _load(cache_path) if cache_path else {}
    if not refresh and key in cache:
        ent = dict(cache[key])
        ent["tune"] = tuple(ent["tune"])
        ent["cached"] = True
        return ent
    ref_rgb, ref_chunk = stylize(style, guide, jitter, p)
    torch.cuda.synchronize()
    rgb = torch.empty_like(ref_rgb)
    chunk = torch.empty_like(ref_chunk)
    results = {}
    for tune in candidates:
        fn = lambda: stylize(style, guide, jitter, p, out_rgb=rgb, out_chunk=chunk, tune=tune)
        ms = _time_events(torch, fn, reps)
        exact = bool(torch.equal(rgb, ref_rgb) and torch.equal(chunk, ref_chunk))
        results[_tkey(tune)] = {"ms": ms, "exact": exact}
    best = min((k for k, v in results.items() if v["exact"]), key=lambda k: results[k]["ms"])
    ent = {"tune": _tparse(best), "ms": results[best]["ms"], "candidates": results,
           "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if cache_path:
        cache[key] = ent
        _store(cache_path, cache)
    ent["tune"] = tuple(ent["tune"])
    ent["cached"] = False
    return ent


def tune_batch(jobs: List[FrameJob], candidates: Iterable[Tuple] = TUNES,
               blocks_per_cu: Iterable[int] = BATCH_BLOCKS_PER_CU, reps: int = 3,
               cache_path: Optional[str] = DEFAULT_CACHE, refresh: bool = False,
               workspace=None) -> dict:
    """Fastest bit-exact (tune, blocks_per_cu) for graph-captured batches of
    this shape mix.  The reference outputs are the default choice's, run as
    separate frames.  Returns {"tune", "blocks_per_cu", "ms", "candidates",
    "cached"}."""
    torch = _torch()
    key = f"{_device_name(torch)}|{batch_signature(jobs)}"
    cache = _load(cache_path) if cache_path else {}
    if not refresh and key in cache:
        ent = dict(cache[key])
        ent["tune"] = tuple(ent["tune"])
        ent["cached"] = True
        return ent
    refs = [stylize(j.style, j.guide, j.jitter, j.params) for j in jobs]
    torch.cuda.synchronize()
    results = {}
    for tune in candidates:
        for bpc in blocks_per_cu:
            b = Batch(use_graph=True, tune=tune, blocks_per_cu=bpc)
            if workspace is None:
                workspace = torch.empty(b.workspace_bytes(jobs), dtype=torch.uint8, device="cuda")
            for j in jobs:  # poison the outputs so a skipped frame cannot pass
                j.out_rgb.fill_(0x5A)
                j.out_chunk.fill_(-1)
            ms = _time_events(torch, lambda: b.run(jobs, workspace=workspace), reps)
            torch.cuda.synchronize()
            exact = all(torch.equal(j.out_rgb, r[0]) and torch.equal(j.out_chunk, r[1])
                        for j, r in zip(jobs, refs))
            b.close()
            results[f"{_tkey(tune)}|{bpc}"] = {"ms": ms, "exact": exact}
    best = min((k for k, v in results.items() if v["exact"]), key=lambda k: results[k]["ms"])
    tstr, bstr = best.split("|")
    ent = {"tune": _tparse(tstr), "blocks_per_cu": int(bstr), "ms": results[best]["ms"],
           "candidates": results, "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if cache_path:
        cache[key] = ent
        _store(cache_path, cache)
    ent["tune"] = tuple(ent["tune"])
    ent["cached"] = False
    return ent
