"""Autotuner for the blend launch: tile shape, LDS fragment batch and schedule.

Each candidate renders the given frame eagerly (median of ``reps`` frames
after a warm-up); the candidate with the fastest whole frame -- projection,
binning, sorting and blend, since the tile shape changes the duplicate count
as much as the blend -- wins.  The blend kernel's own duration (the library's
event timer) is recorded alongside.  Results are cached in a JSON file
(``UMGS_AUTOTUNE_CACHE``, default ~/.cache/unimgs/autotune.json) keyed by the
frame's shape: views and their sizes, Gaussian and triangle counts, SH degree.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Dict, Iterable, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .render import Rasterizer

TILES = ((8, 8), (16, 16), (32, 8))
BATCHES = (32, 64, 128, 256)
SCHEDULES = (0, 1)


def _cache_path() -> str:
    return os.environ.get("UMGS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "unimgs", "autotune.json"))


def signature(cams, N: int, T: int, sh_degree: int, extra: str = "") -> str:
    sizes = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"V{len(cams)}:{sizes}:N{N}:T{T}:sh{sh_degree}:{extra}"


def _load() -> Dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict):
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def tune(cams: Sequence, scene: Dict[str, torch.Tensor], sh_degree: int = 0, k_bind: int = 8,
         tiles: Iterable[Tuple[int, int]] = TILES, batches: Iterable[int] = BATCHES,
         schedules: Iterable[int] = SCHEDULES, reps: int = 3, use_cache: bool = True,
         verbose: bool = False) -> Dict:
    """Best {tile, frag_batch, schedule} for rendering ``scene`` (device
    tensors as accepted by Rasterizer.project) from ``cams``."""
    N = int(scene["means"].shape[0]) if scene.get("means") is not None else 0
    T = int(scene["tri_xyz"].shape[0]) if scene.get("tri_xyz") is not None else 0
    sig = signature(cams, N, T, sh_degree)
    cache = _load() if use_cache else {}
    if sig in cache:
        c = cache[sig]
        return dict(tile=tuple(c["tile"]), frag_batch=c["frag_batch"], schedule=c["schedule"],
                    cached=True, results=c.get("results"))
    results = []
    for tile in tiles:
        r = Rasterizer("cuda:0", tile=tile, sh_degree=sh_degree, k_bind=k_bind)
        for batch in batches:
            for sched in schedules:
                r.set_options(tile=tile, frag_batch=batch, sh_degree=sh_degree, k_bind=k_bind,
                              schedule=sched)
                try:
                    r.render(cams, **scene)      # warm-up (allocation)
                except L.UmgsError as e:
                    # too many duplicates for one frame with this tile shape
                    if e.status != -2:              # CAPACITY
                        raise
                    if verbose:
                        print(f"[autotune] {tile} skipped: {e}", flush=True)
                    break
                blend_ms, frame_ms = [], []
                for _ in range(reps):
                    r.set_profiling(True)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    r.render(cams, **scene)
                    e1.record()
                    torch.cuda.synchronize()
                    prof = r.profile()
                    r.set_profiling(False)
                    blend_ms.append(prof["blend"][1])
                    frame_ms.append(e0.elapsed_time(e1))
                res = dict(tile=list(tile), frag_batch=batch, schedule=sched,
                           blend_ms=statistics.median(blend_ms), frame_ms=statistics.median(frame_ms))
                results.append(res)
                if verbose:
                    print(f"[autotune] {res}", flush=True)
        r.close()
    if not results:
        raise RuntimeError("autotune: no candidate could render the frame")
    best = min(results, key=lambda x: x["frame_ms"])
    entry = dict(tile=best["tile"], frag_batch=best["frag_batch"], schedule=best["schedule"],
                 results=results)
    if use_cache:
        cache[sig] = entry
        _store(cache)
    return dict(tile=tuple(best["tile"]), frag_batch=best["frag_batch"], schedule=best["schedule"],
                cached=False, results=results)
