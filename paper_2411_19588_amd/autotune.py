"""Launch-shape and binning-schedule autotuner for the rasterizer.

Times forward + L1 + backward over the caller's own workload (Gaussians, camera list,
medium) for a set of launch shapes -- tile size, pixels per lane (waves per tile), how
the compositing waves receive records (LDS batches or the scalar cache), LDS batch
size, persistent tile queue -- and then for depth-phase schedules (number of phases,
size of the first), and returns the fastest as a RasterConfig.  Every choice renders
bit-identical images, so it only affects speed.  Results are cached in a JSON file
keyed by the device and a coarse description of the workload.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence

from .rasterizer import RasterConfig

SHAPE_FIELDS = ("tile", "pixels_per_lane", "record_fetch", "lds_batch", "persistent")
SCHEDULE_FIELDS = ("phases", "phase0_shift", "phase_growth")
FIELDS = SHAPE_FIELDS + SCHEDULE_FIELDS


def candidates(tiles=(16, 8), persistent=(0, 1, 2)) -> List[dict]:
    """Launch shapes worth timing (8x8 tiles take one pixel per lane and 64-record batches)."""
    out = []
    for tile in tiles:
        for pers in persistent:
            if tile == 8:
                out.append(dict(tile=8, pixels_per_lane=1, record_fetch="lds", lds_batch=64, persistent=pers))
                out.append(dict(tile=8, pixels_per_lane=1, record_fetch="scalar", lds_batch=64, persistent=pers))
                continue
            for ppl in (1, 2, 4):
                for lb in (64, 256):
                    out.append(dict(tile=16, pixels_per_lane=ppl, record_fetch="lds", lds_batch=lb, persistent=pers))
                out.append(dict(tile=16, pixels_per_lane=ppl, record_fetch="scalar", lds_batch=256, persistent=pers))
    return out


def schedules() -> List[dict]:
    """Depth-phase schedules worth timing: the nearest 1/2^shift of the Gaussians first, each later
    phase 2^growth times wider."""
    return [dict(phases=p, phase0_shift=sh, phase_growth=g)
            for p, sh, g in ((2, 5, 2), (2, 6, 2), (2, 7, 2), (3, 5, 2), (3, 6, 2), (4, 6, 2), (4, 7, 2), (5, 7, 2),
                             (5, 8, 2), (6, 10, 2), (8, 14, 2), (5, 6, 1), (6, 7, 1), (7, 8, 1), (8, 9, 1),
                             (3, 6, 3), (4, 8, 3))]


def workload_key(device_name: str, n: int, sh_degree: int, sizes: Sequence) -> str:
    """Device, Gaussian count (rounded to a power of two), SH degree, view count and
    total pixels (rounded to a power of two)."""
    pixels = sum(int(w) * int(h) for w, h in sizes)
    n2 = 1 << max(0, int(math.ceil(math.log2(max(1, n)))))
    p2 = 1 << max(0, int(math.ceil(math.log2(max(1, pixels)))))
    return f"{device_name}|n{n2}|sh{sh_degree}|v{len(sizes)}|p{p2}"


def pick(timings: Dict[int, float]) -> int:
    """Index of the fastest finite timing (ties: the earlier candidate)."""
    best, best_t = None, math.inf
    for i in sorted(timings):
        t = timings[i]
        if t is not None and math.isfinite(t) and t < best_t:
            best, best_t = i, t
    if best is None:
        raise RuntimeError("no candidate could be timed")
    return best


def load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: Optional[str], key: str, entry: dict) -> None:
    if not path:
        return
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(base: RasterConfig, shape: dict) -> RasterConfig:
    return dataclasses.replace(base, **{k: shape[k] for k in FIELDS if k in shape})


def tune(measure: Callable[[RasterConfig], float], base: RasterConfig = RasterConfig(),
         shapes: Optional[Iterable[dict]] = None, cache_path: Optional[str] = None, key: Optional[str] = None,
         log: Optional[Callable[[str], None]] = None) -> RasterConfig:
    """Return `base` with the launch shape whose `measure(config)` (milliseconds) is lowest.

    A cached entry for `key` is used as is.  `measure` may return None or raise for a
    shape that cannot run; such shapes are skipped.
    """
    if key is not None:
        hit = load_cache(cache_path).get(key)
        if hit and "shape" in hit:
            return apply(base, hit["shape"])
    shapes = list(candidates() if shapes is None else shapes)
    timings: Dict[int, Optional[float]] = {}
    for i, sh in enumerate(shapes):
        try:
            timings[i] = measure(apply(base, sh))
        except (RuntimeError, ValueError) as e:   # e.g. a shape the library rejects
            timings[i] = None
            if log:
                log(f"autotune: {sh} failed: {e}")
        if log and timings[i] is not None:
            log(f"autotune: {sh} {timings[i]:.3f} ms")
    best = pick(timings)
    if key is not None:
        store_cache(cache_path, key, {"shape": shapes[best], "ms": timings[best],
                                      "timed": [[shapes[i], timings[i]] for i in sorted(timings)]})
    return apply(base, shapes[best])


def tune_all(measure: Callable[[RasterConfig], float], base: RasterConfig = RasterConfig(),
             cache_path: Optional[str] = None, key: Optional[str] = None,
             log: Optional[Callable[[str], None]] = None) -> RasterConfig:
    """Launch shape first (at the base schedule), then the depth-phase schedule at that shape."""
    shape = tune(measure, base, candidates(), cache_path, None if key is None else key + "|shape", log)
    return tune(measure, shape, schedules(), cache_path, None if key is None else key + "|schedule", log)


def render_step_timer(params: dict, sh_degree: int, cameras: Sequence, medium, targets, reps: int = 3,
                      device="cuda") -> Callable[[RasterConfig], float]:
    """A `measure` function: milliseconds of one forward + L1 + backward over the views,
    the median of `reps` eager steps after a warm-up step (HIP events on one stream)."""
    import torch

    from .trainer import RenderStep

    def measure(cfg: RasterConfig) -> float:
        rs = RenderStep(params, sh_degree, cameras, medium, targets, cfg, device=device)
        stream = torch.cuda.Stream(device=device)
        with torch.cuda.stream(stream):
            rs.size_capacity(1.25)
            rs.enqueue(stream)
            times = []
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                rs.enqueue(stream)
                b.record(stream)
                b.synchronize()
                times.append(a.elapsed_time(b))
        st, _ = rs.status(stream)
        del rs
        if st != 0:
            return None
        return sorted(times)[len(times) // 2]

    return measure
