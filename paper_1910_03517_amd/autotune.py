"""Autotuner for the apply pass's work split.

Searches the runtime knobs of a context (segment height in rows and apply
grid; see rt_ctx_tune) by timing the full frame-set on the device, and
caches the winner per (GPU architecture, rig signature, options) in a JSON
file.  The knobs never change results, only speed.

    from paper_1910_03517_amd import autotune
    best = autotune.tune(rig, frames_dev, out_dev)          # applies and caches
    autotune.apply_cached(rig)                               # later runs
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import asdict, dataclass

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ringcorr", "autotune.json")
TILE_ROWS = (8, 16, 32, 64)
GRIDS = (0, 512, 768, 1024)


@dataclass(frozen=True)
class Choice:
    tile_rows: int
    grid: int
    us_per_frameset: float


def signature(cams, opts, arch: str) -> str:
    """Stable key of a rig: architecture, every camera's geometry, and the options."""
    parts = [arch, f"nb={opts.n_blocks}", f"bw={opts.band_width}", f"closed={int(opts.closed_ring)}"]
    for c in cams:
        parts.append(f"{c.width}x{c.height}x{c.channels}b{c.bit_depth}r{c.ring}p{c.pos}s{c.pitch_bytes}")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:24]


def candidates(cams, n_blocks: int) -> list[tuple[int, int]]:
    """(tile_rows, grid) pairs worth timing: tile heights up to the tallest block."""
    tallest = max(-(-c.height // n_blocks) for c in cams)
    rows = sorted({r for r in TILE_ROWS if r <= max(tallest, TILE_ROWS[0])} | {min(tallest, TILE_ROWS[-1])})
    return [(r, g) for r in rows for g in GRIDS]


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def time_frameset(rig, frames, outs, iters: int = 30, warmup: int = 5) -> float:
    """Mean microseconds per rt_frameset over `iters` calls, rotating over the given buffers."""
    import torch
    n = len(frames)
    for i in range(warmup):
        rig.frameset(frames[i % n], outs[i % n])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(iters):
        rig.frameset(frames[i % n], outs[i % n])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / iters * 1e3


def tune(rig, frames, outs, cache_path: str | None = DEFAULT_CACHE, iters: int = 30,
         cands: list[tuple[int, int]] | None = None) -> Choice:
    """Time every candidate on this rig, apply the fastest, cache it.

    frames / outs: lists of per-camera device frame lists (one or more
    frame-sets to rotate over).  The estimator state of the rig advances while
    timing; reset it afterwards if that matters.
    """
    arch = device_arch()
    key = signature(rig.cams, rig.opts, arch)
    best = None
    for tile_rows, grid in (cands or candidates(rig.cams, rig.opts.n_blocks)):
        rig.tune(tile_rows, grid)
        us = time_frameset(rig, frames, outs, iters)
        if best is None or us < best.us_per_frameset:
            best = Choice(tile_rows, grid, us)
    rig.tune(best.tile_rows, best.grid)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = asdict(best)
        save_cache(cache, cache_path)
    return best


def apply_cached(rig, cache_path: str = DEFAULT_CACHE) -> Choice | None:
    """Apply a cached choice for this rig if there is one; returns it or None."""
    key = signature(rig.cams, rig.opts, device_arch())
    entry = load_cache(cache_path).get(key)
    if not entry:
        return None
    choice = Choice(int(entry["tile_rows"]), int(entry["grid"]), float(entry["us_per_frameset"]))
    rig.tune(choice.tile_rows, choice.grid)
    return choice
