"""Autotuner for the launch configuration of the correction path.

Two searches, each timed on the device in the launch mode that will use it
and cached per (GPU architecture, rig signature, options, mode) in a JSON
file.  The knobs never change results, only speed.

* eager (one rt_frameset per frame-set on one stream, as the serving
  backend issues its batches): the apply pass's work split, segment height
  in rows and apply grid (rt_ctx_tune);
* pipe (rt_pipe: statistics and estimates in order on one stream, applies
  round-robin over several streams): apply lanes and group size together
  with the work split.

    from paper_1910_03517_amd import autotune
    best = autotune.tune(rig, frames_dev, out_dev)               # eager; applies and caches
    autotune.apply_cached(rig)                                    # later runs
    pc = autotune.tune_pipe(rig, frames_dev, out_dev)            # pipe; tunes the rig, returns lanes/group
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import asdict, dataclass

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ringcorr", "autotune.json")
TILE_ROWS = (8, 16, 32, 64)
GRIDS = (0, 512, 768, 1024)
# Pipe mode: (lanes, group, fuse) forms and work splits worth timing.  Unfused,
# more lanes than 4 or groups larger than the lane count were slower in
# every measurement; one lane is the plain stream order.  Fused, a group is
# one launch of up to 4 frame-sets and the lanes take whole groups in turn
# (rigs of at most 16 cameras).
PIPE_LANES = ((2, 2, 0), (3, 1, 0), (3, 3, 0), (4, 4, 0), (1, 3, 1), (2, 3, 1), (2, 4, 1), (3, 4, 1))
FUSE_MAX_CAMS = 16
FUSE_TIE = 0.03
PIPE_SPLITS = ((32, 0), (48, 0), (64, 0), (32, 512))


@dataclass(frozen=True)
class Choice:
    tile_rows: int
    grid: int
    us_per_frameset: float


def signature(cams, opts, arch: str, mode: str = "eager") -> str:
    """Stable key of a rig: architecture, every camera's geometry, the options
    and the launch mode the knobs were timed in."""
    parts = [arch, f"nb={opts.n_blocks}", f"bw={opts.band_width}", f"closed={int(opts.closed_ring)}"]
    if mode != "eager":
        parts.append(f"mode={mode}")
    if getattr(opts, "vblend", False):
        parts.append("vblend=1")
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


@dataclass(frozen=True)
class PipeChoice:
    lanes: int
    group: int
    tile_rows: int
    grid: int
    us_per_frameset: float
    fuse: int = 0


def pipe_candidates(cams, n_blocks: int) -> list[tuple[int, int, int, int, int]]:
    """(lanes, group, tile_rows, grid, fuse) tuples for the pipe mode; tile
    heights above the tallest block are dropped, and the fused forms for rigs
    of more than FUSE_MAX_CAMS cameras."""
    tallest = max(-(-c.height // n_blocks) for c in cams)
    splits = [(r, g) for r, g in PIPE_SPLITS if r <= max(tallest, PIPE_SPLITS[0][0])]
    forms = [f for f in PIPE_LANES if not f[2] or len(cams) <= FUSE_MAX_CAMS]
    return [(l, gr, r, g, fu) for l, gr, fu in forms for r, g in splits]


def time_pipe(rig, frames, outs, lanes: int, group: int, depth: int = 8, steps: int = 64, warmup: int = 16,
              fuse: int = 0) -> float:
    """Mean microseconds per frame-set through an rt_pipe of `lanes` apply
    streams issued in groups of `group` (fused or not), rotating over the
    given buffers (their count must be a multiple of depth)."""
    import torch
    from . import rt
    n = len(frames)
    stream = torch.cuda.current_stream()
    pipe = rt.Pipe.for_rig(rig, depth=depth, lanes=lanes, group=group, fuse=bool(fuse))
    # A group of frame-sets per library call, as the bench submits them.
    chunks = [(rt.ptr_array_n([frames[(j + u) % n] for u in range(group)]),
               rt.ptr_array_n([outs[(j + u) % n] for u in range(group)]), group) for j in range(n)]
    try:
        for i in range(0, warmup - warmup % group, group):
            pipe.submit_n(None, None, stream, ptrs=chunks[i % n])
        pipe.join(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        timed = steps - steps % group
        e0.record(stream)
        for i in range(0, timed, group):
            pipe.submit_n(None, None, stream, ptrs=chunks[(warmup + i) % n])
        pipe.join(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / timed * 1e3
    finally:
        pipe.close()


def tune_pipe(rig, frames, outs, cache_path: str | None = DEFAULT_CACHE, rounds: int = 3, depth: int = 8,
              cands: list[tuple[int, int, int, int, int]] | None = None) -> PipeChoice:
    """Time every pipe candidate `rounds` times (interleaved, after an
    untimed run that brings the device to its working clocks; the median of
    each candidate's times), tune the rig to the fastest work split, cache the
    choice and return it (the caller builds its pipe with choice.lanes /
    choice.group / choice.fuse)."""
    arch = device_arch()
    key = signature(rig.cams, rig.opts, arch, "pipe")
    cands = cands or pipe_candidates(rig.cams, rig.opts.n_blocks)
    rig.tune(cands[0][2], cands[0][3])
    time_pipe(rig, frames, outs, cands[0][0], cands[0][1], depth, steps=256, fuse=cands[0][4])
    times = {c: [] for c in cands}
    for _ in range(rounds):
        for c in cands:
            lanes, group, tile_rows, grid, fuse = c
            rig.tune(tile_rows, grid)
            times[c].append(time_pipe(rig, frames, outs, lanes, group, depth, fuse=fuse))
    med = {c: sorted(t)[len(t) // 2] for c, t in times.items()}
    c = min(cands, key=lambda k: med[k])
    # A fused form within FUSE_TIE of the fastest is taken instead: it costs
    # the host one wait and one record per group rather than per lane, and
    # short runs (a burst of frame-sets after an idle pipeline) favour it,
    # while over 64 frame-sets the forms measured within 1.5 % of each other.
    fused = [k for k in cands if k[4]]
    if fused and not c[4]:
        f = min(fused, key=lambda k: med[k])
        if med[f] <= med[c] * (1.0 + FUSE_TIE):
            c = f
    choice = PipeChoice(c[0], c[1], c[2], c[3], med[c], c[4])
    rig.tune(choice.tile_rows, choice.grid)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = asdict(choice)
        save_cache(cache, cache_path)
    return choice


def cached_pipe(rig, cache_path: str = DEFAULT_CACHE) -> PipeChoice | None:
    """The cached pipe choice for this rig, with the rig tuned to its work
    split; None if there is none."""
    entry = load_cache(cache_path).get(signature(rig.cams, rig.opts, device_arch(), "pipe"))
    if not entry:
        return None
    try:
        choice = PipeChoice(int(entry["lanes"]), int(entry["group"]), int(entry["tile_rows"]), int(entry["grid"]),
                            float(entry["us_per_frameset"]), int(entry.get("fuse", 0)))
    except (KeyError, TypeError, ValueError):
        return None
    rig.tune(choice.tile_rows, choice.grid)
    return choice
