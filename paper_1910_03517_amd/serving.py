"""Serving several camera rigs from one device.

Each rig streams frame-sets (one frame per camera, already in device memory,
as after a hardware decoder).  A frame-set is corrected with the rig's own
device-resident estimator state, so a rig's frame-sets must run in arrival
order, one after the other; different rigs are independent.

The server:

* admission: a request reserves the device memory of its outputs; requests
  are admitted in arrival order while the reservations fit `mem_budget`
  (a request that does not fit waits, and nothing behind it overtakes it);
  a rig's queue holds at most `queue_limit` unadmitted requests (further
  submits are rejected), and requests that waited longer than `max_wait`
  seconds without being admitted expire (live video: a newer frame-set
  supersedes a stale one);
* continuous batching: each launch carries the oldest admitted frame-set of
  every rig that has one, all in one batched set of kernels; up to
  `max_batches_in_flight` launches are queued on the device stream, whose
  order keeps each rig's frame-sets in sequence;
* completion: a launch's event is polled; on completion the requests are
  stamped, `on_done(request)` runs (the outputs are valid during the
  callback), and their output buffers and memory return to the pool;
* failure isolation: a backend that refuses a rig's frame-set (bad shapes,
  a rig marked failed) fails that request only and launches the rest of the
  batch; a rig that fails `max_failures` times in a row is closed (its later
  submits are rejected).  A device error fails the whole launch and stops
  the server.

The scheduling runs on one thread (`poll` from the caller, or `start` /
`stop` for a background thread); `submit` may be called from any thread.
The backend interface is small so the scheduler can be tested on the CPU
with a fake backend.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable

import numpy as np


class BackendError(Exception):
    """A launch refused some rigs' frame-sets before anything was enqueued."""

    def __init__(self, rigs, msg: str):
        super().__init__(msg)
        self.rigs = sorted(set(rigs))


@dataclass
class Request:
    rig: int
    seq: int
    frames: Any                  # the rig's input frames (valid until the request completes)
    t_arrival: float
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    status: str = "queued"       # queued, admitted, running, done, failed, expired, rejected
    out: Any = None              # output frames from the pool while admitted
    error: str = ""
    ready: Any = None            # device event after which the frames are written (None: already written)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Backend:
    """What the server needs from a device.  Methods run on the scheduler thread."""

    n_rigs: int = 0

    def frameset_bytes(self, rig: int) -> int:
        """Device memory one admitted frame-set of `rig` holds (its outputs)."""
        raise NotImplementedError

    def rig_pixels(self, rig: int) -> int:
        raise NotImplementedError

    def alloc_out(self, rig: int):
        raise NotImplementedError

    def free_out(self, rig: int, out) -> None:
        raise NotImplementedError

    def launch(self, batch: list[Request]):
        """Enqueue one batched frame-set of the requests (distinct rigs) and
        return a completion token; raise BackendError naming the refused
        rigs before enqueuing anything."""
        raise NotImplementedError

    def ready(self, token) -> bool:
        raise NotImplementedError

    def wait(self, token) -> None:
        raise NotImplementedError


@dataclass
class _Launch:
    token: Any
    reqs: list


class Server:
    def __init__(self, backend: Backend, mem_budget: int, max_batches_in_flight: int = 2, queue_limit: int = 8,
                 max_wait: float | None = None, max_failures: int = 3,
                 on_done: Callable[[Request], None] | None = None, clock: Callable[[], float] = time.perf_counter):
        if max_batches_in_flight < 1:
            raise ValueError("max_batches_in_flight must be >= 1")
        for r in range(backend.n_rigs):
            if backend.frameset_bytes(r) > mem_budget:
                raise ValueError(f"rig {r}: one frame-set needs {backend.frameset_bytes(r)} bytes, "
                                 f"more than mem_budget {mem_budget}")
        self.b = backend
        self.mem_budget = mem_budget
        self.max_batches = max_batches_in_flight
        self.queue_limit = queue_limit
        self.max_wait = max_wait
        self.max_failures = max_failures
        self.on_done = on_done
        self.clock = clock
        self.mem_used = 0
        self.mem_peak = 0
        self._lock = threading.Lock()
        self._incoming: collections.deque[Request] = collections.deque()
        self._queued: collections.deque[Request] = collections.deque()       # arrival order, all rigs
        self._admitted = [collections.deque() for _ in range(backend.n_rigs)]
        self._inflight: collections.deque[_Launch] = collections.deque()
        self._seq = [0] * backend.n_rigs
        self._waiting = [0] * backend.n_rigs                                  # unadmitted, per rig
        self._fail_run = [0] * backend.n_rigs
        self.closed_rigs: set[int] = set()
        self.finished: list[Request] = []
        self.batch_sizes: list[int] = []
        self.broken: BaseException | None = None
        self._thread: threading.Thread | None = None
        self._stop = threading.Event()

    # ------------------------------------------------------------------ producers
    def submit(self, rig: int, frames, t_arrival: float | None = None, ready=None) -> Request:
        """Queue one frame-set of `rig` (thread-safe).  `ready` is an event of
        the frames' producer (e.g. a decoder stream), recorded after it wrote
        them: the device work of this frame-set waits for it.  Without one the
        frames must already be complete."""
        if not 0 <= rig < self.b.n_rigs:
            raise ValueError(f"rig {rig} outside 0..{self.b.n_rigs - 1}")
        with self._lock:
            req = Request(rig, self._seq[rig], frames, self.clock() if t_arrival is None else t_arrival, ready=ready)
            self._seq[rig] += 1
            if rig in self.closed_rigs or self.broken is not None:
                req.status, req.error = "rejected", "rig closed" if rig in self.closed_rigs else "server stopped"
                self.finished.append(req)
            elif self._waiting[rig] >= self.queue_limit:
                req.status, req.error = "rejected", "queue full"
                self.finished.append(req)
            else:
                self._waiting[rig] += 1
                self._incoming.append(req)
            return req

    # ------------------------------------------------------------------ scheduling
    def poll(self) -> int:
        """One scheduling pass: retire, expire, admit, launch.  Returns the
        number of requests that changed state."""
        if self.broken is not None:
            return 0
        with self._lock:
            while self._incoming:
                self._queued.append(self._incoming.popleft())
        n = self._retire()
        n += self._expire()
        n += self._admit()
        n += self._launch()
        return n

    def _finish(self, req: Request, status: str, error: str = "") -> None:
        req.status, req.error = status, error
        if req.out is not None:
            self.b.free_out(req.rig, req.out)
            req.out = None
            self.mem_used -= self.b.frameset_bytes(req.rig)
        self.finished.append(req)

    def _retire(self) -> int:
        n = 0
        while self._inflight and self.b.ready(self._inflight[0].token):
            done = self._inflight.popleft()
            t = self.clock()
            for req in done.reqs:
                req.t_done = t
                req.status = "done"
                self._fail_run[req.rig] = 0
                if self.on_done is not None:
                    self.on_done(req)
                self._finish(req, "done")
                n += 1
        return n

    def _expire(self) -> int:
        if self.max_wait is None:
            return 0
        now, n = self.clock(), 0
        keep = collections.deque()
        for req in self._queued:
            if now - req.t_arrival > self.max_wait:
                self._waiting[req.rig] -= 1
                self._finish(req, "expired", f"waited {now - req.t_arrival:.4f} s")
                n += 1
            else:
                keep.append(req)
        self._queued = keep
        return n

    def _admit(self) -> int:
        n = 0
        while self._queued:
            req = self._queued[0]
            if req.rig in self.closed_rigs:
                self._queued.popleft()
                self._waiting[req.rig] -= 1
                self._finish(req, "rejected", "rig closed")
                continue
            need = self.b.frameset_bytes(req.rig)
            if self.mem_used + need > self.mem_budget:
                break
            self._queued.popleft()
            self._waiting[req.rig] -= 1
            req.out = self.b.alloc_out(req.rig)
            self.mem_used += need
            self.mem_peak = max(self.mem_peak, self.mem_used)
            req.t_admit = self.clock()
            req.status = "admitted"
            self._admitted[req.rig].append(req)
            n += 1
        return n

    def _launch(self) -> int:
        n = 0
        while len(self._inflight) < self.max_batches:
            for r in self.closed_rigs:
                while self._admitted[r]:
                    self._finish(self._admitted[r].popleft(), "rejected", "rig closed")
                    n += 1
            batch = [q[0] for q in self._admitted if q]
            if not batch:
                break
            while batch:
                try:
                    token = self.b.launch(batch)
                    break
                except BackendError as e:
                    refused = [r for r in batch if r.rig in e.rigs]
                    if not refused:
                        raise
                    for req in refused:
                        self._admitted[req.rig].popleft()
                        self._fail_run[req.rig] += 1
                        if self._fail_run[req.rig] >= self.max_failures:
                            self.closed_rigs.add(req.rig)
                        self._finish(req, "failed", str(e))
                        n += 1
                    batch = [r for r in batch if r.rig not in e.rigs]
                except Exception as e:  # device error: the context can no longer be trusted
                    self.broken = e
                    for req in batch:
                        self._admitted[req.rig].popleft()
                        self._finish(req, "failed", f"device error: {e}")
                    return n + len(batch)
            if not batch:
                continue
            t = self.clock()
            for req in batch:
                self._admitted[req.rig].popleft()
                req.t_launch = t
                req.status = "running"
            self._inflight.append(_Launch(token, batch))
            self.batch_sizes.append(len(batch))
            n += len(batch)
        return n

    # ------------------------------------------------------------------ driving
    def pending(self) -> int:
        with self._lock:
            inc = len(self._incoming)
        return inc + len(self._queued) + sum(len(q) for q in self._admitted) + sum(len(l.reqs) for l in self._inflight)

    def drain(self, timeout: float = 60.0, idle_sleep: float = 50e-6) -> None:
        """Poll until every submitted request has finished."""
        t0 = time.perf_counter()
        while self.pending() and self.broken is None:
            if self.poll() == 0:
                if time.perf_counter() - t0 > timeout:
                    raise TimeoutError(f"{self.pending()} requests still pending after {timeout} s")
                time.sleep(idle_sleep)

    def start(self, idle_sleep: float = 50e-6) -> None:
        """Run the scheduler on a background thread until stop()."""
        self._stop.clear()

        def loop():
            while not self._stop.is_set() and self.broken is None:
                if self.poll() == 0:
                    time.sleep(idle_sleep)

        self._thread = threading.Thread(target=loop, name="ringcorr-serve", daemon=True)
        self._thread.start()

    def stop(self, drain: bool = True, timeout: float = 60.0) -> None:
        if drain:
            t0 = time.perf_counter()
            while self.pending() and self.broken is None and time.perf_counter() - t0 < timeout:
                time.sleep(1e-3)
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
            self._thread = None
        if self.broken is None:
            self.drain(timeout)

    # ------------------------------------------------------------------ report
    def report(self) -> dict:
        done = [r for r in self.finished if r.status == "done"]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        counts = collections.Counter(r.status for r in self.finished)
        out = {s: counts.get(s, 0) for s in ("done", "failed", "expired", "rejected")}
        if done:
            t0 = min(r.t_arrival for r in done)
            t1 = max(r.t_done for r in done)
            px = sum(self.b.rig_pixels(r.rig) for r in done)
            out.update(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                       max_ms=float(lat.max() * 1e3), span_s=t1 - t0, pixels=px,
                       GPix_s=px / max(t1 - t0, 1e-12) / 1e9)
        out["mean_batch"] = float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0
        out["mem_peak"] = self.mem_peak
        return out


class GpuBackend(Backend):
    """The library behind the server: one context holding every rig's cameras
    (rig r = ring r), pooled output frames.  With lanes = 1, each batch is one
    rt_frameset_batch on one device stream.  With lanes > 1 (plain path), the
    batches go through the frame-set pipeline (rt_pipe_submit_batch): their
    statistics and estimates in order on one stream, their applies
    round-robin over `lanes` streams, so that consecutive batches overlap;
    tables and whole-frame statistics rotate over `depth` slots.  With a
    surrogate, the estimate of each frame-set goes through the network with
    the plain estimate as fallback (one stream)."""

    def __init__(self, rigs, opts=None, surrogate=None, stream=None, device="cuda", lanes=1, depth=4):
        import torch

        from . import rt
        from .surrogate import Workspace
        self.rt = rt
        self.torch = torch
        cams, self.idx = [], []
        for r, rig_cams in enumerate(rigs):
            ids = []
            for p, c in enumerate(rig_cams):
                cam = rt.Camera(c.width, c.height, c.channels, c.bit_depth, r, p)
                ids.append(len(cams))
                cams.append(cam.with_pitch(c.pitch_bytes) if getattr(c, "pitch_bytes", 0) else cam.with_pitch())
            self.idx.append(ids)
        self.n_rigs = len(rigs)
        self.cams = cams
        self.rig = rt.Rig(cams, opts or rt.Options(), device)
        self.masks = [sum(1 << i for i in ids) for ids in self.idx]
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.device = device
        self.surrogate = surrogate
        self.ws = Workspace(self.rig.sizes, device) if surrogate is not None else None
        self._pool = [[] for _ in range(self.n_rigs)]
        self._bytes = [sum(cams[i].height * cams[i].pitch_bytes for i in ids) for ids in self.idx]
        self._pixels = [sum(cams[i].width * cams[i].height for i in ids) for ids in self.idx]
        self.pipe = None
        if lanes > 1 and surrogate is None:
            self.pipe = rt.Pipe.for_rig(self.rig, depth=depth, lanes=lanes, group=1)
        # The apply work split timed for this context (autotune.tune, eager
        # launches as the batches issue them), if one is cached.
        from . import autotune
        self.tuned = autotune.apply_cached(self.rig)
        self.tuned_source = "cache" if self.tuned is not None else "default"

    def autotune(self, frames_per_rig, cache_path=None):
        """Time the apply work splits on this context with one frame-set of
        every rig (device frame lists), keep and cache the fastest."""
        from . import autotune
        frames = [f for r in range(self.n_rigs) for f in frames_per_rig[r]]
        outs = self.rig.alloc_frames()
        kw = {} if cache_path is None else {"cache_path": cache_path}
        self.tuned = autotune.tune(self.rig, [frames], [outs], **kw)
        self.tuned_source = "tuned"
        # Timing advanced every rig's estimator state: back to the initial one.
        b = self.rig.bufs
        b.params.zero_()
        b.params[..., 0] = 1.0
        b.valid.zero_()
        self.torch.cuda.synchronize()
        return self.tuned

    def frameset_bytes(self, rig: int) -> int:
        return self._bytes[rig]

    def rig_pixels(self, rig: int) -> int:
        return self._pixels[rig]

    def alloc_out(self, rig: int):
        if self._pool[rig]:
            return self._pool[rig].pop()
        t = self.torch
        return [t.empty((self.cams[i].height, self.cams[i].pitch_bytes), dtype=t.uint8, device=self.device)
                for i in self.idx[rig]]

    def free_out(self, rig: int, out) -> None:
        self._pool[rig].append(out)

    def rig_cams(self, rig: int) -> list:
        return [self.cams[i] for i in self.idx[rig]]

    def check(self, req: Request) -> str:
        """Why req's frames cannot be launched ("" if they can)."""
        ids = self.idx[req.rig]
        if req.frames is None or len(req.frames) != len(ids):
            return f"expected {len(ids)} frames"
        for n, (f, i) in enumerate(zip(req.frames, ids)):
            c = self.cams[i]
            if not (hasattr(f, "data_ptr") and f.is_cuda and f.dtype == self.torch.uint8
                    and tuple(f.shape) == (c.height, c.pitch_bytes) and f.is_contiguous()
                    and f.data_ptr() % 16 == 0):
                return f"camera frame {n} must be a contiguous uint8 device tensor of shape " \
                       f"({c.height}, {c.pitch_bytes}), 16-byte aligned"
        return ""

    def launch(self, batch: list[Request]):
        bad = {req.rig: f"rig {req.rig}: {msg}" for req in batch if (msg := self.check(req))}
        if bad:
            raise BackendError(list(bad), "; ".join(bad.values()))
        K = len(self.cams)
        frames, outs = [None] * K, [None] * K
        mask = 0
        for req in batch:
            mask |= self.masks[req.rig]
            for n, i in enumerate(self.idx[req.rig]):
                frames[i], outs[i] = req.frames[n], req.out[n]
        st = self.stream
        # The frames' producers: the launch stream waits for every ready event
        # (the pipeline's statistics stream waits for one event recorded after
        # those waits).
        ready = [req.ready for req in batch if req.ready is not None]
        for e in ready:
            st.wait_event(e)
        ev = self.torch.cuda.Event()
        if self.pipe is not None:
            merged = None
            if len(ready) == 1:
                merged = ready[0]
            elif ready:
                merged = self.torch.cuda.Event()
                merged.record(st)
            self.pipe.submit_batch(mask, frames, outs, st, ready_event=merged, done_event=ev)
            return ev
        if self.surrogate is None:
            self.rig.frameset_batch(mask, frames, outs, st)
        else:
            self.rig.set_active(mask)
            self.surrogate.frameset(self.rig, frames, outs, self.rig.bufs.whole_hist, self.ws, st)
        ev.record(st)
        return ev

    def ready(self, token) -> bool:
        return token.query()

    def wait(self, token) -> None:
        token.synchronize()

    def close(self) -> None:
        if self.pipe is not None:
            self.pipe.close()
        self.stream.synchronize()
        self.rig.close()


class ShardedBackend(Backend):
    """Rigs spread over several contexts, for more cameras than one context
    takes (RT_MAX_CAMS): rigs fill the contexts in order, each context a
    GpuBackend with its own device stream (and pipeline), so the contexts'
    work runs concurrently.  A batch is split by context: every context with
    a frame-set in it gets one launch, and the batch completes when all
    have.  A refused frame-set is refused before any context launches.
    shard_cls (default GpuBackend) builds a context's backend from its rigs,
    the options and the remaining keyword arguments."""

    def __init__(self, rigs, opts=None, max_cams: int | None = None, shard_cls=None, **kw):
        import copy
        self._copy = copy.copy
        if max_cams is None:
            from . import rt
            max_cams = rt.RT_MAX_CAMS
        shard_cls = shard_cls or GpuBackend
        groups, cur, n = [], [], 0
        for r, rig_cams in enumerate(rigs):
            if len(rig_cams) > max_cams:
                raise ValueError(f"rig {r} has {len(rig_cams)} cameras, more than a context takes ({max_cams})")
            if cur and n + len(rig_cams) > max_cams:
                groups.append(cur)
                cur, n = [], 0
            cur.append(r)
            n += len(rig_cams)
        if cur:
            groups.append(cur)
        self.shards = []
        try:
            for g in groups:
                self.shards.append(shard_cls([rigs[r] for r in g], opts, **kw))
        except Exception:
            self.close()
            raise
        self.where = {r: (s, l) for s, g in enumerate(groups) for l, r in enumerate(g)}
        self.n_rigs = len(rigs)

    def _at(self, rig: int):
        s, l = self.where[rig]
        return self.shards[s], l

    def rig_cams(self, rig: int) -> list:
        b, l = self._at(rig)
        return b.rig_cams(l)

    def frameset_bytes(self, rig: int) -> int:
        b, l = self._at(rig)
        return b.frameset_bytes(l)

    def rig_pixels(self, rig: int) -> int:
        b, l = self._at(rig)
        return b.rig_pixels(l)

    def alloc_out(self, rig: int):
        b, l = self._at(rig)
        return b.alloc_out(l)

    def free_out(self, rig: int, out) -> None:
        b, l = self._at(rig)
        b.free_out(l, out)

    def launch(self, batch: list[Request]):
        parts, bad = {}, {}
        for req in batch:
            s, l = self.where[req.rig]
            local = self._copy(req)
            local.rig = l
            msg = self.shards[s].check(local)
            if msg:
                bad[req.rig] = f"rig {req.rig}: {msg}"
            parts.setdefault(s, []).append(local)
        if bad:
            raise BackendError(list(bad), "; ".join(bad.values()))
        return [self.shards[s].launch(part) for s, part in sorted(parts.items())]

    def ready(self, token) -> bool:
        return all(ev.query() for ev in token)

    def wait(self, token) -> None:
        for ev in token:
            ev.synchronize()

    def close(self) -> None:
        for b in self.shards:
            b.close()
        self.shards = []
