"""ctypes binding of libringcorr.so (argument marshalling only).

The functions below carry the names of the C-ABI in include/ringcorr.h and do
nothing but convert Python / torch arguments into the C structs and pointers;
every step of the correction runs in the library's HIP kernels.  torch is
used for device memory and streams only.

The library must have been built (python -m paper_1910_03517_amd.build);
loading fails loudly otherwise - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libringcorr.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EUNSUPPORTED, RT_ESTATE = 0, -1, -2, -3, -4, -5
RT_MODE_STANDARD, RT_MODE_SMOOTHING = 0, 1
RT_FIT_MOMENTS, RT_FIT_QUANTILE = 0, 1
RT_MAX_CAMS = 64
CSLOTS, NBINS = 3, 256

EXPORTED = ["rt_ctx_create", "rt_ctx_destroy", "rt_ctx_sizes", "rt_stats", "rt_estimate",
            "rt_build_lut", "rt_apply", "rt_frameset", "rt_frameset_batch", "rt_frameset_ahead", "rt_ctx_set_active", "rt_ctx_check", "rt_ctx_tune", "rt_ctx_tuning",
            "rt_stream_copy", "rt_ctx_timing", "rt_ctx_apply_times", "rt_graph_create", "rt_graph_launch",
            "rt_graph_destroy", "rt_pipe_create", "rt_pipe_submit", "rt_pipe_destroy",
            "rt_pipe_create_lanes", "rt_pipe_join", "rt_pipe_submit_batch", "rt_pipe_submit_n",
            "rt_pipe_set_fuse", "rt_ctx_apply_sets", "rt_graph_set_frames", "rt_pipe_set_removal", "rt_apply_sets",
            "rt_surrogate_features", "rt_estimate_new", "rt_surrogate_targets", "rt_surrogate_select",
            "rt_surrogate_frameset",
            "rt_mlp_forward", "rt_mlp_backward", "rt_mlp_adam", "rt_mlp_mse", "rt_gather_rows", "rt_mlp_train",
            "rt_motion_stats", "rt_estimate_removal", "rt_frameset_removal", "rt_seam_cost",
            "rt_surrogate_frameset_static", "rt_attention",
            "rt_cross_stats", "rt_estimate_cross", "rt_build_cross", "rt_apply_cross", "rt_frameset_cross",
            "rt_status_str", "rt_last_error"]
RT_METHOD_NONE, RT_METHOD_REMOVAL, RT_METHOD_SMOOTHING = 0, 1, 2
MLP_IN, MLP_HID, MLP_OUT = 576, 256, 6


class rt_camera_desc(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32), ("channels", ct.c_int32),
                ("bit_depth", ct.c_int32), ("ring", ct.c_int32), ("pos", ct.c_int32),
                ("pitch_bytes", ct.c_int64)]


class rt_opts(ct.Structure):
    _fields_ = [("n_blocks", ct.c_int32), ("band_width", ct.c_int32), ("closed_ring", ct.c_int32),
                ("mode", ct.c_int32), ("ema_alpha", ct.c_double), ("a_min", ct.c_double),
                ("a_max", ct.c_double), ("vblend", ct.c_int32), ("fit", ct.c_int32)]


class rt_sizes(ct.Structure):
    _fields_ = [("n_cams", ct.c_int32), ("n_blocks", ct.c_int32), ("w_max", ct.c_int32),
                ("reserved", ct.c_int32), ("band_hist", ct.c_int64), ("band_sums", ct.c_int64),
                ("whole_hist", ct.c_int64), ("whole_sums", ct.c_int64), ("params", ct.c_int64),
                ("valid", ct.c_int64), ("lut8", ct.c_int64), ("q16", ct.c_int64), ("weights", ct.c_int64)]


class rt_stats_buf(ct.Structure):
    _fields_ = [("band_hist", ct.c_void_p), ("band_sums", ct.c_void_p),
                ("whole_hist", ct.c_void_p), ("whole_sums", ct.c_void_p)]


class rt_params_buf(ct.Structure):
    _fields_ = [("params", ct.c_void_p), ("valid", ct.c_void_p)]


class rt_lut_buf(ct.Structure):
    _fields_ = [("lut8", ct.c_void_p), ("q16", ct.c_void_p), ("weights", ct.c_void_p)]


class rt_mlp(ct.Structure):
    _fields_ = [("w1", ct.c_void_p), ("b1", ct.c_void_p), ("w2", ct.c_void_p), ("b2", ct.c_void_p),
                ("w3", ct.c_void_p), ("b3", ct.c_void_p)]


class rt_mlp_work(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in ("xb", "tb", "h1", "h2", "y", "dy", "dz1", "dz2")]


class rt_surrogate_work(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in ("X", "H1", "H2", "Y", "p_new", "status", "used", "residual")]


class rt_removal_opts(ct.Structure):
    _fields_ = [("tau", ct.c_int32), ("reserved", ct.c_int32), ("min_kept", ct.c_double)]


class rt_cross_buf(ct.Structure):
    _fields_ = [("cross", ct.c_void_p), ("params3", ct.c_void_p), ("valid3", ct.c_void_p), ("q3", ct.c_void_p),
                ("weights", ct.c_void_p)]


class rt_attention_opts(ct.Structure):
    _fields_ = [("tau", ct.c_int32), ("cell", ct.c_int32), ("m", ct.c_int32), ("theta", ct.c_int32)]


class RtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ringcorr status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ct.CDLL:
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1910_03517_amd.build`")
    lib = ct.CDLL(path)
    P = ct.c_void_p
    lib.rt_ctx_create.argtypes = [ct.POINTER(rt_camera_desc), ct.c_int32, ct.POINTER(rt_opts), ct.POINTER(P)]
    lib.rt_ctx_destroy.argtypes = [P]
    lib.rt_ctx_sizes.argtypes = [P, ct.POINTER(rt_sizes)]
    lib.rt_stats.argtypes = [P, ct.POINTER(P), ct.POINTER(rt_stats_buf), P]
    lib.rt_estimate.argtypes = [P, ct.POINTER(rt_stats_buf), ct.POINTER(rt_params_buf), P]
    lib.rt_build_lut.argtypes = [P, ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf), P]
    lib.rt_apply.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_lut_buf), ct.POINTER(rt_stats_buf), P]
    lib.rt_apply_sets.argtypes = [P, ct.c_int32, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_lut_buf),
                                  ct.POINTER(rt_stats_buf), P]
    lib.rt_frameset.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_stats_buf),
                                ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf), P]
    lib.rt_frameset_batch.argtypes = [P, ct.c_uint64, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_stats_buf),
                                      ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf), P]
    lib.rt_frameset_ahead.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_lut_buf),
                                      ct.POINTER(rt_stats_buf), ct.POINTER(P), ct.POINTER(rt_lut_buf),
                                      ct.POINTER(rt_stats_buf), ct.POINTER(rt_stats_buf), ct.POINTER(rt_params_buf), P]
    lib.rt_ctx_set_active.argtypes = [P, ct.c_uint64]
    lib.rt_ctx_check.argtypes = [P]
    lib.rt_ctx_tune.argtypes = [P, ct.c_int32, ct.c_int32]
    I = ct.POINTER(ct.c_int32)
    lib.rt_ctx_tuning.argtypes = [P, I, I, I]
    lib.rt_stream_copy.argtypes = [P, P, ct.c_int64, ct.c_int32, P]
    lib.rt_ctx_timing.argtypes = [P, ct.c_int32, ct.c_int32]
    lib.rt_graph_create.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_lut_buf), ct.POINTER(rt_stats_buf),
                                    ct.POINTER(P), ct.POINTER(rt_lut_buf), ct.POINTER(rt_stats_buf),
                                    ct.POINTER(rt_params_buf), ct.POINTER(P)]
    lib.rt_graph_launch.argtypes = [P, P]
    lib.rt_graph_set_frames.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(P)]
    lib.rt_pipe_create.argtypes = [P, ct.c_int32, ct.POINTER(rt_stats_buf), ct.POINTER(rt_params_buf),
                                   ct.POINTER(rt_lut_buf), ct.POINTER(rt_stats_buf), ct.POINTER(P)]
    lib.rt_pipe_submit.argtypes = [P, ct.POINTER(P), ct.POINTER(P), P, P, ct.POINTER(ct.c_int32)]
    lib.rt_pipe_submit_n.argtypes = [P, ct.c_int32, ct.POINTER(P), ct.POINTER(P), P, ct.POINTER(ct.c_int32),
                                     ct.POINTER(ct.c_int32)]
    lib.rt_pipe_destroy.argtypes = [P]
    lib.rt_pipe_set_fuse.argtypes = [P, ct.c_int32]
    lib.rt_pipe_set_removal.argtypes = [P, ct.POINTER(rt_removal_opts), P, P]
    lib.rt_ctx_apply_sets.argtypes = [P, ct.POINTER(ct.c_int32), ct.c_int32, ct.POINTER(ct.c_int32)]
    lib.rt_pipe_create_lanes.argtypes = [P, ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(rt_stats_buf),
                                         ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf), ct.POINTER(rt_stats_buf),
                                         ct.POINTER(P)]
    lib.rt_pipe_join.argtypes = [P, P]
    lib.rt_pipe_submit_batch.argtypes = [P, ct.c_uint64, ct.POINTER(P), ct.POINTER(P), P, P, P,
                                         ct.POINTER(ct.c_int32)]
    M = ct.POINTER(rt_mlp)
    lib.rt_surrogate_features.argtypes = [P, ct.POINTER(rt_stats_buf), P, P]
    lib.rt_estimate_new.argtypes = [P, ct.POINTER(rt_stats_buf), P, P, P]
    lib.rt_surrogate_targets.argtypes = [P, P, P, P, P, P]
    lib.rt_surrogate_select.argtypes = [P, P, P, P, ct.c_float, ct.POINTER(rt_params_buf), P, P, P]
    lib.rt_surrogate_frameset.argtypes = [P, M, ct.c_float, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_stats_buf),
                                          P, ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf),
                                          ct.POINTER(rt_surrogate_work), P]
    lib.rt_surrogate_frameset_static.argtypes = [P, M, ct.c_float, ct.POINTER(P), ct.POINTER(P),
                                                 ct.POINTER(rt_stats_buf), P, ct.POINTER(rt_params_buf),
                                                 ct.POINTER(rt_lut_buf), P]
    lib.rt_mlp_forward.argtypes = [M, P, ct.c_int32, P, P, P, P]
    lib.rt_mlp_backward.argtypes = [M, P, P, P, P, P, ct.c_int32, M, P, P, P, P]
    lib.rt_mlp_adam.argtypes = [M, M, M, M, ct.c_int32, ct.c_float, ct.c_float, ct.c_float, ct.c_float, P]
    lib.rt_mlp_mse.argtypes = [P, P, ct.c_int32, P, P]
    lib.rt_gather_rows.argtypes = [P, ct.c_int32, P, ct.c_int32, P, P]
    M = ct.POINTER(rt_mlp)
    lib.rt_mlp_train.argtypes = [M, M, M, M, P, P, ct.c_int32, P, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_float,
                                 ct.c_float, ct.c_float, ct.c_float, ct.POINTER(rt_mlp_work), P, P]
    R = ct.POINTER(rt_removal_opts)
    lib.rt_motion_stats.argtypes = [P, ct.POINTER(P), ct.POINTER(P), R, ct.POINTER(rt_stats_buf), P, P]
    lib.rt_estimate_removal.argtypes = [P, ct.POINTER(rt_stats_buf), P, R, ct.POINTER(rt_params_buf), P, P]
    lib.rt_frameset_removal.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(P), R, ct.POINTER(rt_stats_buf),
                                        P, ct.POINTER(rt_params_buf), ct.POINTER(rt_lut_buf), P, P]
    lib.rt_graph_destroy.argtypes = [P]
    lib.rt_seam_cost.argtypes = [P, ct.POINTER(P), ct.c_int32, P, P, P, ct.c_int32, P]
    lib.rt_attention.argtypes = [P, ct.POINTER(P), ct.POINTER(P), ct.POINTER(rt_attention_opts), P, P, P, P]
    lib.rt_ctx_apply_times.argtypes = [P, ct.POINTER(ct.c_float), ct.c_int32, ct.POINTER(ct.c_int32)]
    X = ct.POINTER(rt_cross_buf)
    S = ct.POINTER(rt_stats_buf)
    lib.rt_cross_stats.argtypes = [P, ct.POINTER(P), X, P]
    lib.rt_estimate_cross.argtypes = [P, S, X, P]
    lib.rt_build_cross.argtypes = [P, X, P]
    lib.rt_apply_cross.argtypes = [P, ct.POINTER(P), ct.POINTER(P), X, S, P]
    lib.rt_frameset_cross.argtypes = [P, ct.POINTER(P), ct.POINTER(P), S, X, P]
    for name in EXPORTED:
        getattr(lib, name).restype = ct.c_int32
    lib.rt_status_str.argtypes = [ct.c_int32]
    lib.rt_status_str.restype = ct.c_char_p
    lib.rt_last_error.argtypes = []
    lib.rt_last_error.restype = ct.c_char_p
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != RT_OK:
        raise RtError(status, load().rt_last_error().decode())


def _stream_handle(stream) -> ct.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def ptr_array_n(frame_sets) -> ct.Array:
    """Device pointers of several frame-sets back to back (rt_pipe_submit_n's layout)."""
    flat = [t for fs in frame_sets for t in fs]
    return _ptr_array(flat)


def _ptr_array(tensors) -> ct.Array:
    """Device pointers of tensors (or plain ints); None becomes NULL."""
    arr = (ct.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else (t.data_ptr() if hasattr(t, "data_ptr") else int(t))
    return arr


def _p(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------- C-ABI calls

def rt_ctx_create(cams, opts: "Options") -> ct.c_void_p:
    lib = load()
    arr = (rt_camera_desc * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = rt_camera_desc(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos, c.pitch_bytes)
    o = opts.to_c()
    ctx = ct.c_void_p()
    _check(lib.rt_ctx_create(arr, len(cams), ct.byref(o), ct.byref(ctx)))
    return ctx


def rt_ctx_destroy(ctx) -> None:
    _check(load().rt_ctx_destroy(ctx))


def rt_ctx_sizes(ctx) -> rt_sizes:
    s = rt_sizes()
    _check(load().rt_ctx_sizes(ctx, ct.byref(s)))
    return s


def rt_ctx_check(ctx) -> None:
    _check(load().rt_ctx_check(ctx))


def rt_ctx_tune(ctx, tile_rows: int, grid: int = 0) -> None:
    _check(load().rt_ctx_tune(ctx, tile_rows, grid))


def rt_ctx_tuning(ctx) -> tuple[int, int, int]:
    a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(load().rt_ctx_tuning(ctx, ct.byref(a), ct.byref(b), ct.byref(c)))
    return a.value, b.value, c.value


class LutSet:
    """One slot of tables (lut8, q16, weights) of a context's sizes."""

    def __init__(self, sizes: rt_sizes, device="cuda"):
        import torch
        K, NB, WM = sizes.n_cams, sizes.n_blocks, max(sizes.w_max, 1)
        self.lut8 = torch.zeros((K, 2, NB, CSLOTS, NBINS), dtype=torch.uint8, device=device)
        self.q16 = torch.zeros((K, 2, NB, CSLOTS, 2), dtype=torch.int64, device=device)
        self.weights = torch.zeros((K, WM), dtype=torch.int16, device=device)


class WholeSet:
    """One slot of whole-frame statistics (whole_hist, whole_sums) of a context's sizes."""

    def __init__(self, sizes: rt_sizes, device="cuda"):
        import torch
        K = sizes.n_cams
        self.whole_hist = torch.zeros((K, CSLOTS, NBINS), dtype=torch.int32, device=device)
        self.whole_sums = torch.zeros((K, CSLOTS, 3), dtype=torch.int64, device=device)


class Pipe:
    """rt_pipe, the frame-set pipeline: per frame-set the kernels of
    rt_frameset, split over HIP streams by the library.  The band statistics,
    estimate and tables of consecutive frame-sets run in order on the
    pipeline's own stream, ahead of the bandwidth-bound applies, which go
    round-robin over `lanes` streams (the caller's first), issued `group`
    frame-sets at a time, so that the estimate of frame-set t+1 overlaps the
    apply of t and, with lanes > 1, consecutive applies overlap each other.
    Tables and whole-frame statistics rotate over `depth` slots (>= lanes,
    >= group); band statistics and the estimator state are single buffers,
    so the results are exactly those of consecutive rt_frameset calls.  Call
    join() before depending on the results of submitted frame-sets.

    luts / wholes are sequences of `depth` objects with lut8, q16, weights /
    whole_hist, whole_sums tensors; bufs provides band_hist, band_sums,
    params, valid.  Pipe.for_rig allocates the slots of a Rig."""

    @classmethod
    def for_rig(cls, rig: "Rig", depth: int = 2, lanes: int = 1, group: int = 1, fuse: bool = False) -> "Pipe":
        luts = [LutSet(rig.sizes, rig.device) for _ in range(depth)]
        wholes = [WholeSet(rig.sizes, rig.device) for _ in range(depth)]
        p = cls(rig.ctx, rig.bufs, luts, wholes, lanes=lanes, group=group, fuse=fuse)
        p.luts, p.whole = luts, wholes
        return p

    def __init__(self, ctx, bufs, luts, wholes, lanes: int = 1, group: int = 1, fuse: bool = False):
        depth = len(luts)
        assert len(wholes) == depth
        la = (rt_lut_buf * depth)(*[rt_lut_buf(_p(l.lut8), _p(l.q16), _p(l.weights)) for l in luts])
        wa = (rt_stats_buf * depth)(*[rt_stats_buf(None, None, _p(w.whole_hist), _p(w.whole_sums)) for w in wholes])
        bb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), None, None)
        pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
        h = ct.c_void_p()
        _check(load().rt_pipe_create_lanes(ctx, depth, lanes, group, ct.byref(bb), ct.byref(pb), la, wa,
                                           ct.byref(h)))
        self.handle = h
        self.depth = depth
        self.lanes = lanes
        self.group = group
        self.fuse = False
        self._keep = (bufs, luts, wholes)
        self._slot = ct.c_int32()
        if fuse:
            self.set_fuse(True)

    def set_removal(self, kept_sums, method=None, tau: int = 20, min_kept: float = 0.25, on: bool = True) -> None:
        """rt_pipe_set_removal: later submits estimate with object removal
        against each camera's previously submitted frame (kept_sums int64
        [K][2][NB][3][3], method uint8 [K][2][NB] or None); on=False turns it
        off.  A submitted frame-set's inputs must stay unchanged until the
        next frame-set's apply has finished."""
        if not on:
            _check(load().rt_pipe_set_removal(self.handle, None, None, None))
            self._removal = None
            return
        ro = rt_removal_opts(tau, 0, min_kept)
        _check(load().rt_pipe_set_removal(self.handle, ct.byref(ro), _p(kept_sums),
                                          _p(method) if method is not None else None))
        self._removal = (kept_sums, method)

    def set_fuse(self, fuse: bool) -> None:
        """rt_pipe_set_fuse: a group's applies as launches of up to 4
        frame-sets on one lane, groups taking the lanes in turn."""
        _check(load().rt_pipe_set_fuse(self.handle, int(bool(fuse))))
        self.fuse = bool(fuse)

    def submit(self, frames, out_frames, stream=None, frame_ptrs=None, out_ptrs=None, ready_event=None) -> int:
        """Enqueue one frame-set; returns its slot.  frame_ptrs / out_ptrs may
        pass prebuilt pointer arrays (see ptr_array) to save host time;
        ready_event (a torch.cuda.Event recorded after the frames were written)
        orders the statistics after the frames' producer."""
        fa = frame_ptrs if frame_ptrs is not None else _ptr_array(frames)
        oa = out_ptrs if out_ptrs is not None else _ptr_array(out_frames)
        ev = ct.c_void_p(ready_event.cuda_event) if ready_event is not None else None
        _check(load().rt_pipe_submit(self.handle, fa, oa, _stream_handle(stream), ev, ct.byref(self._slot)))
        return self._slot.value

    def submit_n(self, frames_list, outs_list, stream=None, ptrs=None) -> list:
        """Several frame-sets in one library call (rt_pipe_submit_n); ptrs may
        pass prebuilt (frames, outs, n) from ptr_array_n (frames_list and
        outs_list are then ignored).  Returns the slots."""
        if ptrs is not None:
            fa, oa, n = ptrs
        else:
            fa, oa, n = ptr_array_n(frames_list), ptr_array_n(outs_list), len(frames_list)
        slots = (ct.c_int32 * n)()
        done = ct.c_int32()
        _check(load().rt_pipe_submit_n(self.handle, n, fa, oa, _stream_handle(stream), slots, ct.byref(done)))
        return list(slots)

    def submit_batch(self, active: int, frames, out_frames, stream=None, ready_event=None, done_event=None) -> int:
        """submit() for the cameras in bitmask `active` (whole rings); entries of
        the other cameras may be None.  done_event (a torch.cuda.Event) is
        recorded right after this frame-set's apply (pipelines with group 1)."""
        ev = ct.c_void_p(ready_event.cuda_event) if ready_event is not None else None
        if done_event is not None and not done_event.cuda_event:
            # torch creates an event's HIP handle at its first record; the
            # library's record after the apply supersedes this one.
            import torch
            done_event.record(stream if stream is not None else torch.cuda.current_stream())
        dv = ct.c_void_p(done_event.cuda_event) if done_event is not None else None
        _check(load().rt_pipe_submit_batch(self.handle, ct.c_uint64(active), _ptr_array(frames),
                                           _ptr_array(out_frames), _stream_handle(stream), ev, dv,
                                           ct.byref(self._slot)))
        return self._slot.value

    def join(self, stream=None) -> None:
        """Issue pending applies; order `stream` after every frame-set submitted so far."""
        _check(load().rt_pipe_join(self.handle, _stream_handle(stream)))

    def close(self) -> None:
        if self.handle is not None:
            load().rt_pipe_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MlpTensors:
    """One set of network tensors on the device (weights, gradients or moments)."""
    NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")
    SHAPES = {"w1": (MLP_IN, MLP_HID), "b1": (MLP_HID,), "w2": (MLP_HID, MLP_HID), "b2": (MLP_HID,),
              "w3": (MLP_HID, MLP_OUT), "b3": (MLP_OUT,)}

    def __init__(self, arrays: dict | None = None, device="cuda"):
        import torch
        for n in self.NAMES:
            if arrays is None:
                t = torch.zeros(self.SHAPES[n], dtype=torch.float32, device=device)
            else:
                t = torch.as_tensor(np.asarray(arrays[n], np.float32), device=device).contiguous()
                assert tuple(t.shape) == self.SHAPES[n], n
            setattr(self, n, t)

    def c(self) -> rt_mlp:
        return rt_mlp(*[_p(getattr(self, n)) for n in self.NAMES])

    def host(self) -> dict:
        return {n: getattr(self, n).cpu().numpy().copy() for n in self.NAMES}


def rt_surrogate_features(ctx, band_hist, whole_hist, X, stream=None) -> None:
    sb = rt_stats_buf(_p(band_hist), None, _p(whole_hist), None)
    _check(load().rt_surrogate_features(ctx, ct.byref(sb), _p(X), _stream_handle(stream)))


def rt_estimate_new(ctx, band_sums, p_new, status, stream=None) -> None:
    sb = rt_stats_buf(None, _p(band_sums), None, None)
    _check(load().rt_estimate_new(ctx, ct.byref(sb), _p(p_new), _p(status), _stream_handle(stream)))


def rt_surrogate_targets(ctx, p_new, status, T, mask, stream=None) -> None:
    _check(load().rt_surrogate_targets(ctx, _p(p_new), _p(status), _p(T), _p(mask), _stream_handle(stream)))


def rt_surrogate_select(ctx, Y, p_new, status, tol, params, valid, used, residual, stream=None) -> None:
    pb = rt_params_buf(_p(params), _p(valid))
    _check(load().rt_surrogate_select(ctx, _p(Y), _p(p_new), _p(status), float(tol), ct.byref(pb), _p(used),
                                      _p(residual), _stream_handle(stream)))


def rt_surrogate_frameset(ctx, w: MlpTensors, tol, frames, out_frames, bufs: "Buffers", whole_hist_prev, work,
                          stream=None) -> None:
    """work: any object with X, H1, H2, Y, p_new, status, used, residual tensors."""
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    lb = rt_lut_buf(_p(bufs.lut8), _p(bufs.q16), _p(bufs.weights))
    wk = rt_surrogate_work(*[_p(getattr(work, n)) for n, _ in rt_surrogate_work._fields_])
    _check(load().rt_surrogate_frameset(ctx, ct.byref(w.c()), float(tol), _ptr_array(frames), _ptr_array(out_frames),
                                        ct.byref(sb), _p(whole_hist_prev), ct.byref(pb), ct.byref(lb), ct.byref(wk),
                                        _stream_handle(stream)))


def rt_surrogate_frameset_static(ctx, w: MlpTensors, tol, frames, out_frames, bufs: "Buffers", whole_hist_prev,
                                 stream=None) -> None:
    """rt_surrogate_frameset with the library's static workspace (allocates nothing)."""
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    lb = rt_lut_buf(_p(bufs.lut8), _p(bufs.q16), _p(bufs.weights))
    _check(load().rt_surrogate_frameset_static(ctx, ct.byref(w.c()), float(tol), _ptr_array(frames),
                                               _ptr_array(out_frames), ct.byref(sb), _p(whole_hist_prev),
                                               ct.byref(pb), ct.byref(lb), _stream_handle(stream)))


def rt_mlp_forward(w: MlpTensors, X, n, H1, H2, Y, stream=None) -> None:
    _check(load().rt_mlp_forward(ct.byref(w.c()), _p(X), n, _p(H1), _p(H2), _p(Y), _stream_handle(stream)))


def rt_mlp_backward(w: MlpTensors, X, H1, H2, Y, T, n, grad: MlpTensors, dY, dZ1, dZ2, stream=None) -> None:
    _check(load().rt_mlp_backward(ct.byref(w.c()), _p(X), _p(H1), _p(H2), _p(Y), _p(T), n, ct.byref(grad.c()),
                                  _p(dY), _p(dZ1), _p(dZ2), _stream_handle(stream)))


def rt_mlp_adam(w: MlpTensors, grad: MlpTensors, m: MlpTensors, v: MlpTensors, step: int, lr: float,
                beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(load().rt_mlp_adam(ct.byref(w.c()), ct.byref(grad.c()), ct.byref(m.c()), ct.byref(v.c()), step, lr,
                              beta1, beta2, eps, _stream_handle(stream)))


def rt_mlp_mse(Y, T, n, out, stream=None) -> None:
    _check(load().rt_mlp_mse(_p(Y), _p(T), n, _p(out), _stream_handle(stream)))


def rt_gather_rows(src, row_len, idx, n, dst, stream=None) -> None:
    _check(load().rt_gather_rows(_p(src), row_len, _p(idx), n, _p(dst), _stream_handle(stream)))


def rt_mlp_train(w, g, m, v, X, T, idx, batch: int, n_steps: int, step0: int, lr: float, work: dict, losses,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    """n_steps Adam steps on mini-batches idx[s*batch:(s+1)*batch] of (X, T); work: dict of the
    rt_mlp_work tensors; losses: device float32 [n_steps]."""
    wk = rt_mlp_work(*[_p(work[n]) for n in ("xb", "tb", "h1", "h2", "y", "dy", "dz1", "dz2")])
    _check(load().rt_mlp_train(ct.byref(w.c()), ct.byref(g.c()), ct.byref(m.c()), ct.byref(v.c()), _p(X), _p(T),
                               int(X.shape[0]), _p(idx), batch, n_steps, step0, lr, beta1, beta2, eps,
                               ct.byref(wk), _p(losses), _stream_handle(stream)))


def ptr_array(tensors) -> ct.Array:
    """Prebuilt C array of device pointers, reusable across calls."""
    return _ptr_array(tensors)


class Graph:
    """A captured frame-set (rt_graph_create); launch() replays it."""

    def __init__(self, ctx, frames, out_frames, lut, whole, bufs, next_frames=None, next_lut=None):
        lb = rt_lut_buf(_p(lut.lut8), _p(lut.q16), _p(lut.weights))
        wb = rt_stats_buf(None, None, _p(whole.whole_hist), _p(whole.whole_sums))
        bb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), None, None)
        pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
        nf = _ptr_array(next_frames) if next_frames is not None else None
        nl = ct.byref(rt_lut_buf(_p(next_lut.lut8), _p(next_lut.q16), _p(next_lut.weights))) if next_lut is not None else None
        h = ct.c_void_p()
        _check(load().rt_graph_create(ctx, _ptr_array(frames), _ptr_array(out_frames), ct.byref(lb), ct.byref(wb),
                                      nf, nl, ct.byref(bb), ct.byref(pb), ct.byref(h)))
        self.handle = h
        self._keep = (frames, out_frames, lut, whole, bufs, next_frames, next_lut)

    def launch(self, stream=None) -> None:
        _check(load().rt_graph_launch(self.handle, _stream_handle(stream)))

    def set_frames(self, frames, out_frames, next_frames=None, frame_ptrs=None, out_ptrs=None,
                   next_ptrs=None) -> None:
        """rt_graph_set_frames: later launches read `frames`, write
        `out_frames` (and, two-branch, gather the statistics of
        `next_frames`); prebuilt pointer arrays (ptr_array) may be passed
        instead.  The caller keeps the tensors alive while launches use them."""
        fa = frame_ptrs if frame_ptrs is not None else _ptr_array(frames)
        oa = out_ptrs if out_ptrs is not None else _ptr_array(out_frames)
        na = next_ptrs if next_ptrs is not None else (_ptr_array(next_frames) if next_frames is not None else None)
        _check(load().rt_graph_set_frames(self.handle, fa, oa, na))

    def close(self) -> None:
        if self.handle is not None:
            load().rt_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rt_ctx_timing(ctx, slots: int, every: int = 1) -> None:
    _check(load().rt_ctx_timing(ctx, slots, every))


def rt_ctx_apply_times(ctx, max_n: int) -> list[float]:
    buf = (ct.c_float * max(max_n, 1))()
    n = ct.c_int32()
    _check(load().rt_ctx_apply_times(ctx, buf, max_n, ct.byref(n)))
    return [buf[i] for i in range(n.value)]


def rt_ctx_apply_sets(ctx, max_n: int) -> list[int]:
    """Frame-sets covered by each launch that rt_ctx_apply_times reports."""
    buf = (ct.c_int32 * max(max_n, 1))()
    n = ct.c_int32()
    _check(load().rt_ctx_apply_sets(ctx, buf, max_n, ct.byref(n)))
    return [buf[i] for i in range(n.value)]


def rt_stream_copy(dst, src, nbytes: int, vec_bytes: int = 16, stream=None) -> None:
    _check(load().rt_stream_copy(ct.c_void_p(dst.data_ptr()), ct.c_void_p(src.data_ptr()), nbytes, vec_bytes,
                                 _stream_handle(stream)))


def rt_stats(ctx, frames, band_hist, band_sums, whole_hist=None, whole_sums=None, stream=None) -> None:
    sb = rt_stats_buf(_p(band_hist), _p(band_sums), _p(whole_hist), _p(whole_sums))
    _check(load().rt_stats(ctx, _ptr_array(frames), ct.byref(sb), _stream_handle(stream)))


def rt_estimate(ctx, band_hist, band_sums, params, valid, stream=None) -> None:
    sb = rt_stats_buf(_p(band_hist), _p(band_sums), None, None)
    pb = rt_params_buf(_p(params), _p(valid))
    _check(load().rt_estimate(ctx, ct.byref(sb), ct.byref(pb), _stream_handle(stream)))


def rt_build_lut(ctx, params, valid, lut8, q16, weights, stream=None) -> None:
    pb = rt_params_buf(_p(params), _p(valid))
    lb = rt_lut_buf(_p(lut8), _p(q16), _p(weights))
    _check(load().rt_build_lut(ctx, ct.byref(pb), ct.byref(lb), _stream_handle(stream)))


def rt_apply_sets(ctx, frames_list, outs_list, luts, wholes, stream=None, ptrs=None) -> None:
    """rt_apply_sets: the applies (with whole-frame statistics) of len(luts)
    frame-sets in one launch; luts / wholes are LutSet / WholeSet objects,
    ptrs may pass prebuilt (frames, outs) arrays from ptr_array_n."""
    n = len(luts)
    fa, oa = ptrs if ptrs is not None else (ptr_array_n(frames_list), ptr_array_n(outs_list))
    la = (rt_lut_buf * n)(*[rt_lut_buf(_p(l.lut8), _p(l.q16), _p(l.weights)) for l in luts])
    wa = (rt_stats_buf * n)(*[rt_stats_buf(None, None, _p(w.whole_hist), _p(w.whole_sums)) for w in wholes])
    _check(load().rt_apply_sets(ctx, n, fa, oa, la, wa, _stream_handle(stream)))


def rt_apply(ctx, frames, out_frames, lut8, q16, weights, whole_hist=None, whole_sums=None, stream=None) -> None:
    lb = rt_lut_buf(_p(lut8), _p(q16), _p(weights))
    wb = None
    if whole_hist is not None or whole_sums is not None:
        wb = ct.byref(rt_stats_buf(None, None, _p(whole_hist), _p(whole_sums)))
    _check(load().rt_apply(ctx, _ptr_array(frames), _ptr_array(out_frames), ct.byref(lb), wb,
                           _stream_handle(stream)))


def rt_frameset(ctx, frames, out_frames, bufs: "Buffers", stream=None) -> None:
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    lb = rt_lut_buf(_p(bufs.lut8), _p(bufs.q16), _p(bufs.weights))
    _check(load().rt_frameset(ctx, _ptr_array(frames), _ptr_array(out_frames), ct.byref(sb), ct.byref(pb),
                              ct.byref(lb), _stream_handle(stream)))


def rt_frameset_batch(ctx, active: int, frames, out_frames, bufs: "Buffers", stream=None) -> None:
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    lb = rt_lut_buf(_p(bufs.lut8), _p(bufs.q16), _p(bufs.weights))
    _check(load().rt_frameset_batch(ctx, ct.c_uint64(active), _ptr_array(frames), _ptr_array(out_frames),
                                    ct.byref(sb), ct.byref(pb), ct.byref(lb), _stream_handle(stream)))


def rt_frameset_ahead(ctx, frames, out_frames, lut, whole, next_frames, next_lut, next_whole,
                      bufs: "Buffers", stream=None, ptrs=None) -> None:
    """rt_frameset_ahead: the apply of frame-set t (frames -> out_frames with
    LutSet `lut`, statistics into WholeSet `whole`; frames None: none) and,
    in the same launch, the estimate of frame-set t + 1 (next_frames into
    bufs' band statistics and estimator state, tables into `next_lut`,
    `next_whole` cleared; next_frames None: none).  ptrs may pass prebuilt
    (frames, out_frames, next_frames) arrays from ptr_array, None for a part
    not requested."""
    def lut_ref(l):
        return ct.byref(rt_lut_buf(_p(l.lut8), _p(l.q16), _p(l.weights))) if l is not None else None

    def whole_ref(w):
        return ct.byref(rt_stats_buf(None, None, _p(w.whole_hist), _p(w.whole_sums))) if w is not None else None

    bb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), None, None)
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    if ptrs is not None:
        fa, oa, na = ptrs
    else:
        fa = _ptr_array(frames) if frames is not None else None
        oa = _ptr_array(out_frames) if frames is not None else None
        na = _ptr_array(next_frames) if next_frames is not None else None
    _check(load().rt_frameset_ahead(ctx, fa, oa, lut_ref(lut), whole_ref(whole), na, lut_ref(next_lut),
                                    whole_ref(next_whole), ct.byref(bb), ct.byref(pb), _stream_handle(stream)))


def rt_ctx_set_active(ctx, active: int) -> None:
    _check(load().rt_ctx_set_active(ctx, ct.c_uint64(active)))


def _removal(tau: int, min_kept: float) -> rt_removal_opts:
    return rt_removal_opts(int(tau), 0, float(min_kept))


def rt_seam_cost(ctx, frames, factor, seam, interior, rows=None, row_stride: int = 0, stream=None) -> None:
    """Seam gradient cost of every seam and interior reference (float64 [K]
    tensors seam, interior; rows float64 [K][2][row_stride] or None)."""
    _check(load().rt_seam_cost(ctx, _ptr_array(frames), factor, _p(seam), _p(interior), _p(rows), row_stride,
                               _stream_handle(stream)))


class CrossSet:
    """Device buffers of the cross-channel 3x3 maps of one context (shapes as
    the C-ABI documents); the state starts as the identity, not yet valid."""

    def __init__(self, sizes: "rt_sizes", device="cuda"):
        import torch
        K, NB = sizes.n_cams, sizes.n_blocks
        e = dict(device=device)
        self.cross = torch.zeros((K, 2, NB, 3), dtype=torch.int64, **e)
        self.params3 = torch.zeros((K, 2, NB, 12), dtype=torch.float64, **e)
        self.params3[..., 0] = 1.0
        self.params3[..., 4] = 1.0
        self.params3[..., 8] = 1.0
        self.valid3 = torch.zeros((K, 2, NB), dtype=torch.uint8, **e)
        self.q3 = torch.zeros((K, 2, NB, 12), dtype=torch.int64, **e)
        self.weights = torch.zeros((K, sizes.w_max), dtype=torch.int16, **e)

    def c(self) -> rt_cross_buf:
        return rt_cross_buf(_p(self.cross), _p(self.params3), _p(self.valid3), _p(self.q3), _p(self.weights))

    def host(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in ("cross", "params3", "valid3", "q3", "weights")}


def rt_cross_stats(ctx, frames, x: CrossSet, stream=None) -> None:
    xb = x.c()
    _check(load().rt_cross_stats(ctx, _ptr_array(frames), ct.byref(xb), _stream_handle(stream)))


def rt_estimate_cross(ctx, band_sums, x: CrossSet, stream=None) -> None:
    sb = rt_stats_buf(None, _p(band_sums), None, None)
    xb = x.c()
    _check(load().rt_estimate_cross(ctx, ct.byref(sb), ct.byref(xb), _stream_handle(stream)))


def rt_build_cross(ctx, x: CrossSet, stream=None) -> None:
    xb = x.c()
    _check(load().rt_build_cross(ctx, ct.byref(xb), _stream_handle(stream)))


def rt_apply_cross(ctx, frames, out_frames, x: CrossSet, whole_hist=None, whole_sums=None, stream=None) -> None:
    xb = x.c()
    wb = rt_stats_buf(None, None, _p(whole_hist), _p(whole_sums)) if whole_hist is not None else None
    _check(load().rt_apply_cross(ctx, _ptr_array(frames), _ptr_array(out_frames), ct.byref(xb),
                                 ct.byref(wb) if wb is not None else None, _stream_handle(stream)))


def rt_frameset_cross(ctx, frames, out_frames, bufs, x: CrossSet, stream=None) -> None:
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    xb = x.c()
    _check(load().rt_frameset_cross(ctx, _ptr_array(frames), _ptr_array(out_frames), ct.byref(sb), ct.byref(xb),
                                    _stream_handle(stream)))


def rt_attention(ctx, frames, prev_frames, tau, cell, m, theta, cells, windows=None, selected=None,
                 stream=None) -> None:
    """Difference approach of the attention mechanisms (cells u32 [K][hc][wc];
    windows u32 / selected u8 [K][hc-m+1][wc-m+1] or None)."""
    ao = rt_attention_opts(int(tau), int(cell), int(m), int(theta))
    _check(load().rt_attention(ctx, _ptr_array(frames), _ptr_array(prev_frames), ct.byref(ao), _p(cells),
                               _p(windows), _p(selected), _stream_handle(stream)))


def rt_motion_stats(ctx, frames, prev_frames, tau, min_kept, band_hist, band_sums, kept_sums, stream=None) -> None:
    ro = _removal(tau, min_kept)
    sb = rt_stats_buf(_p(band_hist), _p(band_sums), None, None)
    pf = None if prev_frames is None else _ptr_array(prev_frames)
    _check(load().rt_motion_stats(ctx, _ptr_array(frames), pf, ct.byref(ro), ct.byref(sb), _p(kept_sums),
                                  _stream_handle(stream)))


def rt_estimate_removal(ctx, band_hist, band_sums, kept_sums, tau, min_kept, params, valid, method=None,
                        stream=None) -> None:
    ro = _removal(tau, min_kept)
    sb = rt_stats_buf(_p(band_hist), _p(band_sums), None, None)
    pb = rt_params_buf(_p(params), _p(valid))
    _check(load().rt_estimate_removal(ctx, ct.byref(sb), _p(kept_sums), ct.byref(ro), ct.byref(pb), _p(method),
                                      _stream_handle(stream)))


def rt_frameset_removal(ctx, frames, prev_frames, out_frames, tau, min_kept, bufs: "Buffers", kept_sums,
                        method=None, stream=None) -> None:
    ro = _removal(tau, min_kept)
    sb = rt_stats_buf(_p(bufs.band_hist), _p(bufs.band_sums), _p(bufs.whole_hist), _p(bufs.whole_sums))
    pb = rt_params_buf(_p(bufs.params), _p(bufs.valid))
    lb = rt_lut_buf(_p(bufs.lut8), _p(bufs.q16), _p(bufs.weights))
    pf = None if prev_frames is None else _ptr_array(prev_frames)
    _check(load().rt_frameset_removal(ctx, _ptr_array(frames), pf, _ptr_array(out_frames), ct.byref(ro),
                                      ct.byref(sb), _p(kept_sums), ct.byref(pb), ct.byref(lb), _p(method),
                                      _stream_handle(stream)))


# ----------------------------------------------------------------------------- convenience

@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    channels: int = 3
    bit_depth: int = 8
    ring: int = 0
    pos: int = 0
    pitch_bytes: int = 0

    @property
    def bps(self) -> int:
        return 1 if self.bit_depth == 8 else 2

    @property
    def row_bytes(self) -> int:
        return self.width * self.channels * self.bps

    def with_pitch(self, pitch: int | None = None) -> "Camera":
        p = pitch if pitch is not None else (self.row_bytes + 15) // 16 * 16
        return Camera(self.width, self.height, self.channels, self.bit_depth, self.ring, self.pos, p)


@dataclass(frozen=True)
class Options:
    n_blocks: int = 16
    band_width: int = 32
    closed_ring: bool = True
    smoothing: bool = False
    ema_alpha: float = 0.05
    a_min: float = 0.125
    a_max: float = 8.0
    vblend: bool = False     # blend the maps of adjacent blocks row by row
    fit: str = "moments"     # "moments" or "quantile" (least squares on 64 quantiles)

    def to_c(self) -> rt_opts:
        fits = {"moments": RT_FIT_MOMENTS, "quantile": RT_FIT_QUANTILE}
        if self.fit not in fits:
            raise ValueError(f"unknown fit {self.fit!r}")
        return rt_opts(self.n_blocks, self.band_width, int(self.closed_ring),
                       RT_MODE_SMOOTHING if self.smoothing else RT_MODE_STANDARD,
                       self.ema_alpha, self.a_min, self.a_max, int(self.vblend), fits[self.fit])


class Buffers:
    """Caller-owned device buffers of one context, shaped as the C-ABI documents."""

    def __init__(self, sizes: rt_sizes, device="cuda"):
        import torch
        K, NB, WM = sizes.n_cams, sizes.n_blocks, sizes.w_max
        e = dict(device=device)
        self.band_hist = torch.zeros((K, 2, NB, CSLOTS, NBINS), dtype=torch.int32, **e)
        self.band_sums = torch.zeros((K, 2, NB, CSLOTS, 3), dtype=torch.int64, **e)
        self.whole_hist = torch.zeros((K, CSLOTS, NBINS), dtype=torch.int32, **e)
        self.whole_sums = torch.zeros((K, CSLOTS, 3), dtype=torch.int64, **e)
        self.params = torch.zeros((K, 2, NB, CSLOTS, 2), dtype=torch.float64, **e)
        self.params[..., 0] = 1.0
        self.valid = torch.zeros((K, 2, NB, CSLOTS), dtype=torch.uint8, **e)
        self.lut8 = torch.zeros((K, 2, NB, CSLOTS, NBINS), dtype=torch.uint8, **e)
        self.q16 = torch.zeros((K, 2, NB, CSLOTS, 2), dtype=torch.int64, **e)
        self.weights = torch.zeros((K, max(WM, 1)), dtype=torch.int16, **e)
        for name, t in self.__dict__.items():
            assert t.numel() == getattr(sizes, name), name

    def host(self) -> dict:
        """Copies of every buffer as numpy arrays (unsigned views where the ABI is unsigned)."""
        out = {}
        for name, t in self.__dict__.items():
            a = t.cpu().numpy()
            if name in ("band_hist", "whole_hist"):
                a = a.view(np.uint32)
            elif name in ("band_sums", "whole_sums"):
                a = a.view(np.uint64)
            elif name == "weights":
                a = a.view(np.uint16)
            out[name] = a
        return out


class Rig:
    """A context plus its buffers; frames are torch tensors laid out per camera."""

    def __init__(self, cams, opts: Options = Options(), device="cuda"):
        self.cams = [c if c.pitch_bytes else c.with_pitch() for c in cams]
        self.opts = opts
        self.ctx = rt_ctx_create(self.cams, opts)
        self.sizes = rt_ctx_sizes(self.ctx)
        self.bufs = Buffers(self.sizes, device)
        self.device = device

    def close(self) -> None:
        if self.ctx is not None:
            rt_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # frame helpers ----------------------------------------------------------
    def alloc_frames(self) -> list:
        """Zeroed device frames with each camera's pitch (tensors of shape (H, pitch) bytes)."""
        import torch
        return [torch.zeros((c.height, c.pitch_bytes), dtype=torch.uint8, device=self.device) for c in self.cams]

    def upload(self, frames_np) -> list:
        out = self.alloc_frames()
        self.upload_into(out, frames_np)
        return out

    def upload_into(self, dev, frames_np) -> None:
        import torch
        for d, c, f in zip(dev, self.cams, frames_np):
            raw = np.ascontiguousarray(f).view(np.uint8).reshape(c.height, c.row_bytes)
            d[:, :c.row_bytes].copy_(torch.from_numpy(raw))

    def download(self, frames_dev) -> list:
        out = []
        for d, c in zip(frames_dev, self.cams):
            raw = d[:, :c.row_bytes].cpu().numpy()
            dt = np.uint8 if c.bps == 1 else np.uint16
            out.append(np.ascontiguousarray(raw).view(dt).reshape(c.height, c.width, c.channels))
        return out

    # the C-ABI steps ----------------------------------------------------------
    def stats(self, frames, whole=True, stream=None) -> None:
        b = self.bufs
        rt_stats(self.ctx, frames, b.band_hist, b.band_sums,
                 b.whole_hist if whole else None, b.whole_sums if whole else None, stream)

    def estimate(self, stream=None) -> None:
        b = self.bufs
        rt_estimate(self.ctx, b.band_hist, b.band_sums, b.params, b.valid, stream)

    def build_lut(self, stream=None) -> None:
        b = self.bufs
        rt_build_lut(self.ctx, b.params, b.valid, b.lut8, b.q16, b.weights, stream)

    def apply(self, frames, out_frames, whole=False, stream=None) -> None:
        b = self.bufs
        rt_apply(self.ctx, frames, out_frames, b.lut8, b.q16, b.weights,
                 b.whole_hist if whole else None, b.whole_sums if whole else None, stream)

    def frameset(self, frames, out_frames, stream=None) -> None:
        rt_frameset(self.ctx, frames, out_frames, self.bufs, stream)

    def frameset_removal(self, frames, prev_frames, out_frames, kept_sums, method=None, tau: int = 20,
                         min_kept: float = 0.25, stream=None) -> None:
        """Frame-set with object removal against prev_frames (None: nothing moves)
        and the smoothing fallback; kept_sums int64 [K][2][NB][3][3], method
        uint8 [K][2][NB] (may be None)."""
        rt_frameset_removal(self.ctx, frames, prev_frames, out_frames, tau, min_kept, self.bufs, kept_sums, method,
                            stream)

    def seam_cost(self, frames, factor: int = 8, rows: bool = False, stream=None):
        """Seam gradient cost of every seam and the interior reference of every
        camera of `frames` (device tensors); returns (seam, interior[, rows])
        as float64 device tensors, [K] and [K][2][floor(max H / factor)]."""
        import torch
        K = self.sizes.n_cams
        dev = frames[0].device
        seam = torch.empty(K, dtype=torch.float64, device=dev)
        interior = torch.empty(K, dtype=torch.float64, device=dev)
        rbuf, stride = None, 0
        if rows:
            stride = max(1, max(c.height for c in self.cams) // factor)
            rbuf = torch.full((K, 2, stride), float("nan"), dtype=torch.float64, device=dev)
        rt_seam_cost(self.ctx, frames, factor, seam, interior, rbuf, stride, stream)
        return (seam, interior, rbuf) if rows else (seam, interior)

    def attention(self, frames, prev_frames, tau: int = 20, cell: int = 16, m: int = 8, theta: int = 256,
                  stream=None):
        """Attention map of the difference approach: (cells, windows, selected)
        device tensors laid out over the largest camera's cell grid."""
        import torch
        K = self.sizes.n_cams
        hc = -(-max(c.height for c in self.cams) // cell)
        wc = -(-max(c.width for c in self.cams) // cell)
        dev = frames[0].device
        cells = torch.empty((K, hc, wc), dtype=torch.int32, device=dev)
        shape = (K, max(hc - m + 1, 0), max(wc - m + 1, 0))
        win = torch.empty(shape, dtype=torch.int32, device=dev)
        sel = torch.empty(shape, dtype=torch.uint8, device=dev)
        rt_attention(self.ctx, frames, prev_frames, tau, cell, m, theta, cells, win, sel, stream)
        return cells, win, sel

    def frameset_batch(self, active: int, frames, out_frames, stream=None) -> None:
        """Frame-set of the cameras in bitmask `active` (whole rings); the
        entries of inactive cameras in frames / out_frames may be None."""
        rt_frameset_batch(self.ctx, active, frames, out_frames, self.bufs, stream)

    def set_active(self, active: int) -> None:
        """Restrict later calls to the cameras in bitmask `active` (whole rings)."""
        rt_ctx_set_active(self.ctx, active)

    def check(self) -> None:
        rt_ctx_check(self.ctx)

    def tune(self, tile_rows: int, grid: int = 0) -> None:
        rt_ctx_tune(self.ctx, tile_rows, grid)

    def tuning(self) -> tuple[int, int, int]:
        return rt_ctx_tuning(self.ctx)
