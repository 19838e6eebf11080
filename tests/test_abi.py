"""C-ABI library: it loads, exports every symbol the header declares, and its
host-side validation rejects bad rigs and options before touching the device.
No compute calls: these run without a GPU."""
import ctypes as ct
import os
import re

import pytest

from paper_1910_03517_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ringcorr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*]+\s+\**(rt_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rt_stats", "rt_estimate", "rt_build_lut", "rt_apply", "rt_frameset", "rt_ctx_create"):
        assert n in names
    assert sorted(rt.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    lib = rt.load()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_status_strings():
    lib = rt.load()
    assert lib.rt_status_str(rt.RT_OK) == b"ok"
    assert lib.rt_status_str(rt.RT_EINVAL) == b"invalid argument"
    assert lib.rt_status_str(12345) == b"unknown status"


def _create(cams, opts):
    lib = rt.load()
    arr = (rt.rt_camera_desc * max(len(cams), 1))()
    for i, c in enumerate(cams):
        arr[i] = rt.rt_camera_desc(*c)
    o = opts.to_c() if isinstance(opts, rt.Options) else opts
    ctx = ct.c_void_p(1234)
    st = lib.rt_ctx_create(arr, len(cams), ct.byref(o), ct.byref(ctx))
    return st, ctx, lib.rt_last_error().decode()


GOOD = (64, 32, 3, 8, 0, 0, 192)


@pytest.mark.parametrize("cams,opts,needle", [
    ([], rt.Options(), "n_cams"),
    ([GOOD] * 65, rt.Options(), "n_cams"),
    ([GOOD], rt.Options(n_blocks=0), "n_blocks"),
    ([GOOD], rt.Options(band_width=0), "band_width"),
    ([GOOD], rt.Options(ema_alpha=0.0), "ema_alpha"),
    ([GOOD], rt.Options(ema_alpha=1.5), "ema_alpha"),
    ([GOOD], rt.Options(a_min=2.0, a_max=1.0), "a_min"),
    ([(0, 32, 3, 8, 0, 0, 192)], rt.Options(), "size"),
    ([(64, 32, 2, 8, 0, 0, 192)], rt.Options(), "channels"),
    ([(64, 32, 3, 7, 0, 0, 192)], rt.Options(), "bit_depth"),
    ([(64, 32, 3, 12, 0, 0, 400)], rt.Options(), "16-bit"),
    ([(64, 32, 3, 8, 0, 0, 100)], rt.Options(), "pitch"),
    ([(64, 32, 3, 8, 0, 0, 200)], rt.Options(), "pitch"),
    ([GOOD, (64, 32, 3, 8, 0, 0, 192)], rt.Options(), "positions"),
    ([GOOD, (64, 32, 3, 8, 0, 2, 192)], rt.Options(), "positions"),
    ([GOOD, (64, 32, 1, 8, 0, 1, 64)], rt.Options(), "mixes"),
])
def test_create_rejects_invalid(cams, opts, needle):
    st, ctx, msg = _create(cams, opts)
    assert st == rt.RT_EINVAL
    assert ctx.value is None
    assert needle in msg


def test_null_arguments_are_rejected():
    lib = rt.load()
    assert lib.rt_ctx_create(None, 1, None, None) == rt.RT_EINVAL
    assert lib.rt_stats(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_estimate(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_build_lut(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_apply(None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_frameset(None, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_frameset_batch(None, 1, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_frameset_ahead(None, None, None, None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_ctx_set_active(None, 1) == rt.RT_EINVAL
    assert lib.rt_ctx_sizes(None, None) == rt.RT_EINVAL
    assert lib.rt_ctx_destroy(None) == rt.RT_OK
    assert lib.rt_ctx_check(None) == rt.RT_EINVAL
    assert lib.rt_ctx_tune(None, 8, 0) == rt.RT_EINVAL
    assert lib.rt_ctx_tuning(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_stream_copy(None, None, 16, 16, None) == rt.RT_EINVAL
    assert lib.rt_ctx_timing(None, 4, 1) == rt.RT_EINVAL
    assert lib.rt_graph_create(None, None, None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_graph_launch(None, None) == rt.RT_EINVAL
    assert lib.rt_graph_destroy(None) == rt.RT_OK
    assert lib.rt_graph_set_frames(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_pipe_create(None, 2, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_pipe_submit(None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_pipe_destroy(None) == rt.RT_OK
    assert lib.rt_pipe_create_lanes(None, 2, 2, 1, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_pipe_join(None, None) == rt.RT_EINVAL
    assert lib.rt_pipe_submit_batch(None, 1, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_surrogate_features(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_estimate_new(None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_surrogate_targets(None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_surrogate_select(None, None, None, None, 1e-3, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_surrogate_frameset(None, None, 1e-3, None, None, None, None, None, None, None,
                                     None) == rt.RT_EINVAL
    assert lib.rt_mlp_forward(None, None, 1, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_mlp_backward(None, None, None, None, None, None, 1, None, None, None, None,
                               None) == rt.RT_EINVAL
    assert lib.rt_mlp_adam(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == rt.RT_EINVAL
    assert lib.rt_mlp_mse(None, None, 1, None, None) == rt.RT_EINVAL
    assert lib.rt_gather_rows(None, 1, None, 1, None, None) == rt.RT_EINVAL
    assert lib.rt_ctx_apply_times(None, None, 0, None) == rt.RT_EINVAL
    assert lib.rt_ctx_apply_sets(None, None, 0, None) == rt.RT_EINVAL
    assert lib.rt_pipe_set_fuse(None, 1) == rt.RT_EINVAL
    assert lib.rt_pipe_set_removal(None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_apply_sets(None, 1, None, None, None, None, None) == rt.RT_EINVAL
