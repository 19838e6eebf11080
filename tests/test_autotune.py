"""Autotuner host logic (CPU): signatures, candidates, cache round trip; and
on the GPU that tuning picks a valid knob pair without changing results."""
import os

import numpy as np
import pytest

from paper_1910_03517_amd import autotune, rt


def test_signature_depends_on_geometry_and_options():
    cams = [rt.Camera(1920, 1080, 3, 8, 0, p).with_pitch() for p in range(3)]
    o = rt.Options()
    s0 = autotune.signature(cams, o, "gfx950")
    assert s0 == autotune.signature(list(cams), rt.Options(), "gfx950")
    assert s0 != autotune.signature(cams, rt.Options(n_blocks=64), "gfx950")
    assert s0 != autotune.signature(cams, o, "gfx942")
    assert s0 != autotune.signature(cams[:2], o, "gfx950")
    cams2 = cams[:2] + [rt.Camera(1920, 1080, 3, 8, 0, 2).with_pitch(5776)]
    assert s0 != autotune.signature(cams2, o, "gfx950")


def test_candidates_respect_block_height():
    cams = [rt.Camera(640, 40, 3, 8, 0, 0).with_pitch()]
    c = autotune.candidates(cams, 4)             # blocks of 10 rows
    assert all(r <= 10 for r, _ in c) and (10, 0) in c
    big = autotune.candidates([rt.Camera(1920, 1080, 3, 8, 0, 0).with_pitch()], 16)
    assert {r for r, _ in big} >= {16, 32, 64}
    assert all(g in autotune.GRIDS for _, g in big)


def test_cache_round_trip(tmp_path):
    p = os.path.join(tmp_path, "sub", "t.json")
    assert autotune.load_cache(p) == {}
    autotune.save_cache({"k": {"tile_rows": 32, "grid": 0, "us_per_frameset": 80.5}}, p)
    assert autotune.load_cache(p)["k"]["tile_rows"] == 32
    with open(p, "w") as f:
        f.write("not json")
    assert autotune.load_cache(p) == {}


@pytest.mark.gpu
def test_autotune_on_device_keeps_results(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_03517_amd import synth
    print("case: autotune 3x640x240 rgb8", flush=True)
    spec = synth.RigSpec("tune", 13, [synth.CamSpec(640, 240, 3, 8, 0, p) for p in range(3)])
    cams = [rt.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos).with_pitch() for c in spec.cams]
    frames = synth.rig_frames(spec, 0)
    ref = rt.Rig(cams, rt.Options())
    dev = ref.upload(frames)
    out_ref = ref.alloc_frames()
    ref.frameset(dev, out_ref)
    tuned = rt.Rig(cams, rt.Options())
    out = tuned.alloc_frames()
    path = os.path.join(tmp_path, "at.json")
    best = autotune.tune(tuned, [dev], [out], cache_path=path, iters=3,
                         cands=[(8, 0), (16, 1024), (32, 0)])
    assert (best.tile_rows, best.grid) in [(8, 0), (16, 1024), (32, 0)]
    assert tuned.tuning()[:2] == (best.tile_rows, best.grid)
    tuned.bufs.valid.zero_()
    tuned.frameset(dev, out)
    torch.cuda.synchronize()
    for a, b in zip(tuned.download(out), ref.download(out_ref)):
        assert np.array_equal(a, b)
    again = rt.Rig(cams, rt.Options())
    got = autotune.apply_cached(again, path)
    assert got is not None and again.tuning()[:2] == (best.tile_rows, best.grid)
    for r in (ref, tuned, again):
        r.close()


def test_pipe_candidates_and_mode_in_signature():
    cams = [rt.Camera(1920, 1080, 3, 8, 0, p).with_pitch() for p in range(14)]
    c = autotune.pipe_candidates(cams, 16)
    assert len(c) == len(autotune.PIPE_LANES) * len(autotune.PIPE_SPLITS)
    assert all(group <= lanes for lanes, group, _, _, fuse in c if not fuse)
    assert all(group <= 4 for _, group, _, _, fuse in c if fuse)
    small = autotune.pipe_candidates([rt.Camera(320, 120, 3, 8, 0, 0).with_pitch()], 16)   # blocks of 8 rows
    assert {r for _, _, r, _, _ in small} == {32}              # taller splits dropped, the smallest kept
    many = autotune.pipe_candidates([rt.Camera(320, 120, 3, 8, 0, p).with_pitch() for p in range(17)], 16)
    assert many and not any(fuse for *_, fuse in many)         # fused launches take at most 16 cameras
    o = rt.Options()
    assert autotune.signature(cams, o, "gfx950") != autotune.signature(cams, o, "gfx950", "pipe")
    assert autotune.signature(cams, o, "gfx950") == autotune.signature(cams, o, "gfx950", "eager")
