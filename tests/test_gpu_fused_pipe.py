"""GPU parity of the fused pipeline applies (rt_pipe_set_fuse): the applies
of a group issued as launches of up to four frame-sets on one lane, groups
taking the lanes in turn.  Every output, the whole-frame statistics and tables
of the slots still intact, and the final estimator state equal consecutive
rt_frameset (or rt_frameset_batch) calls bit for bit; launches split at four
frame-sets and at a change of the active cameras."""
import ctypes as ct

import numpy as np
import pytest

from tests.gpu_helpers import rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def mixed_rings():
    """A closed RGB8 ring, an open gray16 chain and a one-camera RGB8 ring."""
    spec = ([synth.CamSpec(200, 90, 3, 8, 0, p) for p in (1, 0, 2)]
            + [synth.CamSpec(120, 64, 1, 16, 4, p) for p in (1, 0)]
            + [synth.CamSpec(160, 48, 3, 8, 9, 0)])
    return spec, rt_cams(spec, 1)


def sequential(cams, opts, dev, masks=None):
    """Consecutive rt_frameset (or rt_frameset_batch) calls: per step the
    outputs, whole-frame statistics and tables, and the final state."""
    rig = rt.Rig(cams, opts)
    out = rig.alloc_frames()
    steps = []
    for t, d in enumerate(dev):
        if masks is None:
            rig.frameset(d, out)
        else:
            rig.frameset_batch(masks[t], d, out)
        torch.cuda.synchronize()
        steps.append(dict(out=rig.download(out), wh=rig.bufs.whole_hist.cpu().numpy().copy(),
                          ws=rig.bufs.whole_sums.cpu().numpy().copy(), q16=rig.bufs.q16.cpu().numpy().copy(),
                          lut8=rig.bufs.lut8.cpu().numpy().copy()))
    h = rig.bufs.host()
    rig.close()
    return steps, h


def check_against(par, pipe, outs, slots, steps, href, depth, masks=None):
    T = len(outs)
    for t in range(T):
        active = masks[t] if masks is not None else (1 << len(outs[t])) - 1
        for k, (a, b) in enumerate(zip(par.download(outs[t]), steps[t]["out"])):
            if (active >> k) & 1:
                assert np.array_equal(a, b), f"frame-set {t} camera {k}"
        if t >= T - depth and masks is None:
            w, L = pipe.whole[slots[t]], pipe.luts[slots[t]]
            assert np.array_equal(w.whole_hist.cpu().numpy(), steps[t]["wh"]), f"t {t}"
            assert np.array_equal(w.whole_sums.cpu().numpy(), steps[t]["ws"]), f"t {t}"
            assert np.array_equal(L.q16.cpu().numpy(), steps[t]["q16"]), f"t {t}"
            assert np.array_equal(L.lut8.cpu().numpy(), steps[t]["lut8"]), f"t {t}"
    hp = par.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), href["params"].view(np.uint64))
    assert np.array_equal(hp["valid"], href["valid"])


@pytest.mark.parametrize("depth,lanes,group", [(1, 1, 1), (2, 2, 2), (4, 2, 2), (3, 1, 3), (5, 3, 3), (8, 2, 4),
                                               (8, 3, 8), (8, 1, 6), (6, 2, 5)])
def test_fused_pipeline_matches_sequential(depth, lanes, group):
    """Mixed rings, 11 frame-sets with smoothing and drifting gains: groups
    of one frame-set up to groups that split into two launches (more than
    four frame-sets), the last group partial, slots reused."""
    say(f"case: fused pipeline depth {depth} lanes {lanes} group {group}, mixed rings, 11 frame-sets")
    spec, cams = mixed_rings()
    opts = rt.Options(n_blocks=5, band_width=12, smoothing=True, closed_ring=False)
    rng = np.random.default_rng(40 + depth * 10 + group)
    T = 11
    frames = [[synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec] for _ in range(T)]
    par = rt.Rig(cams, opts)
    dev = [par.upload(f) for f in frames]
    outs = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    steps, href = sequential(cams, opts, dev)
    pipe = rt.Pipe.for_rig(par, depth=depth, lanes=lanes, group=group, fuse=True)
    slots = [pipe.submit(dev[t], outs[t]) for t in range(T)]
    pipe.join()
    torch.cuda.synchronize()
    par.check()
    check_against(par, pipe, outs, slots, steps, href, depth)
    pipe.close()
    par.close()


def test_fused_pipeline_blended_maps_and_quantile_fit():
    """The fused launch with the maps blended between blocks (its own kernel
    form) and the quantile fit, through submit_n in groups of 4."""
    say("case: fused pipeline, vblend + quantile fit, 5x256x120 rgb8, 9 frame-sets")
    spec = synth.RigSpec("fused combo 5x256x120", 35, [synth.CamSpec(256, 120, 3, 8, 0, p) for p in range(5)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, fit="quantile", vblend=True, smoothing=True)
    T = 9
    par = rt.Rig(cams, opts)
    dev = [par.upload(synth.rig_frames(spec, t, drift=True)) for t in range(T)]
    outs = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    steps, href = sequential(cams, opts, dev)
    pipe = rt.Pipe.for_rig(par, depth=8, lanes=2, group=4, fuse=True)
    slots = pipe.submit_n(dev, outs)
    pipe.join()
    torch.cuda.synchronize()
    par.check()
    check_against(par, pipe, outs, slots, steps, href, 8)
    pipe.close()
    par.close()


def test_fused_pipeline_active_masks_and_timing():
    """submit_batch with the active rings changing inside groups of 4: a
    launch holds only frame-sets of one mask, and the results equal
    consecutive rt_frameset_batch calls.  The context's timing of the same
    run reports one entry per launch, with the frame-sets it covered."""
    say("case: fused pipeline, masks changing inside groups, 3 rings, 10 frame-sets, timed")
    cams_spec = (synth.ring_of(3, 320, 96, ring=0) + synth.ring_of(2, 256, 64, ring=1)
                 + synth.ring_of(4, 200, 50, ring=2))
    spec = synth.RigSpec("fused masks", 36, cams_spec)
    cams = rt_cams(spec.cams)
    rings = [sum(1 << i for i, c in enumerate(spec.cams) if c.ring == r) for r in range(3)]
    every = rings[0] | rings[1] | rings[2]
    masks = [rings[0], rings[0], rings[1], every, every, every, every, every, rings[2], rings[0] | rings[2]]
    T = len(masks)
    opts = rt.Options(n_blocks=4, band_width=16, smoothing=True)
    par = rt.Rig(cams, opts)
    dev = [par.upload(synth.rig_frames(spec, t, drift=True)) for t in range(T)]
    outs = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    steps, href = sequential(cams, opts, dev, masks)
    rt.rt_ctx_timing(par.ctx, 64, 1)
    pipe = rt.Pipe.for_rig(par, depth=8, lanes=2, group=4, fuse=True)
    slots = []
    for t in range(T):
        m = masks[t]
        slots.append(pipe.submit_batch(m, [d if (m >> i) & 1 else None for i, d in enumerate(dev[t])],
                                       [o if (m >> i) & 1 else None for i, o in enumerate(outs[t])]))
    pipe.join()
    torch.cuda.synchronize()
    par.check()
    check_against(par, pipe, outs, slots, steps, href, 8, masks)
    sets = rt.rt_ctx_apply_sets(par.ctx, 64)
    times = rt.rt_ctx_apply_times(par.ctx, 64)
    # Two single launches while the pipeline fills, then groups of 4 cut at
    # mask changes: [m0] [m0] | [m1] [every x3] | [every x2] [m2] [m0|m2].
    assert sets == [1, 1, 1, 3, 2, 1, 1], sets
    assert len(times) == len(sets) and all(x > 0 for x in times)
    rt.rt_ctx_timing(par.ctx, 0)
    pipe.close()
    par.close()


def test_set_fuse_validation():
    """fuse outside {0, 1} is refused, a rig of more than 16 cameras cannot
    fuse, and switching back and forth between submits keeps the results."""
    say("case: set_fuse validation")
    lib = rt.load()
    spec = synth.RigSpec("fuse 17", 37, [synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(17)])
    big = rt.Rig(rt_cams(spec.cams), rt.Options(n_blocks=2, band_width=8))
    pipe = rt.Pipe.for_rig(big, depth=2, lanes=1, group=1)
    assert lib.rt_pipe_set_fuse(pipe.handle, 2) == rt.RT_EINVAL
    assert lib.rt_pipe_set_fuse(pipe.handle, -1) == rt.RT_EINVAL
    assert lib.rt_pipe_set_fuse(pipe.handle, 1) == rt.RT_EUNSUPPORTED
    assert lib.rt_pipe_set_fuse(pipe.handle, 0) == rt.RT_OK
    pipe.close()
    big.close()
    spec = synth.RigSpec("fuse toggle 4x160x64", 38, [synth.CamSpec(160, 64, 3, 8, 0, p) for p in range(4)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=4, band_width=12, smoothing=True)
    T = 9
    par = rt.Rig(cams, opts)
    dev = [par.upload(synth.rig_frames(spec, t, drift=True)) for t in range(T)]
    outs = [par.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    steps, href = sequential(cams, opts, dev)
    pipe = rt.Pipe.for_rig(par, depth=6, lanes=3, group=3)
    slots = []
    for t in range(T):
        if t in (2, 4, 7):
            pipe.set_fuse(not pipe.fuse)   # issues the pending applies first
        slots.append(pipe.submit(dev[t], outs[t]))
    pipe.join()
    torch.cuda.synchronize()
    check_against(par, pipe, outs, slots, steps, href, 6)
    st = ct.c_int32(0)
    assert lib.rt_ctx_apply_sets(None, ct.byref(st), 1, ct.byref(st)) == rt.RT_EINVAL
    pipe.close()
    par.close()


@pytest.mark.parametrize("vblend", [False, True])
def test_apply_sets_equals_single_applies(vblend):
    """rt_apply_sets over 1..4 frame-sets (each with its own tables, built
    from a different frame-set) equals rt_apply with whole-frame statistics
    per frame-set, outputs and statistics bit for bit; refusals for n outside
    1..4 and for more than 16 cameras."""
    say(f"case: rt_apply_sets vblend={vblend}, 3 rgb8 + 2 gray16 cameras")
    spec = ([synth.CamSpec(200, 90, 3, 8, 0, p) for p in (1, 0, 2)]
            + [synth.CamSpec(120, 64, 1, 16, 4, p) for p in (1, 0)])
    cams = rt_cams(spec, 1)
    opts = rt.Options(n_blocks=5, band_width=12, closed_ring=False, vblend=vblend)
    rig = rt.Rig(cams, opts)
    rng = np.random.default_rng(51)
    frames = [[synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec] for _ in range(4)]
    dev = [rig.upload(f) for f in frames]
    luts = [rt.LutSet(rig.sizes) for _ in range(4)]
    b = rig.bufs
    for t in range(4):
        rt.rt_stats(rig.ctx, dev[t], b.band_hist, b.band_sums)
        rt.rt_estimate(rig.ctx, b.band_hist, b.band_sums, b.params, b.valid)
        rt.rt_build_lut(rig.ctx, b.params, b.valid, luts[t].lut8, luts[t].q16, luts[t].weights)
    torch.cuda.synchronize()
    ref_out, ref_w = [], []
    for t in range(4):
        out = rig.alloc_frames()
        w = rt.WholeSet(rig.sizes)
        rt.rt_apply(rig.ctx, dev[t], out, luts[t].lut8, luts[t].q16, luts[t].weights, w.whole_hist, w.whole_sums)
        torch.cuda.synchronize()
        ref_out.append(rig.download(out))
        ref_w.append((w.whole_hist.cpu().numpy(), w.whole_sums.cpu().numpy()))
    for n in (1, 3, 4):
        outs = [rig.alloc_frames() for _ in range(n)]
        wholes = [rt.WholeSet(rig.sizes) for _ in range(n)]
        for w in wholes:                      # stale values: the call clears them
            w.whole_hist.fill_(7)
            w.whole_sums.fill_(9)
        rt.rt_apply_sets(rig.ctx, dev[:n], outs, luts[:n], wholes)
        torch.cuda.synchronize()
        for t in range(n):
            for k, (a, e) in enumerate(zip(rig.download(outs[t]), ref_out[t])):
                assert np.array_equal(a, e), f"n {n} frame-set {t} camera {k}"
            assert np.array_equal(wholes[t].whole_hist.cpu().numpy(), ref_w[t][0]), f"n {n} t {t} whole_hist"
            assert np.array_equal(wholes[t].whole_sums.cpu().numpy(), ref_w[t][1]), f"n {n} t {t} whole_sums"
    rig.check()
    lib = rt.load()
    fa, oa = rt.ptr_array_n(dev[:1]), rt.ptr_array_n([rig.alloc_frames()])
    la = (rt.rt_lut_buf * 1)(rt.rt_lut_buf(rt._p(luts[0].lut8), rt._p(luts[0].q16), rt._p(luts[0].weights)))
    w0 = rt.WholeSet(rig.sizes)
    wa = (rt.rt_stats_buf * 1)(rt.rt_stats_buf(None, None, rt._p(w0.whole_hist), rt._p(w0.whole_sums)))
    for n in (0, 5, -1):
        assert lib.rt_apply_sets(rig.ctx, n, fa, oa, la, wa, None) == rt.RT_EINVAL, n
    rig.close()
    big = rt.Rig(rt_cams([synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(17)]),
                 rt.Options(n_blocks=2, band_width=8))
    assert lib.rt_apply_sets(big.ctx, 1, None, None, None, None, None) == rt.RT_EUNSUPPORTED
    big.close()
