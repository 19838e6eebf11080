"""GPU parity of rt_frameset_ahead, the frame-set loop with one launch per
frame-set (the apply of frame-set t beside the seam statistics, estimate and
tables of frame-set t + 1): over a sequence, every output, the whole-frame
statistics and tables of each frame-set, and the final estimator state equal
consecutive rt_frameset calls bit for bit; argument refusals."""
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


def eager(cams, opts, dev, active=None):
    """Consecutive rt_frameset calls: per frame-set the outputs, whole-frame
    statistics and tables; the final state."""
    rig = rt.Rig(cams, opts)
    if active is not None:
        rig.set_active(active)
    out = rig.alloc_frames()
    steps = []
    for d in dev:
        rig.frameset(d, out)
        torch.cuda.synchronize()
        b = rig.bufs
        steps.append(dict(out=rig.download(out), wh=b.whole_hist.cpu().numpy().copy(),
                          ws=b.whole_sums.cpu().numpy().copy(), q16=b.q16.cpu().numpy().copy(),
                          lut8=b.lut8.cpu().numpy().copy()))
    h = rig.bufs.host()
    rig.close()
    return steps, h


def ahead_loop(rig, dev, outs, stale=True):
    """rt_frameset_ahead for t = 0..T with two table and two whole-statistics
    buffers taken in turn; per frame-set the whole statistics and tables as
    they stand after its apply."""
    luts = [rt.LutSet(rig.sizes) for _ in range(2)]
    wholes = [rt.WholeSet(rig.sizes) for _ in range(2)]
    if stale:                                  # the estimate part clears them
        for w in wholes:
            w.whole_hist.fill_(7)
            w.whole_sums.fill_(9)
    got = []
    T = len(dev)
    for t in range(T + 1):
        a, e = (t - 1) % 2, t % 2
        rt.rt_frameset_ahead(rig.ctx, dev[t - 1] if t else None, outs[t - 1] if t else None,
                             luts[a] if t else None, wholes[a] if t else None,
                             dev[t] if t < T else None, luts[e] if t < T else None, wholes[e] if t < T else None,
                             rig.bufs)
        if t:
            torch.cuda.synchronize()
            got.append(dict(wh=wholes[a].whole_hist.cpu().numpy().copy(), ws=wholes[a].whole_sums.cpu().numpy().copy(),
                            q16=luts[a].q16.cpu().numpy().copy(), lut8=luts[a].lut8.cpu().numpy().copy()))
    torch.cuda.synchronize()
    return got


def compare(rig, outs, got, steps, href, active):
    for t, (g, s) in enumerate(zip(got, steps)):
        for k, (a, b) in enumerate(zip(rig.download(outs[t]), s["out"])):
            if (active >> k) & 1:
                assert np.array_equal(a, b), f"frame-set {t} camera {k}"
        for key in ("wh", "ws", "q16", "lut8"):
            assert np.array_equal(g[key], s[key]), f"frame-set {t} {key}"
    hp = rig.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), href["params"].view(np.uint64))
    assert np.array_equal(hp["valid"], href["valid"])


@pytest.mark.parametrize("vblend,fit", [(False, "moments"), (True, "moments"), (False, "quantile"), (True, "quantile")])
def test_ahead_loop_matches_frameset(vblend, fit):
    """Mixed rings, 7 frame-sets with smoothing: the look-ahead loop equals
    consecutive rt_frameset calls, with blended maps and the quantile fit."""
    say(f"case: rt_frameset_ahead vblend={vblend} fit={fit}, mixed rings, 7 frame-sets")
    spec, cams = mixed_rings()
    opts = rt.Options(n_blocks=5, band_width=12, smoothing=True, closed_ring=False, vblend=vblend, fit=fit)
    rng = np.random.default_rng(71 + vblend + 2 * (fit == "quantile"))
    T = 7
    frames = [[synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec] for _ in range(T)]
    rig = rt.Rig(cams, opts)
    dev = [rig.upload(f) for f in frames]
    outs = [rig.alloc_frames() for _ in range(T)]
    torch.cuda.synchronize()
    steps, href = eager(cams, opts, dev)
    got = ahead_loop(rig, dev, outs)
    rig.check()
    compare(rig, outs, got, steps, href, (1 << len(cams)) - 1)
    rig.close()


def test_ahead_loop_many_seam_blocks_and_active_set():
    """Twelve cameras in two rings with 8 blocks (more seam blocks than the
    two-unit estimate launch takes, so rt_frameset uses its other form),
    with only the second ring active."""
    say("case: rt_frameset_ahead 12 cameras, 8 blocks, second ring active")
    spec = ([synth.CamSpec(176, 72, 3, 8, 0, p) for p in (1, 0, 2, 3, 4, 5)]
            + [synth.CamSpec(144, 80, 3, 8, 6, p) for p in (2, 0, 1, 3, 5, 4)])
    cams = rt_cams(spec, 1)
    opts = rt.Options(n_blocks=8, band_width=10, smoothing=True)
    rng = np.random.default_rng(77)
    T = 5
    frames = [[synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in spec] for _ in range(T)]
    for active in ((1 << 12) - 1, ((1 << 6) - 1) << 6):
        rig = rt.Rig(cams, opts)
        rig.set_active(active)
        dev = [rig.upload(f) for f in frames]
        outs = [rig.alloc_frames() for _ in range(T)]
        torch.cuda.synchronize()
        steps, href = eager(cams, opts, dev, active)
        got = ahead_loop(rig, dev, outs, stale=False)
        compare(rig, outs, got, steps, href, active)
        rig.close()


def test_ahead_refusals():
    """Neither part requested, shared tables or whole statistics between the
    two parts, NULL buffers: RT_EINVAL before anything is enqueued."""
    say("case: rt_frameset_ahead refusals")
    spec, cams = mixed_rings()
    rig = rt.Rig(cams, rt.Options(n_blocks=5, band_width=12, closed_ring=False))
    dev = rig.upload([synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, np.random.default_rng(3))
                      for c in spec])
    out = rig.alloc_frames()
    L, W = rt.LutSet(rig.sizes), rt.WholeSet(rig.sizes)
    L2, W2 = rt.LutSet(rig.sizes), rt.WholeSet(rig.sizes)
    lib = rt.load()
    P = ct.c_void_p
    K = len(cams)
    assert lib.rt_frameset_ahead(rig.ctx, None, None, None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    with pytest.raises(rt.RtError):
        rt.rt_frameset_ahead(rig.ctx, dev, out, L, W, dev, L, W2, rig.bufs)
    with pytest.raises(rt.RtError):
        rt.rt_frameset_ahead(rig.ctx, dev, out, L, W, dev, L2, W, rig.bufs)
    L3 = rt.LutSet(rig.sizes)
    L3.weights = L.weights                       # tables distinct, weights shared
    with pytest.raises(rt.RtError):
        rt.rt_frameset_ahead(rig.ctx, dev, out, L, W, dev, L3, W2, rig.bufs)
    with pytest.raises(rt.RtError):
        rt.rt_frameset_ahead(rig.ctx, dev, out, None, W, None, None, None, rig.bufs)
    with pytest.raises(rt.RtError):
        rt.rt_frameset_ahead(rig.ctx, None, None, None, None, dev, L2, None, rig.bufs)
    nulls = (P * K)()
    assert lib.rt_frameset_ahead(rig.ctx, None, None, None, None, nulls, None, None, None, None, None) == rt.RT_EINVAL
    torch.cuda.synchronize()
    rig.check()
    rig.close()
