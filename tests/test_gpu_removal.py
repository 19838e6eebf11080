"""GPU parity of object removal with the smoothing fallback (section 3.1's
supplemental methods for moving objects, chosen per seam unit) against the
oracle: band and kept sums bit for bit, the method of every unit exactly,
parameters bitwise equal (within 1e-4 at worst), tables and pixels bit for
bit - from tiny ragged geometries to the full 14x1920x1080 rig with an object
crossing a seam - and the same method through the frame-set pipeline."""
import ctypes as ct

import numpy as np
import pytest

from tests.gpu_helpers import assert_ints_equal, assert_params_close, oracle_cams, oracle_opts, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def kept_buf(rig):
    K, NB = rig.sizes.n_cams, rig.sizes.n_blocks
    return (torch.zeros((K, 2, NB, 3, 3), dtype=torch.int64, device="cuda"),
            torch.full((K, 2, NB), 255, dtype=torch.uint8, device="cuda"))


def perturbed(frames, rng, bd, frac):
    """Previous frames: each pixel moved by up to +-3 tau on a random fraction of pixels."""
    out = []
    for f in frames:
        maxv = (1 << bd) - 1
        step = 20 << (bd - 8)
        d = rng.integers(-3 * step, 3 * step + 1, f.shape)
        m = rng.random(f.shape[:2]) < frac
        out.append(np.clip(f.astype(np.int64) + d * m[:, :, None], 0, maxv).astype(f.dtype))
    return out


CASES = [
    # (W, H, C, bit_depth, K, closed, NB, B, pad, moving fraction)
    (1, 1, 3, 8, 1, True, 1, 32, 0, 0.5),
    (2, 3, 1, 8, 3, True, 2, 1, 0, 0.5),
    (3, 7, 3, 8, 2, True, 16, 32, 0, 0.3),      # H < NB: empty blocks
    (5, 9, 3, 8, 3, False, 4, 2, 2, 0.9),       # open chain, mostly moving
    (17, 13, 3, 8, 2, True, 3, 32, 1, 0.2),     # W < 2B, right band not 4-pixel aligned
    (33, 31, 3, 8, 4, True, 7, 5, 0, 0.5),      # band of 5: a ragged group
    (64, 48, 1, 8, 2, True, 4, 8, 1, 0.6),      # gray8
    (61, 40, 1, 10, 2, True, 5, 6, 0, 0.5),     # 10-bit, odd band start
    (77, 66, 1, 16, 2, True, 16, 32, 1, 0.4),   # 16-bit
    (130, 70, 3, 8, 3, True, 16, 32, 0, 0.85),  # around the kept-fraction limit
    (1031, 67, 3, 8, 2, True, 64, 30, 3, 0.5),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}b{c[3]}k{c[4]}" for c in CASES])
def test_motion_stats_and_removal_estimate(case):
    W, H, C, bd, K, closed, NB, B, pad, frac = case
    say("case: removal steps", case)
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    spec = [synth.CamSpec(W, H, C, bd, 0, p) for p in range(K)]
    cams = rt_cams(spec, pad)
    for smoothing in (False, True):
        opts = rt.Options(n_blocks=NB, band_width=B, closed_ring=closed, smoothing=smoothing)
        co, oo = oracle_cams(cams), oracle_opts(opts)
        rig = rt.Rig(cams, opts)
        frames = [synth.tiny_frame(H, W, C, bd, rng) for _ in range(K)]
        prev = perturbed(frames, rng, bd, frac)
        dev, pdev = rig.upload(frames), rig.upload(prev)
        kept, method = kept_buf(rig)
        b = rig.bufs
        prev_p = rng.uniform(0.7, 1.4, tuple(b.params.shape))
        prev_v = rng.integers(0, 2, tuple(b.valid.shape)).astype(np.uint8)
        b.params.copy_(torch.as_tensor(prev_p, device="cuda"))
        b.valid.copy_(torch.as_tensor(prev_v, device="cuda"))
        rt.rt_motion_stats(rig.ctx, dev, pdev, 20, 0.25, b.band_hist, b.band_sums, kept)
        rt.rt_estimate_removal(rig.ctx, b.band_hist, b.band_sums, kept, 20, 0.25, b.params, b.valid, method)
        torch.cuda.synchronize()
        h = b.host()
        bh_o = np.stack([rc.band_stats(f, c, oo)[0] for f, c in zip(frames, co)])
        bs_o = np.stack([rc.band_stats(f, c, oo)[1] for f, c in zip(frames, co)])
        kept_o = np.stack([rc.kept_band_sums(f, p, c, oo, 20) for f, p, c in zip(frames, prev, co)])
        assert_ints_equal(h["band_hist"], bh_o, "band_hist")
        assert_ints_equal(h["band_sums"], bs_o, "band_sums")
        assert_ints_equal(kept.cpu().numpy(), kept_o, "kept_sums")
        p_o, v_o, m_o = rc.estimate_removal(co, oo, bs_o, kept_o, prev_p, prev_v, 0.25)
        assert_ints_equal(method.cpu().numpy(), m_o, "method")
        assert_ints_equal(h["valid"], v_o, "valid")
        assert_params_close(h["params"], p_o)
        assert np.array_equal(h["params"].view(np.uint64), p_o.view(np.uint64)), "params not bitwise equal"
        # Without previous frames nothing moves: kept sums are the band sums.
        rt.rt_motion_stats(rig.ctx, dev, None, 20, 0.25, b.band_hist, b.band_sums, kept)
        torch.cuda.synchronize()
        assert_ints_equal(kept.cpu().numpy(), bs_o, "kept_sums without previous frames")
        rig.close()


def removal_sequence(rig_spec, opts, n_frames, objects, check_every=1, drift=True):
    """Frame-sets t = 0 .. n_frames - 1 through rt_frameset_removal (the
    previous frame-set as prev_frames from t = 1) against the oracle's
    frameset_removal sequence."""
    cams = rt_cams(rig_spec.cams)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    kept, method = kept_buf(rig)
    outs = rig.alloc_frames()
    prev_np, prev_dev = None, None
    prev_p = prev_v = None
    seen = set()
    for t in range(n_frames):
        frames = synth.rig_frames(rig_spec, t, drift=drift, objects=objects)
        dev = rig.upload(frames)
        rig.frameset_removal(dev, prev_dev, outs, kept, method)
        torch.cuda.synchronize()
        ref = rc.frameset_removal(co, oo, frames, prev_np, prev_p, prev_v)
        if t % check_every == 0 or t == n_frames - 1:
            g = rig.bufs.host()
            assert_ints_equal(kept.cpu().numpy(), ref["kept_sums"], f"t {t}: kept_sums")
            assert_ints_equal(method.cpu().numpy(), ref["method"], f"t {t}: method")
            assert_ints_equal(g["band_sums"], ref["band_sums"], f"t {t}: band_sums")
            assert_ints_equal(g["whole_hist"], ref["whole_hist"], f"t {t}: whole_hist")
            assert_ints_equal(g["valid"], ref["valid"], f"t {t}: valid")
            assert np.array_equal(g["params"].view(np.uint64), ref["params"].view(np.uint64)), f"t {t}: params"
            lut8_o, q16_o = rc.build_luts(co, oo, g["params"])
            assert_ints_equal(g["q16"], q16_o, f"t {t}: q16")
            got = rig.download(outs)
            for k in range(len(cams)):
                assert_ints_equal(got[k], ref["out"][k], f"t {t}: out[{k}]")
        seen |= set(np.unique(ref["method"]).tolist())
        prev_np, prev_dev = frames, dev
        prev_p, prev_v = ref["params"], ref["valid"]
    rig.close()
    return seen


def test_small_rig_object_crossing_sequence():
    say("case: removal sequence, 4x320x180 rgb8 with an object crossing a seam")
    spec = synth.RigSpec("removal small", 31, [synth.CamSpec(320, 180, 3, 8, 0, p) for p in range(4)])
    ob = synth.MovingObject(x0=250.0, y0=100, w=60, h=40, speed=12.0)
    seen = removal_sequence(spec, rt.Options(n_blocks=8, band_width=16), 10, (ob,))
    assert rc.METHOD_REMOVAL in seen


def test_small_rig_object_covering_blocks_takes_the_fallback():
    """A tall object over a whole band block: the fallback (smoothing) is taken
    there.  It moves by half the period of its stripes per frame, so every
    pixel of it changes between frames and none of the covered band remains."""
    say("case: removal sequence, fallback")
    spec = synth.RigSpec("removal cover", 32, [synth.CamSpec(128, 64, 3, 8, 0, p) for p in range(3)])
    ob = synth.MovingObject(x0=100.0, y0=0, w=40, h=64, speed=8.0)
    seen = removal_sequence(spec, rt.Options(n_blocks=4, band_width=8, smoothing=True), 6, (ob,))
    assert rc.METHOD_SMOOTHING in seen and rc.METHOD_REMOVAL in seen


def test_rig14_object_crossing_full_size():
    """The full 14x1920x1080 rig, an object crossing the seam between cameras
    0 and 1, five frame-sets (checked on every one)."""
    say("case: removal sequence, 14x1920x1080 rgb8")
    spec = synth.rig14_1080p()
    ob = synth.seam_crossing(spec, 0, speed=48.0, frames=5)
    removal_sequence(spec, rt.Options(), 5, (ob,), check_every=1)


def test_uneven_rig_removal():
    say("case: removal sequence, uneven rig")
    spec = synth.uneven_rig()
    ob = synth.seam_crossing(spec, 1, speed=64.0, frames=3)
    removal_sequence(spec, rt.Options(), 3, (ob,))


def test_no_previous_frames_equals_the_plain_frameset():
    say("case: removal without previous frames == rt_frameset")
    spec = synth.RigSpec("removal plain", 33, [synth.CamSpec(200, 90, 3, 8, 0, p) for p in range(3)]
                         + [synth.CamSpec(64, 40, 1, 12, 1, p) for p in range(2)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=6, band_width=12, smoothing=True)
    a, b = rt.Rig(cams, opts), rt.Rig(cams, opts)
    kept, method = kept_buf(b)
    oa, ob_ = a.alloc_frames(), b.alloc_frames()
    for t in range(3):
        dev = a.upload(synth.rig_frames(spec, t, drift=True))
        a.frameset(dev, oa)
        b.frameset_removal(dev, None, ob_, kept, method)
        torch.cuda.synchronize()
        ha, hb = a.bufs.host(), b.bufs.host()
        for n in ("band_hist", "band_sums", "whole_hist", "whole_sums", "params", "valid", "lut8", "q16", "weights"):
            assert np.array_equal(ha[n], hb[n]), n
        for x, y in zip(a.download(oa), b.download(ob_)):
            assert np.array_equal(x, y)
    a.close()
    b.close()


def test_removal_validation():
    spec = [synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(2)]
    rig = rt.Rig(rt_cams(spec), rt.Options(n_blocks=2, band_width=8))
    dev, out = rig.alloc_frames(), rig.alloc_frames()
    kept, method = kept_buf(rig)
    with pytest.raises(rt.RtError, match="tau"):
        rig.frameset_removal(dev, dev, out, kept, method, tau=-1)
    with pytest.raises(rt.RtError, match="min_kept"):
        rig.frameset_removal(dev, dev, out, kept, method, min_kept=1.5)
    with pytest.raises(rt.RtError, match="kept_sums"):
        rt.rt_motion_stats(rig.ctx, dev, dev, 20, 0.25, rig.bufs.band_hist, rig.bufs.band_sums, None)
    with pytest.raises(rt.RtError, match="prev_frames"):
        rig.frameset_removal(dev, [dev[0], None], out, kept, method)
    rig.check()
    rig.close()


@pytest.mark.parametrize("lanes,group,fuse", [(1, 1, False), (3, 3, False), (2, 3, True)])
def test_pipeline_removal_matches_eager_and_oracle(lanes, group, fuse):
    """Object removal through the frame-set pipeline (each frame-set compared
    with the one submitted before it) over 9 frame-sets with an object
    crossing a seam: every output, the final state, kept sums and methods
    equal consecutive rt_frameset_removal calls, and the outputs the oracle's
    removal sequence; turning removal off gives the plain pipeline again."""
    say(f"case: pipeline removal lanes {lanes} group {group} fuse {fuse}, 4x320x180 rgb8, 9 frame-sets")
    spec = synth.RigSpec("pipe removal", 41, [synth.CamSpec(320, 180, 3, 8, 0, p) for p in range(4)])
    ob = synth.MovingObject(x0=250.0, y0=100, w=60, h=40, speed=12.0)
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, band_width=16, smoothing=True)
    T = 9
    frames = [synth.rig_frames(spec, t, drift=True, objects=(ob,)) for t in range(T)]
    # eager sequence
    seq = rt.Rig(cams, opts)
    kept_s, method_s = kept_buf(seq)
    dev = [seq.upload(f) for f in frames]
    out_s = seq.alloc_frames()
    eager = []
    for t in range(T):
        seq.frameset_removal(dev[t], dev[t - 1] if t else None, out_s, kept_s, method_s)
        torch.cuda.synchronize()
        eager.append(seq.download(out_s))
    hs = seq.bufs.host()
    # pipeline
    par = rt.Rig(cams, opts)
    kept_p, method_p = kept_buf(par)
    outs = [par.alloc_frames() for _ in range(T)]
    pipe = rt.Pipe.for_rig(par, depth=8, lanes=lanes, group=group, fuse=fuse)
    pipe.set_removal(kept_p, method_p)
    for t in range(T):
        pipe.submit(dev[t], outs[t])
    pipe.join()
    torch.cuda.synchronize()
    par.check()
    for t in range(T):
        for k, (a, b) in enumerate(zip(par.download(outs[t]), eager[t])):
            assert np.array_equal(a, b), f"frame-set {t} camera {k}"
    hp = par.bufs.host()
    assert np.array_equal(hp["params"].view(np.uint64), hs["params"].view(np.uint64))
    assert np.array_equal(hp["valid"], hs["valid"])
    assert np.array_equal(kept_p.cpu().numpy(), kept_s.cpu().numpy())
    assert np.array_equal(method_p.cpu().numpy(), method_s.cpu().numpy())
    # the oracle's removal sequence on the same frames
    co, oo = oracle_cams(cams), oracle_opts(opts)
    pp = pv = None
    seen = set()
    for t in range(T):
        ref = rc.frameset_removal(co, oo, frames[t], frames[t - 1] if t else None, pp, pv)
        pp, pv = ref["params"], ref["valid"]
        seen |= set(np.unique(ref["method"]).tolist())
        for k, (a, b) in enumerate(zip(par.download(outs[t]), ref["out"])):
            assert_ints_equal(a, b, f"oracle t {t} camera {k}")
    assert rc.METHOD_REMOVAL in seen
    # removal off: the next frame-sets follow the plain pipeline
    pipe.set_removal(None, on=False)
    extra = [synth.rig_frames(spec, T + t, drift=True) for t in range(2)]
    dx = [par.upload(f) for f in extra]
    ox = [par.alloc_frames() for _ in range(2)]
    for t in range(2):
        pipe.submit(dx[t], ox[t])
    pipe.join()
    torch.cuda.synchronize()
    for t in range(2):
        seq.frameset(dx[t], out_s)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(par.download(ox[t]), seq.download(out_s))):
            assert np.array_equal(a, b), f"after removal off: frame-set {t} camera {k}"
    pipe.close()
    seq.close()
    par.close()


def test_pipeline_removal_validation():
    say("case: pipeline removal validation")
    spec = synth.RigSpec("pipe removal val", 42, [synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(2)])
    cams = rt_cams(spec.cams)
    lib = rt.load()
    q = rt.Rig(cams, rt.Options(n_blocks=2, band_width=8, fit="quantile"))
    kq, _ = kept_buf(q)
    pq = rt.Pipe.for_rig(q, depth=2)
    ro = rt.rt_removal_opts(20, 0, 0.25)
    assert lib.rt_pipe_set_removal(pq.handle, ct.byref(ro), rt._p(kq), None) == rt.RT_EUNSUPPORTED
    pq.close()
    q.close()
    rig = rt.Rig(cams, rt.Options(n_blocks=2, band_width=8))
    kept, _ = kept_buf(rig)
    pipe = rt.Pipe.for_rig(rig, depth=2)
    for tau, mk in [(-1, 0.25), (256, 0.25), (20, -0.1), (20, 1.5), (20, float("nan"))]:
        bad = rt.rt_removal_opts(tau, 0, mk)
        assert lib.rt_pipe_set_removal(pipe.handle, ct.byref(bad), rt._p(kept), None) == rt.RT_EINVAL, (tau, mk)
    assert lib.rt_pipe_set_removal(pipe.handle, ct.byref(ro), None, None) == rt.RT_EINVAL
    # in place: refused while removal is on, accepted once it is off
    pipe.set_removal(kept)
    dev = rig.upload(synth.rig_frames(spec, 0))
    with pytest.raises(rt.RtError, match="in-place"):
        pipe.submit(dev, dev)
    assert lib.rt_pipe_set_removal(pipe.handle, None, None, None) == rt.RT_OK
    pipe.submit(dev, dev)
    pipe.join()
    torch.cuda.synchronize()
    rig.check()
    pipe.close()
    rig.close()
