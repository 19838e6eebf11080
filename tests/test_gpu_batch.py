"""GPU parity of rt_frameset_batch: frame-sets of a subset of the rings of one
context.  Every step is compared with the oracle (bit-exact statistics,
tables, pixels; parameters bitwise), each ring's results in the mix equal
those of the ring served alone, and nothing of an inactive camera changes."""
import ctypes as ct
import numpy as np
import pytest

from tests.gpu_helpers import compare_step, oracle_cams, oracle_opts, rt_cams, say, assert_ints_equal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1910_03517_amd import rt, synth  # noqa: E402

PER_CAMERA = ("band_hist", "band_sums", "whole_hist", "whole_sums", "params", "valid", "lut8", "q16", "weights")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def three_rings():
    cams = (synth.ring_of(3, 320, 96, ring=0) + synth.ring_of(2, 256, 64, ring=1)
            + synth.ring_of(4, 200, 50, ring=2))
    return synth.RigSpec("3 rings: 3x320x96 + 2x256x64 + 4x200x50 rgb8", 9, cams)


def ring_indices(spec, r):
    return sorted((i for i, c in enumerate(spec.cams) if c.ring == r), key=lambda i: spec.cams[i].pos)


def cam_mask(idx):
    m = 0
    for i in idx:
        m |= 1 << i
    return m


def slice_host(h, idx, w_max):
    out = {n: h[n][idx] for n in PER_CAMERA}
    out["weights"] = out["weights"][:, :w_max]
    return out


def ring_frames(spec, r, t):
    frames = synth.rig_frames(spec, t, drift=True)
    return [frames[i] for i in ring_indices(spec, r)]


@pytest.mark.parametrize("grid", [0, 5, 40])
def test_batched_rings_match_oracle_and_alone(grid):
    """grid 0: one workgroup per tile; 5: fewer workgroups than cameras (shares
    run across cameras and rings); 40: whole shares per camera."""
    spec = three_rings()
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=4, band_width=16, smoothing=True)
    mix = rt.Rig(cams, opts)
    mix.tune(16, grid)
    rings = spec.rings
    idx = {r: ring_indices(spec, r) for r in rings}
    sub_cams = {r: [cams[i] for i in idx[r]] for r in rings}
    alone = {r: rt.Rig(sub_cams[r], opts) for r in rings}
    in_mix = mix.alloc_frames()
    out_mix = mix.alloc_frames()
    t_of = {r: 0 for r in rings}
    prev = {r: (None, None) for r in rings}
    schedule = [(0, 1, 2), (0,), (1, 2), (1,), (0, 1, 2), (2,), (0, 2)]
    for step, active in enumerate(schedule):
        say(f"case: batch grid {grid} step {step} rings {active}")
        before = mix.bufs.host()
        out_before = mix.download(out_mix)
        frames_in = [None] * len(cams)
        frames_out = [None] * len(cams)
        mask = 0
        for r in active:
            fr = ring_frames(spec, r, t_of[r])
            for n, i in enumerate(idx[r]):
                raw = np.ascontiguousarray(fr[n]).view(np.uint8).reshape(cams[i].height, cams[i].row_bytes)
                in_mix[i][:, :cams[i].row_bytes].copy_(torch.from_numpy(raw))
                frames_in[i], frames_out[i] = in_mix[i], out_mix[i]
            mask |= cam_mask(idx[r])
        mix.frameset_batch(mask, frames_in, frames_out)
        torch.cuda.synchronize()
        h = mix.bufs.host()
        outs = mix.download(out_mix)
        for r in rings:
            if r in active:
                continue
            for i in idx[r]:
                for n in PER_CAMERA:
                    assert np.array_equal(h[n][i], before[n][i]), f"inactive camera {i}: {n} changed"
                assert np.array_equal(outs[i], out_before[i]), f"inactive camera {i}: output changed"
        for r in active:
            fr = ring_frames(spec, r, t_of[r])
            co, oo = oracle_cams(sub_cams[r]), oracle_opts(opts)
            g = slice_host(h, idx[r], max(c.width for c in sub_cams[r]))
            g["out"] = [outs[i] for i in idx[r]]
            res = compare_step(co, oo, fr, g, *prev[r])
            assert res["bitwise"], f"step {step} ring {r}: params not bitwise equal"
            prev[r] = (res["ref"]["params"], res["ref"]["valid"])
            # The same frame-set served alone, in its own context.
            a = alone[r]
            dev = a.upload(fr)
            o = a.alloc_frames()
            a.frameset(dev, o)
            torch.cuda.synchronize()
            ha = a.bufs.host()
            for n in PER_CAMERA:
                ga = ha[n] if n != "weights" else ha[n][:, :g["weights"].shape[1]]
                assert np.array_equal(ga, g[n]), f"step {step} ring {r}: {n} differs alone vs mix"
            for x, y in zip(a.download(o), g["out"]):
                assert np.array_equal(x, y), f"step {step} ring {r}: output differs alone vs mix"
            t_of[r] += 1
    for a in alone.values():
        a.close()
    mix.close()


def test_batch_mask_validation():
    spec = three_rings()
    cams = rt_cams(spec.cams)
    rig = rt.Rig(cams, rt.Options(n_blocks=2))
    dev = rig.alloc_frames()
    out = rig.alloc_frames()
    ring0 = cam_mask(ring_indices(spec, 0))
    for bad, needle in [(0, "empty"), (ring0 & ~1, "ring"), (1 << len(cams), "beyond")]:
        with pytest.raises(rt.RtError, match=needle):
            rig.frameset_batch(bad, dev, out)
    frames = [d if (ring0 >> i) & 1 else None for i, d in enumerate(dev)]
    with pytest.raises(rt.RtError, match="NULL"):
        rig.frameset_batch(ring0 | cam_mask(ring_indices(spec, 1)), frames, out)
    rig.frameset_batch(ring0, frames, [o if f is not None else None for o, f in zip(out, frames)])
    rig.check()
    rig.close()


def test_context_active_set_separate_calls():
    """rt_ctx_set_active restricts rt_stats / rt_estimate / rt_build_lut /
    rt_apply: a ring's results equal the oracle's, the other rings' buffers
    and outputs stay as they were."""
    spec = three_rings()
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=3, band_width=24)
    rig = rt.Rig(cams, opts)
    dev = rig.upload(synth.rig_frames(spec, 0))
    out = rig.alloc_frames()
    rig.frameset(dev, out)
    torch.cuda.synchronize()
    r = 2
    idx = ring_indices(spec, r)
    mask = cam_mask(idx)
    before = rig.bufs.host()
    out_before = rig.download(out)
    fr = ring_frames(spec, r, 5)
    for n, i in enumerate(idx):
        raw = np.ascontiguousarray(fr[n]).view(np.uint8).reshape(cams[i].height, cams[i].row_bytes)
        dev[i][:, :cams[i].row_bytes].copy_(torch.from_numpy(raw))
    rig.set_active(mask)
    fin = [d if (mask >> i) & 1 else None for i, d in enumerate(dev)]
    fout = [o if (mask >> i) & 1 else None for i, o in enumerate(out)]
    prev_p, prev_v = before["params"][idx], before["valid"][idx]
    say("case: set_active ring 2, separate calls")
    rig.stats(fin, whole=False)
    rig.estimate()
    rig.build_lut()
    rig.apply(fin, fout, whole=True)
    torch.cuda.synchronize()
    h = rig.bufs.host()
    outs = rig.download(out)
    for i in range(len(cams)):
        if (mask >> i) & 1:
            continue
        for n in PER_CAMERA:
            assert np.array_equal(h[n][i], before[n][i]), f"inactive camera {i}: {n} changed"
        assert np.array_equal(outs[i], out_before[i])
    sub = [cams[i] for i in idx]
    g = slice_host(h, idx, max(c.width for c in sub))
    g["out"] = [outs[i] for i in idx]
    res = compare_step(oracle_cams(sub), oracle_opts(opts), fr, g, prev_p, prev_v)
    assert res["bitwise"]
    # The context's set does not leak into rt_frameset_batch, and can be widened again.
    rig.set_active(cam_mask(range(len(cams))))
    rig.frameset(dev, out)
    rig.check()
    rig.close()


def test_pipe_submit_batch_validation():
    """rt_pipe_submit_batch rejects an empty mask, a mask that splits a ring,
    and a completion event on a pipeline that issues applies in groups; a
    rejected call enqueues nothing and the pipeline stays usable."""
    spec = three_rings()
    cams = rt_cams(spec.cams)
    rig = rt.Rig(cams, rt.Options(n_blocks=2))
    dev = rig.alloc_frames()
    out = rig.alloc_frames()
    ring0 = cam_mask(ring_indices(spec, 0))
    grouped = rt.Pipe.for_rig(rig, depth=4, lanes=2, group=2)
    for bad, needle in [(0, "empty"), (ring0 & ~1, "ring")]:
        with pytest.raises(rt.RtError, match=needle):
            grouped.submit_batch(bad, dev, out)
    with pytest.raises(rt.RtError, match="group 1"):
        grouped.submit_batch(ring0, dev, out, done_event=torch.cuda.Event())
    grouped.submit_batch(ring0, dev, out)
    grouped.join()
    grouped.close()
    single = rt.Pipe.for_rig(rig, depth=2, lanes=2, group=1)
    done = torch.cuda.Event()
    single.submit_batch(ring0, [d if (ring0 >> i) & 1 else None for i, d in enumerate(dev)],
                        [o if (ring0 >> i) & 1 else None for i, o in enumerate(out)], done_event=done)
    done.synchronize()
    single.join()
    single.close()
    rig.check()
    rig.close()



def test_pipe_submit_n_matches_single_submits():
    """rt_pipe_submit_n over 7 frame-sets (groups of 3, the last partial)
    gives the outputs, whole-frame statistics and state of seven single
    submits; a frame-set with a missing frame stops the call after the ones
    before it, which stay submitted."""
    spec = synth.RigSpec("submit_n 3x96x64", 77, [synth.CamSpec(96, 64, 3, 8, 0, p) for p in range(3)])
    cams = rt_cams(spec.cams)
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(7)]
    results = {}
    for how in ("single", "n"):
        rig = rt.Rig(cams, rt.Options(n_blocks=4, smoothing=True))
        pipe = rt.Pipe.for_rig(rig, depth=8, lanes=3, group=3)
        dev = [rig.upload(f) for f in frames]
        outs = [rig.alloc_frames() for _ in frames]
        torch.cuda.synchronize()
        if how == "single":
            slots = [pipe.submit(dev[t], outs[t]) for t in range(7)]
        else:
            slots = pipe.submit_n(dev[:4], outs[:4]) + pipe.submit_n(dev[4:], outs[4:])
        pipe.join()
        torch.cuda.synchronize()
        rig.check()
        results[how] = ([rig.download(o) for o in outs], rig.bufs.host()["params"],
                        pipe.whole[slots[-1]].whole_hist.cpu().numpy(), slots)
        pipe.close()
        rig.close()
    a, b = results["single"], results["n"]
    assert a[3] == b[3]
    for t in range(7):
        for k in range(3):
            assert np.array_equal(a[0][t][k], b[0][t][k]), (t, k)
    assert np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64))
    assert np.array_equal(a[2], b[2])
    rig = rt.Rig(cams, rt.Options(n_blocks=4))
    pipe = rt.Pipe.for_rig(rig, depth=4, lanes=2, group=2)
    dev = [rig.upload(f) for f in frames[:3]]
    outs = [rig.alloc_frames() for _ in range(3)]
    fa = rt.ptr_array_n(dev)
    fa[4] = None                                   # camera 1 of frame-set 1
    oa = rt.ptr_array_n(outs)
    slots = (ct.c_int32 * 3)()
    done = ct.c_int32()
    st = rt.load().rt_pipe_submit_n(pipe.handle, 3, fa, oa, None, slots, ct.byref(done))
    assert st == rt.RT_EINVAL and done.value == 1
    pipe.join()
    torch.cuda.synchronize()
    rig.check()
    pipe.close()
    rig.close()
