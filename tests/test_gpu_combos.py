"""GPU parity of the options combined (the oracle takes the same options):
maps blended between blocks with object removal, the quantile fit with the
blended maps on the uneven rig (8-bit RGB and 16-bit gray rings), and both
through the frame-set pipeline."""
import numpy as np
import pytest

from tests.gpu_helpers import compare_step, oracle_cams, oracle_opts, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def test_removal_with_blended_maps():
    from tests.test_gpu_removal import removal_sequence
    say("case: removal sequence with vblend, 4x320x180 rgb8")
    spec = synth.RigSpec("removal vblend", 33, [synth.CamSpec(320, 180, 3, 8, 0, p) for p in range(4)])
    ob = synth.MovingObject(x0=250.0, y0=100, w=60, h=40, speed=12.0)
    seen = removal_sequence(spec, rt.Options(n_blocks=8, band_width=16, vblend=True), 6, (ob,))
    assert rc.METHOD_REMOVAL in seen


def test_uneven_rig_quantile_fit_and_blended_maps():
    spec = synth.uneven_rig()
    cams = rt_cams(spec.cams)
    opts = rt.Options(fit="quantile", vblend=True, smoothing=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    out = rig.alloc_frames()
    pp = pv = None
    for t in range(2):
        say(f"case: uneven rig, quantile fit and vblend, t={t}")
        frames = synth.rig_frames(spec, t, drift=True)
        rig.frameset(rig.upload(frames), out)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        h["out"] = rig.download(out)
        r = compare_step(co, oo, frames, h, pp, pv)
        assert r["bitwise"], f"t {t}: parameters not bitwise equal"
        pp, pv = r["ref"]["params"], r["ref"]["valid"]
    rig.close()


def test_pipeline_with_quantile_fit_and_blended_maps():
    spec = synth.RigSpec("combo pipe 5x256x120", 34, [synth.CamSpec(256, 120, 3, 8, 0, p) for p in range(5)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=8, fit="quantile", vblend=True, smoothing=True)
    rig = rt.Rig(cams, opts)
    pipe = rt.Pipe.for_rig(rig, depth=8, lanes=3, group=3)
    n = 7
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(n)]
    dev = [rig.upload(f) for f in frames]
    outs = [rig.alloc_frames() for _ in range(n)]
    torch.cuda.synchronize()
    say("case: pipeline with quantile fit and vblend")
    pipe.submit_n(dev, outs)
    pipe.join()
    torch.cuda.synchronize()
    rig.check()
    co, oo = oracle_cams(cams), oracle_opts(opts)
    pp = pv = None
    for t in range(n):
        ref = rc.frameset(co, oo, frames[t], pp, pv)
        pp, pv = ref["params"], ref["valid"]
        for k, (x, y) in enumerate(zip(rig.download(outs[t]), ref["out"])):
            assert np.array_equal(x, y), f"frame-set {t} camera {k}"
    assert np.array_equal(rig.bufs.host()["params"].view(np.uint64), pp.view(np.uint64))
    pipe.close()
    rig.close()
