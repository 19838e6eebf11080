"""rt_surrogate_frameset_static, the entry point for callers that cannot
allocate (its workspace is the library's static device array), against
rt_surrogate_frameset with a caller workspace on a twin context: outputs,
statistics, estimator state and tables bit for bit, over two calls in a row
on one GPU, the second with a smaller rig (fewer units) so that the shared
array holds the first call's larger contents.  Plus the unit limit."""
import numpy as np
import pytest

from tests.gpu_helpers import rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1910_03517_amd import rt, synth  # noqa: E402
from paper_1910_03517_amd import surrogate as su  # noqa: E402

BUF_FIELDS = ("band_hist", "band_sums", "whole_hist", "whole_sums", "params", "valid", "lut8", "q16", "weights")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def one_rig(spec, opts, w, tol, frames_t):
    """The same frame-sets through the static entry point and through the
    workspace one (twin contexts); every result compared bit for bit."""
    cams = rt_cams(spec.cams)
    rigs = [rt.Rig(cams, opts) for _ in range(2)]
    ws = su.Workspace(rigs[1].sizes)
    outs = [r.alloc_frames() for r in rigs]
    used = 0
    for t in frames_t:
        dev = rigs[0].upload(synth.rig_frames(spec, t, drift=True))
        rt.rt_surrogate_frameset_static(rigs[0].ctx, w, tol, dev, outs[0], rigs[0].bufs, rigs[0].bufs.whole_hist)
        rt.rt_surrogate_frameset(rigs[1].ctx, w, tol, dev, outs[1], rigs[1].bufs, rigs[1].bufs.whole_hist, ws)
        torch.cuda.synchronize()
        ha, hb = rigs[0].bufs.host(), rigs[1].bufs.host()
        for n in BUF_FIELDS:
            assert np.array_equal(ha[n], hb[n]), f"{spec.name} t {t}: {n}"
        for x, y in zip(rigs[0].download(outs[0]), rigs[1].download(outs[1])):
            assert np.array_equal(x, y), f"{spec.name} t {t}: corrected frames"
        used += int(ws.used.sum().item())
    for r in rigs:
        r.check()
        r.close()
    return used


@pytest.mark.parametrize("tol", [0.05, 1e30])
def test_static_workspace_matches_caller_workspace(tol):
    w = rt.MlpTensors(synth.mlp_init(4))
    big = synth.RigSpec("6x480x272 rgb8", 21, [synth.CamSpec(480, 272, 3, 8, 0, p) for p in range(6)])
    small = synth.RigSpec("3x320x120 rgb8", 22, [synth.CamSpec(320, 120, 3, 8, 0, p) for p in range(3)])
    say(f"case: static surrogate frame-set, tol {tol}: {big.name} (192 units) then {small.name} (48 units)")
    u1 = one_rig(big, rt.Options(n_blocks=16, band_width=16, smoothing=True), w, tol, range(3))
    u2 = one_rig(small, rt.Options(n_blocks=8, band_width=16), w, tol, range(2))
    if tol == 1e30:
        assert u1 > 0 and u2 > 0


def test_static_workspace_unit_limit():
    say("case: static surrogate frame-set beyond RT_STATIC_UNITS")
    cams = [rt.Camera(8, 8, 3, 8, 0, p).with_pitch() for p in range(64)]
    rig = rt.Rig(cams, rt.Options(n_blocks=17, band_width=2))     # 64 x 2 x 17 = 2176 units
    w = rt.MlpTensors(synth.mlp_init(0))
    dev, out = rig.alloc_frames(), rig.alloc_frames()
    with pytest.raises(rt.RtError, match="static workspace"):
        rt.rt_surrogate_frameset_static(rig.ctx, w, 0.1, dev, out, rig.bufs, rig.bufs.whole_hist)
    rig.close()
