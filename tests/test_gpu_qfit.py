"""GPU parity of the quantile least-squares fit (option fit = "quantile": the
affine map of section 3.1 fitted by least squares on 64 quantiles of the two
facing bands instead of their two moments) against the oracle: parameters bit
for bit (exact integer sums, one binary64 division), tables and pixels, through
rt_estimate (one wave per unit), the fused frame-set kernel in both of its
forms (512 threads up to 64 seam blocks, 256 beyond), smoothing over several
frame-sets, the pipeline, the 14x1920x1080 rig, and the entry points that
refuse the option."""
import ctypes as ct

import numpy as np
import pytest

from tests.gpu_helpers import assert_ints_equal, compare_step, oracle_cams, oracle_opts, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


CASES = [
    # (W, H, C, bit_depth, K, NB, closed)
    (40, 24, 3, 8, 3, 2, True),
    (67, 35, 3, 8, 2, 5, False),     # open chain: the outer sides face nothing
    (33, 40, 1, 8, 4, 7, True),
    (61, 45, 1, 12, 2, 4, True),
    (77, 66, 1, 16, 3, 16, True),
    (9, 20, 3, 8, 2, 20, True),      # one row per block, 4-column bands
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}c{c[2]}b{c[3]}k{c[4]}nb{c[5]}" for c in CASES])
def test_rt_estimate_quantile(case):
    W, H, C, bd, K, NB, closed = case
    say("case: quantile rt_estimate", case)
    rng = np.random.default_rng([91, W, H, C, bd, NB])
    cams = rt_cams([synth.CamSpec(W, H, C, bd, 0, p) for p in range(K)], pad=1)
    opts = rt.Options(n_blocks=NB, band_width=8, closed_ring=closed, fit="quantile", smoothing=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    pp = pv = None
    for t in range(3):
        frames = [synth.tiny_frame(H, W, C, bd, rng) for _ in range(K)]
        rig.stats(rig.upload(frames), whole=False)
        rig.estimate()
        torch.cuda.synchronize()
        h = rig.bufs.host()
        bh = np.stack([rc.band_stats(f, c, oo)[0] for f, c in zip(frames, co)])
        bs = np.stack([rc.band_stats(f, c, oo)[1] for f, c in zip(frames, co)])
        assert_ints_equal(h["band_hist"], bh, "band_hist")
        p, v = rc.estimate(co, oo, bs, pp, pv, band_hist=bh)
        assert_ints_equal(h["valid"], v, f"t {t} valid")
        assert np.array_equal(h["params"].view(np.uint64), p.view(np.uint64)), f"t {t}: params"
        pp, pv = p, v
    rig.close()


@pytest.mark.parametrize("K,NB", [(3, 16), (5, 16)], ids=["wide-48-seam-blocks", "narrow-80-seam-blocks"])
def test_frameset_quantile(K, NB):
    spec = synth.RigSpec(f"quantile {K}x200x96", 92, [synth.CamSpec(200, 96, 3, 8, 0, p) for p in range(K)])
    cams = rt_cams(spec.cams)
    opts = rt.Options(n_blocks=NB, fit="quantile", smoothing=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    out = rig.alloc_frames()
    pp = pv = None
    for t in range(3):
        say(f"case: quantile frame-set K={K} t={t}")
        frames = synth.rig_frames(spec, t, drift=True)
        rig.frameset(rig.upload(frames), out)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        h["out"] = rig.download(out)
        r = compare_step(co, oo, frames, h, pp, pv)
        assert r["bitwise"], f"t {t}: params not bitwise equal"
        pp, pv = r["ref"]["params"], r["ref"]["valid"]
    rig.close()


def test_quantile_differs_from_moments_and_pipeline_matches():
    """The two fits give different maps on the same frames, and three
    frame-sets through the pipeline (2 lanes) equal consecutive frame-sets."""
    spec = synth.RigSpec("quantile pipe 4x160x64", 93, [synth.CamSpec(160, 64, 3, 8, 0, p) for p in range(4)])
    cams = rt_cams(spec.cams)
    frames = [synth.rig_frames(spec, t, drift=True) for t in range(3)]
    res = {}
    for fit in ("moments", "quantile"):
        rig = rt.Rig(cams, rt.Options(n_blocks=8, fit=fit, smoothing=True))
        out = rig.alloc_frames()
        for f in frames:
            rig.frameset(rig.upload(f), out)
        torch.cuda.synchronize()
        res[fit] = (rig.bufs.host()["params"], rig.download(out))
        rig.close()
    assert not np.array_equal(res["moments"][0], res["quantile"][0])
    rig = rt.Rig(cams, rt.Options(n_blocks=8, fit="quantile", smoothing=True))
    pipe = rt.Pipe.for_rig(rig, depth=4, lanes=2, group=1)
    dev = [rig.upload(f) for f in frames]
    outs = [rig.alloc_frames() for _ in frames]
    torch.cuda.synchronize()
    for t in range(3):
        pipe.submit(dev[t], outs[t])
    pipe.join()
    torch.cuda.synchronize()
    assert np.array_equal(rig.bufs.host()["params"].view(np.uint64), res["quantile"][0].view(np.uint64))
    for k, (a, b) in enumerate(zip(rig.download(outs[2]), res["quantile"][1])):
        assert_ints_equal(a, b, f"pipeline camera {k}")
    pipe.close()
    rig.close()


def test_rig14_quantile_frameset():
    spec = synth.rig14_1080p()
    cams = rt_cams(spec.cams)
    opts = rt.Options(fit="quantile")
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    say("case: quantile frame-set rig14")
    frames = synth.rig_frames(spec, 0)
    out = rig.alloc_frames()
    rig.frameset(rig.upload(frames), out)
    torch.cuda.synchronize()
    h = rig.bufs.host()
    h["out"] = rig.download(out)
    assert compare_step(co, oo, frames, h)["bitwise"]
    rig.close()


def test_quantile_option_validation():
    cams = rt_cams([synth.CamSpec(64, 32, 3, 8, 0, p) for p in range(2)])
    with pytest.raises(ValueError):
        rt.Options(fit="median").to_c()
    o = rt.Options().to_c()
    o.fit = 7
    arr = (rt.rt_camera_desc * 2)(*[rt.rt_camera_desc(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos,
                                                       c.pitch_bytes) for c in cams])
    ctx = ct.c_void_p()
    assert rt.load().rt_ctx_create(arr, 2, ct.byref(o), ct.byref(ctx)) == rt.RT_EINVAL
    rig = rt.Rig(cams, rt.Options(n_blocks=4, fit="quantile"))
    frames = rig.upload([np.zeros((32, 64, 3), np.uint8)] * 2)
    out = rig.alloc_frames()
    kept = torch.zeros(tuple(rig.bufs.band_sums.shape), dtype=torch.int64, device="cuda")
    with pytest.raises(rt.RtError) as e:
        rig.frameset_removal(frames, None, out, kept)
    assert e.value.status == rt.RT_EUNSUPPORTED
    p_new = torch.zeros(tuple(rig.bufs.params.shape), dtype=torch.float64, device="cuda")
    status = torch.zeros(tuple(rig.bufs.valid.shape), dtype=torch.int32, device="cuda")
    with pytest.raises(rt.RtError) as e:
        rt.rt_estimate_new(rig.ctx, rig.bufs.band_sums, p_new, status)
    assert e.value.status == rt.RT_EUNSUPPORTED
    rig.close()
