"""GPU parity of the row-wise blend of adjacent blocks' maps (section 5's
convex combinations of adjacent maps, option vblend) against the oracle:
corrected frames bit for bit (with and without the fused whole-frame
statistics, which stay bit-exact), over small ragged rigs of every sample
type, random per-block maps (the row-blended direct path of 8-bit maps and
the per-sample path of maps beyond 24 bits and of 16-bit samples), and whole
frame-sets up to the 14x1920x1080 rig."""
import numpy as np
import pytest

from tests.gpu_helpers import assert_ints_equal, oracle_cams, oracle_opts, rt_cams, say

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
    # (W, H, C, bit_depth, K, NB)
    (37, 16, 3, 8, 2, 16),       # one row per block
    (64, 67, 3, 8, 3, 5),
    (33, 40, 1, 8, 2, 7),
    (61, 45, 1, 12, 2, 4),
    (77, 66, 1, 16, 2, 16),
    (130, 300, 3, 8, 2, 64),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}c{c[2]}b{c[3]}nb{c[5]}" for c in CASES])
def test_vblend_apply_random_maps(case):
    W, H, C, bd, K, NB = case
    say("case: vblend apply", case)
    rng = np.random.default_rng([61, W, H, C, bd, NB])
    spec = [synth.CamSpec(W, H, C, bd, 0, p) for p in range(K)]
    cams = rt_cams(spec, pad=1)
    opts = rt.Options(n_blocks=NB, band_width=8, vblend=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    frames = [synth.tiny_frame(H, W, C, bd, rng) for _ in range(K)]
    dev, out = rig.upload(frames), rig.alloc_frames()
    params = np.zeros(tuple(rig.bufs.params.shape))
    params[..., 0] = rng.uniform(0.5, 2.0, params.shape[:-1])
    params[..., 1] = rng.uniform(-40, 40, params.shape[:-1]) * (1 << (bd - 8))
    rig.bufs.params.copy_(torch.as_tensor(params, device="cuda"))
    rig.bufs.valid.fill_(1)
    rig.build_lut()
    for whole in (True, False):
        rig.apply(dev, out, whole=whole)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        got = rig.download(out)
        for k in range(K):
            ref = rc.apply_camera(frames[k], co[k], oo, h["lut8"][k], h["q16"][k])
            assert_ints_equal(got[k], ref, f"cam {k} whole={whole}")
        if whole:
            for k in range(K):
                wh, ws = rc.whole_stats(frames[k], co[k])
                assert_ints_equal(h["whole_hist"][k], wh, f"cam {k} whole_hist")
                assert_ints_equal(h["whole_sums"][k], ws, f"cam {k} whole_sums")
    rig.close()


def test_vblend_apply_maps_beyond_24_bits():
    """8-bit maps with gains of a few hundred (|A| >= 2^23) cannot be
    evaluated in 32-bit integers: those segments take the per-sample 64-bit
    path, the others the row-blended direct one, in the same launch."""
    rng = np.random.default_rng(63)
    W, H, K, NB = 96, 48, 2, 6
    spec = [synth.CamSpec(W, H, 3, 8, 0, p) for p in range(K)]
    cams = rt_cams(spec, pad=1)
    opts = rt.Options(n_blocks=NB, band_width=8, vblend=True)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    frames = [synth.tiny_frame(H, W, 3, 8, rng) for _ in range(K)]
    dev, out = rig.upload(frames), rig.alloc_frames()
    params = np.zeros(tuple(rig.bufs.params.shape))
    params[..., 0] = rng.uniform(0.5, 2.0, params.shape[:-1])
    params[..., 1] = rng.uniform(-40, 40, params.shape[:-1])
    params[1, :, 3:, :, 0] = rng.uniform(150, 300, params[1, :, 3:, :, 0].shape)    # camera 1, lower blocks
    rig.bufs.params.copy_(torch.as_tensor(params, device="cuda"))
    rig.bufs.valid.fill_(1)
    rig.build_lut()
    assert np.abs(rig.bufs.host()["q16"][1, :, 3:, :, 0]).min() >= 1 << 23
    for whole in (True, False):
        rig.apply(dev, out, whole=whole)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        for k, g in enumerate(rig.download(out)):
            assert_ints_equal(g, rc.apply_camera(frames[k], co[k], oo, h["lut8"][k], h["q16"][k]), f"cam {k} whole={whole}")
        if whole:
            for k in range(K):
                assert_ints_equal(h["whole_hist"][k], rc.whole_stats(frames[k], co[k])[0], f"cam {k} whole_hist")
    rig.close()


@pytest.mark.parametrize("which", ["small", "rig14"])
def test_vblend_frameset(which):
    if which == "small":
        spec = synth.RigSpec("vblend 3x320x120", 62, [synth.CamSpec(320, 120, 3, 8, 0, p) for p in range(3)])
        opts = rt.Options(n_blocks=16, vblend=True, smoothing=True)
        frames_t = range(3)
    else:
        spec = synth.rig14_1080p()
        opts = rt.Options(vblend=True)
        frames_t = range(1)
    say("case: vblend frame-set", spec.name)
    cams = rt_cams(spec.cams)
    rig = rt.Rig(cams, opts)
    co, oo = oracle_cams(cams), oracle_opts(opts)
    out = rig.alloc_frames()
    pp = pv = None
    for t in frames_t:
        frames = synth.rig_frames(spec, t, drift=True)
        rig.frameset(rig.upload(frames), out)
        torch.cuda.synchronize()
        h = rig.bufs.host()
        ref = rc.frameset(co, oo, frames, pp, pv)
        assert np.array_equal(h["params"].view(np.uint64), ref["params"].view(np.uint64)), f"t {t}: params"
        assert_ints_equal(h["q16"], ref["q16"], f"t {t}: q16")
        assert_ints_equal(h["whole_hist"], ref["whole_hist"], f"t {t}: whole_hist")
        for k, (g, r) in enumerate(zip(rig.download(out), ref["out"])):
            assert_ints_equal(g, r, f"t {t}: cam {k}")
        pp, pv = ref["params"], ref["valid"]
    rig.close()


def test_vblend_validation():
    cams = rt_cams([synth.CamSpec(32, 8, 3, 8, 0, p) for p in range(2)])
    with pytest.raises(rt.RtError, match="vblend"):
        rt.Rig(cams, rt.Options(n_blocks=16, vblend=True))        # 8 rows < 16 blocks
    rt.Rig(cams, rt.Options(n_blocks=8, vblend=True)).close()
