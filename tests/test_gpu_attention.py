"""GPU parity of the difference approach of the attention mechanisms
(section 3.3) against the oracle: on-pixel counts per cell, window counts
and selected windows bit for bit, from tiny ragged rigs of every sample type
to the full 14x1920x1080 rig with a vehicle crossing a seam."""
import numpy as np
import pytest

from tests.gpu_helpers import assert_ints_equal, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import attention as at  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def check(rig, cams, frames, prev, tau, cell, m, theta, label):
    dev, pdev = rig.upload(frames), rig.upload(prev)
    cells, win, sel = rig.attention(dev, pdev, tau, cell, m, theta)
    torch.cuda.synchronize()
    cells, win, sel = cells.cpu().numpy(), win.cpu().numpy(), sel.cpu().numpy()
    for k, cam in enumerate(cams):
        ref = at.attention(frames[k], prev[k], cam.bit_depth, tau, cell, m, theta)
        hc, wc = ref["cells"].shape
        what = f"{label} cam {k} c{cell} m{m}"
        assert_ints_equal(cells[k, :hc, :wc], ref["cells"], what + " cells")
        assert not cells[k, hc:].any() and not cells[k, :, wc:].any(), what + ": cells beyond the camera"
        hw, ww = ref["windows"].shape
        if win.size:
            assert_ints_equal(win[k, :hw, :ww], ref["windows"], what + " windows")
            assert_ints_equal(sel[k, :hw, :ww], ref["selected"].astype(np.uint8), what + " selected")
            assert not win[k, hw:].any() and not win[k, :, ww:].any(), what + ": windows beyond the camera"
            assert not sel[k, hw:].any() and not sel[k, :, ww:].any(), what + ": selections beyond the camera"


def perturbed(frames, rng, bd, frac):
    out = []
    for f in frames:
        step = 30 << (bd - 8)
        d = rng.integers(-2 * step, 2 * step + 1, f.shape)
        mask = rng.random(f.shape[:2]) < frac
        out.append(np.clip(f.astype(np.int64) + d * mask[:, :, None], 0, (1 << bd) - 1).astype(f.dtype))
    return out


CASES = [
    # (widths, heights, C, bit_depth, cell, m, theta)
    ([13, 40, 9], [11, 30, 7], 3, 8, 4, 2, 3),      # ragged widths, a camera shorter than a cell row
    ([64, 64], [64, 48], 3, 8, 16, 3, 40),
    ([50, 31], [33, 20], 1, 8, 8, 1, 10),
    ([61, 77], [40, 45], 1, 12, 12, 2, 20),
    ([96, 33], [70, 64], 1, 16, 20, 3, 50),
    ([130, 70], [66, 90], 3, 8, 256, 1, 0),          # one cell per camera
    ([40], [40], 3, 8, 4, 11, 5),                     # window larger than the grid
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[2]}b{c[3]}cell{c[4]}m{c[5]}" for c in CASES])
def test_attention_small_rigs(case):
    widths, heights, C, bd, cell, m, theta = case
    say("case: attention", case)
    rng = np.random.default_rng([51, C, bd, cell, m])
    spec = [synth.CamSpec(w, h, C, bd, 0, p) for p, (w, h) in enumerate(zip(widths, heights))]
    cams = rt_cams(spec, pad=1)
    rig = rt.Rig(cams, rt.Options(n_blocks=4, band_width=4))
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in cams]
    prev = perturbed(frames, rng, bd, 0.3)
    for tau in (0, 20):
        check(rig, cams, frames, prev, tau, cell, m, theta, f"small tau {tau}")
    rig.close()


def test_attention_validation():
    cams = rt_cams([synth.CamSpec(32, 16, 3, 8, 0, p) for p in range(2)])
    rig = rt.Rig(cams, rt.Options(n_blocks=2, band_width=4))
    f = rig.alloc_frames()
    cells = torch.zeros((2, 4, 8), dtype=torch.int32, device="cuda")
    for kw, msg in ((dict(cell=6), "cell"), (dict(cell=260), "cell"), (dict(m=0), "m "), (dict(m=65), "m "),
                    (dict(tau=-1), "tau")):
        args = dict(tau=20, cell=4, m=2, theta=3)
        args.update(kw)
        with pytest.raises(rt.RtError, match=msg):
            rt.rt_attention(rig.ctx, f, f, args["tau"], args["cell"], args["m"], args["theta"], cells)
    with pytest.raises(rt.RtError, match="prev_frames"):
        rt.rt_attention(rig.ctx, f, [f[0], None], 20, 4, 2, 3, cells)
    rig.close()


def test_attention_full_rig_moving_vehicle():
    spec = synth.rig14_1080p()
    say("case: attention full rig", spec.name)
    cams = rt_cams(spec.cams)
    rig = rt.Rig(cams, rt.Options())
    ob = synth.seam_crossing(spec, 0, speed=24.0, frames=12)
    prev = synth.rig_frames(spec, 5, objects=(ob,))
    frames = synth.rig_frames(spec, 6, objects=(ob,))
    check(rig, cams, frames, prev, 20, 16, 8, 256, "rig14")
    # With low sensor noise (gains up to 2 amplify the default noise past tau
    # on a fifth of the pixels) the selected windows are those around the
    # vehicle: on cameras 0 and 1 only.
    prev = synth.rig_frames(spec, 5, objects=(ob,), noise_sigma=1.0)
    frames = synth.rig_frames(spec, 6, objects=(ob,), noise_sigma=1.0)
    check(rig, cams, frames, prev, 20, 16, 8, 256, "rig14 low noise")
    cells, win, sel = rig.attention(rig.upload(frames), rig.upload(prev), 20, 16, 8, 256)
    s = sel.cpu().numpy().reshape(len(cams), -1).sum(axis=1)
    assert s[0] + s[1] > 0 and s[2:].sum() == 0, s
    rig.close()
