"""GPU parity of the seam gradient cost monitor (section 4.2, the
gradient-cost equation) against the oracle: every row value and every mean,
for every seam of every ring and the interior reference of every camera,
from tiny ragged rigs to the full 14x1920x1080 rig and the uneven rig, on
input and on corrected frames.

Bar: row values bit for bit where every step but the square roots is exact
in binary64 (one channel, or box areas that are powers of two: sums of
integers, exact divisions, exact squares); otherwise within 1e-15 relative
(the three channel squares may be added in another order).  Means within
1e-12 relative (the rows are summed in another order); NaN exactly where the
oracle has no row."""
import math

import numpy as np
import pytest

from tests.gpu_helpers import oracle_cams, oracle_opts, rt_cams, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ringcorr as rc  # noqa: E402
from paper_1910_03517_amd import rt, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rt.load()


def check(rig, cams, opts, frames_np, dev, factor, label):
    seam, interior, rows = rig.seam_cost(dev, factor, rows=True)
    torch.cuda.synchronize()
    seam, interior, rows = seam.cpu().numpy(), interior.cpu().numpy(), rows.cpu().numpy()
    ref = rc.seam_costs(oracle_cams(cams), oracle_opts(opts), frames_np, factor)
    pow2 = (factor & (factor - 1)) == 0
    for k, cam in enumerate(cams):
        exact = pow2 or cam.channels == 1
        for kind, (got_m, ref_m, ref_rows) in enumerate(((seam[k], ref["seam"][k], ref["seam_rows"][k]),
                                                         (interior[k], ref["interior"][k], ref["interior_rows"][k]))):
            what = f"{label} f{factor} cam {k} {'seam' if kind == 0 else 'interior'}"
            if ref_rows.size == 0:
                assert math.isnan(got_m) and math.isnan(ref_m), what
                continue
            g = rows[k, kind, :ref_rows.size]
            assert np.all(np.isnan(rows[k, kind, ref_rows.size:])), f"{what}: rows written past the seam's rows"
            if exact:
                bad = np.flatnonzero(g.view(np.uint64) != ref_rows.view(np.uint64))
                assert bad.size == 0, f"{what}: row {bad[0]} gpu {g[bad[0]]!r} ref {ref_rows[bad[0]]!r}"
            else:
                assert np.all(np.abs(g - ref_rows) <= 1e-15 * np.maximum(ref_rows, 1e-300)), what
            assert abs(got_m - ref_m) <= 1e-12 * max(abs(ref_m), 1e-300), f"{what}: mean {got_m!r} vs {ref_m!r}"


CASES = [
    # (widths, heights, C, bit_depth, closed, factors)
    ([16], [8], 3, 8, True, (8,)),                         # one camera facing itself, one box row
    ([40, 24, 33], [24, 24, 24], 3, 8, True, (1, 3, 8)),    # ragged widths, odd interior halves
    ([40, 24, 33], [24, 24, 24], 3, 8, False, (8,)),        # open chain: last seam undefined
    ([64, 48], [37, 29], 3, 8, True, (2, 8)),               # heights differ: rows of the shorter
    ([15, 64, 31], [16, 16, 16], 3, 8, True, (8,)),         # too narrow for two boxes
    ([48, 48], [7, 40], 3, 8, True, (8,)),                  # shorter than one box
    ([50, 70], [30, 30], 1, 8, True, (1, 5, 8)),            # gray8
    ([61, 40], [40, 33], 1, 12, True, (3, 8)),              # 12-bit
    ([77, 64, 90], [66, 66, 48], 1, 16, True, (4, 8, 64)),  # 16-bit, large factor
    ([256, 200], [200, 130], 3, 8, True, (64,)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"k{len(c[0])}c{c[2]}b{c[3]}{'c' if c[4] else 'o'}" for c in CASES])
def test_seam_cost_small_rigs(case):
    widths, heights, C, bd, closed, factors = case
    say("case: seam cost", case)
    rng = np.random.default_rng([31, len(widths), C, bd, int(closed)])
    spec = [synth.CamSpec(w, h, C, bd, 0, p) for p, (w, h) in enumerate(zip(widths, heights))]
    cams = rt_cams(spec, pad=1)
    opts = rt.Options(n_blocks=4, band_width=8, closed_ring=closed)
    rig = rt.Rig(cams, opts)
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in cams]
    dev = rig.upload(frames)
    for f in factors:
        check(rig, cams, opts, frames, dev, f, "small")
    rig.close()


def test_seam_cost_mixed_rings_and_active_set():
    """Two rings in one context; the active set restricts what is written."""
    rng = np.random.default_rng(8)
    spec = [synth.CamSpec(96, 48, 3, 8, 0, 1), synth.CamSpec(80, 48, 3, 8, 0, 0),
            synth.CamSpec(64, 40, 1, 16, 1, 0), synth.CamSpec(64, 40, 1, 16, 1, 1), synth.CamSpec(64, 40, 1, 16, 1, 2)]
    cams = rt_cams(spec)
    opts = rt.Options(n_blocks=4, band_width=8)
    rig = rt.Rig(cams, opts)
    frames = [synth.tiny_frame(c.height, c.width, c.channels, c.bit_depth, rng) for c in cams]
    dev = rig.upload(frames)
    check(rig, cams, opts, frames, dev, 8, "mixed")
    seam = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    interior = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    rig.set_active(0b00011)
    rt.rt_seam_cost(rig.ctx, [dev[0], dev[1], None, None, None], 8, seam, interior)
    torch.cuda.synchronize()
    s = seam.cpu().numpy()
    assert np.all(s[2:] == -1.0), "inactive cameras were written"
    ref = rc.seam_costs(oracle_cams(cams), oracle_opts(opts), frames, 8)
    assert abs(s[0] - ref["seam"][0]) <= 1e-12 * ref["seam"][0]
    rig.set_active((1 << 5) - 1)
    rig.close()


def test_seam_cost_validation():
    spec = [synth.CamSpec(32, 16, 3, 8, 0, p) for p in range(2)]
    cams = rt_cams(spec)
    rig = rt.Rig(cams, rt.Options(n_blocks=2, band_width=8))
    dev = rig.alloc_frames()
    seam = torch.zeros(2, dtype=torch.float64, device="cuda")
    inter = torch.zeros(2, dtype=torch.float64, device="cuda")
    for bad in (0, 65):
        with pytest.raises(rt.RtError, match="factor"):
            rt.rt_seam_cost(rig.ctx, dev, bad, seam, inter)
    rows = torch.zeros((2, 2, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(rt.RtError, match="row_stride"):
        rt.rt_seam_cost(rig.ctx, dev, 8, seam, inter, rows, 1)   # 16 / 8 = 2 rows needed
    with pytest.raises(rt.RtError, match="seam"):
        rt.rt_seam_cost(rig.ctx, dev, 8, None, inter)
    rig.close()


@pytest.mark.parametrize("which", ["rig14", "uneven"])
def test_seam_cost_full_rigs_input_and_corrected(which):
    """Full-size rigs in the bench's shapes: every seam and interior on the
    input frames and on the corrected output of one frame-set."""
    spec = synth.rig14_1080p() if which == "rig14" else synth.uneven_rig()
    say("case: seam cost full rig", spec.name)
    cams = rt_cams(spec.cams)
    opts = rt.Options()
    rig = rt.Rig(cams, opts)
    frames = synth.rig_frames(spec, 0)
    dev = rig.upload(frames)
    out = rig.alloc_frames()
    rig.frameset(dev, out)
    torch.cuda.synchronize()
    check(rig, cams, opts, frames, dev, 8, "input")
    corrected = rig.download(out)
    check(rig, cams, opts, corrected, out, 8, "corrected")
    # The correction lowers the seam cost of the distorted RGB cameras.
    rgb = [k for k, c in enumerate(cams) if c.channels == 3]
    s_in = rig.seam_cost(dev)[0].cpu().numpy()[rgb]
    s_out = rig.seam_cost(out)[0].cpu().numpy()[rgb]
    assert s_out.sum() < 0.5 * s_in.sum(), (s_in, s_out)
    rig.close()
