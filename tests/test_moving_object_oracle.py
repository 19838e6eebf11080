"""Section 4.1's comparison of the correction methods around a moving object
(standard correction, object removal, exponential smoothing; 16 and 64
vertical blocks), reproduced with the oracle on a synthetic scene: a striped
vehicle crosses the seam between the first two cameras of a three-camera
ring in the ground region, 12 frames.  Measured as the discolouration of the
seam-side correction domains in the blocks the vehicle overlaps
(paper_1910_03517_amd.evaluate), the paper's claims that this scene shows:

* the standard correction discolours the block next to the vehicle, with
  large and with small blocks, most right before and after the crossing;
* object removal looks natural;
* exponential smoothing looks natural in general, but lags: the disturbance
  lingers after the crossing;
* object removal is preferred when applicable: the automatic choice
  (removal where a quarter of both facing bands remains, smoothing
  elsewhere) does no worse than smoothing.

The paper also shows removal failing when the vehicle fills most of a block.
On this synthetic ground the few band pixels that remain are statistically
like the rest of the block, so removal stays natural there; the failure
needs remaining pixels that misrepresent the block, which the scene does not
model.
"""
import numpy as np
import pytest

from oracle import ringcorr as rc
from paper_1910_03517_amd import evaluate, synth

W, H, T = 320, 240, 12


def run(nb: int, mode: str):
    spec = synth.RigSpec("moving-object 3x320x240", 7, [synth.CamSpec(W, H, 3, 8, 0, p) for p in range(3)])
    ob = synth.seam_crossing(spec, 0, speed=24.0, frames=T, rows=(0.62, 0.665), width_frac=0.08)
    cams = [rc.Camera(W, H, 3, 8, 0, p) for p in range(3)]
    opts = rc.Options(n_blocks=nb, smoothing=(mode == "smoothing"))
    rows = evaluate.affected_rows(H, nb, ob.y0, ob.h)
    ml, mr = evaluate.seam_halves_mask(H, W, W, rows)
    runs = {}
    for tag, objs in (("obj", (ob,)), ("ref", ())):
        pp = pv = prev = None
        seq = []
        for t in range(T):
            fr = synth.rig_frames(spec, t, objects=objs)
            if mode in ("removal", "auto"):
                r = rc.frameset_removal(cams, opts, fr, prev, pp, pv, min_kept=0.0 if mode == "removal" else 0.25)
            else:
                r = rc.frameset(cams, opts, fr, pp, pv)
            pp, pv, prev = r["params"], r["valid"], fr
            seq.append((fr, r["out"]))
        runs[tag] = seq
    d = []
    for t in range(T):
        (fo, oo), (fr_, orf) = runs["obj"][t], runs["ref"][t]
        d.append(evaluate.discolouration([(fo[0], fr_[0], oo[0], orf[0], ml), (fo[1], fr_[1], oo[1], orf[1], mr)]))
    return np.array(d)


@pytest.fixture(scope="module")
def table():
    return {(nb, m): run(nb, m) for nb in (16, 64) for m in ("standard", "removal", "auto", "smoothing")}


def test_nothing_differs_before_the_vehicle_reaches_a_band(table):
    for d in table.values():
        assert np.all(d[:4] == 0.0)


def test_standard_correction_discolours_the_block_next_to_the_vehicle(table):
    for nb in (16, 64):
        assert table[nb, "standard"].max() > 5.0


def test_object_removal_is_natural(table):
    for nb in (16, 64):
        assert table[nb, "removal"].max() < 0.1 * table[nb, "standard"].max()
        assert table[nb, "removal"].max() < 1.0


def test_smoothing_is_natural_but_lags(table):
    for nb in (16, 64):
        s, st = table[nb, "smoothing"], table[nb, "standard"]
        assert s.max() < 0.2 * st.max()
        # after the crossing the standard correction is back to the reference, smoothing is not yet
        assert np.all(st[-3:] == 0.0) and np.all(s[-3:] > 0.0)


def test_automatic_choice_no_worse_than_smoothing(table):
    for nb in (16, 64):
        assert table[nb, "auto"].max() <= table[nb, "smoothing"].max()
        assert table[nb, "auto"].mean() <= table[nb, "smoothing"].mean()
