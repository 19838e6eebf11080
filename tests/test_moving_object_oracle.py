"""Section 4.1's comparison of the correction methods around a moving object
(standard correction, object removal, exponential smoothing; 16 and 64
vertical blocks), reproduced with the oracle on a synthetic scene: a striped
vehicle crosses the seam between the first two cameras of a three-camera
ring in the ground region, 12 frames.  The paper's claims, as measured
discolouration of the seam-side correction domains in the blocks the
vehicle overlaps (paper_1910_03517_amd.evaluate):

* the standard correction discolours the block next to the vehicle, with
  large and with small blocks;
* object removal looks natural while enough of the block remains, and
  degrades when the vehicle fills most of a block (64 blocks);
* exponential smoothing looks natural in general, but lags: the
  disturbance lingers after the crossing;
* object removal is preferred when applicable: with the automatic choice
  (removal where a quarter of both facing bands remains, smoothing
  elsewhere) the small blocks fare better than with removal alone.
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


def test_object_removal_is_natural_with_large_blocks_and_degrades_with_small(table):
    assert table[16, "removal"].max() < 0.1 * table[16, "standard"].max()
    assert table[16, "removal"].max() < 1.0
    assert table[64, "removal"].max() > 2.0 * table[16, "removal"].max()


def test_smoothing_is_natural_but_lags(table):
    for nb in (16, 64):
        s, st = table[nb, "smoothing"], table[nb, "standard"]
        assert s.max() < 0.2 * st.max()
        # after the crossing the standard correction is back to the reference, smoothing is not yet
        assert np.all(st[-3:] == 0.0) and np.all(s[-3:] > 0.0)


def test_automatic_choice_helps_small_blocks(table):
    assert table[64, "auto"].max() < table[64, "removal"].max()
    assert table[64, "auto"].max() <= table[64, "smoothing"].max()
