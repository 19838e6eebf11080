"""Pins of the oracle's seam gradient cost (section 4.2, the gradient-cost
equation with frames downsampled by a factor in both directions) and of its
rig-wide form (every seam of every ring, plus the interior reference at each
image centre).

Independent checks: a pure-Python brute force with exact rationals (box sums
by loops, no numpy reshapes), the ring adjacency written out by hand, and
closed forms for ramps and two-tone images."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ringcorr as rc


def brute_rows(left, right, f):
    """Row values (d+ + d-)/2 by loops: exact box means as Fractions, the
    Euclidean norms as exact squared sums, one square root each."""
    H = min(len(left), len(right))
    n = H // f
    Wl, Wr, C = len(left[0]), len(right[0]), len(left[0][0])
    if n == 0 or Wl < 2 * f or Wr < 2 * f:
        return []

    def box(img, r0, c0, ch):
        s = 0
        for r in range(r0, r0 + f):
            for c in range(c0, c0 + f):
                s += int(img[r][c][ch])
        return Fraction(s, f * f)

    out = []
    for i in range(n):
        sp = sm = Fraction(0)
        for ch in range(C):
            im1 = box(left, i * f, Wl - 2 * f, ch)     # second box column left of the seam
            im0 = box(left, i * f, Wl - f, ch)         # box column touching the seam, left side
            ip0 = box(right, i * f, 0, ch)             # box column touching the seam, right side
            ip1 = box(right, i * f, f, ch)
            sp += ((ip1 - ip0) - (ip0 - im0)) ** 2
            sm += ((im1 - im0) - (im0 - ip0)) ** 2
        out.append((math.sqrt(sp) + math.sqrt(sm)) / 2)
    return out


@pytest.mark.parametrize("f", [1, 2, 3, 8])
@pytest.mark.parametrize("C,maxv", [(3, 255), (1, 255), (1, 4095)])
def test_rows_against_brute_force(f, C, maxv):
    rng = np.random.default_rng([7, f, C, maxv])
    for _ in range(3):
        hl, hr = int(rng.integers(f, 5 * f + 3)), int(rng.integers(f, 5 * f + 3))
        wl, wr = int(rng.integers(2 * f, 4 * f + 5)), int(rng.integers(2 * f, 4 * f + 5))
        dt = np.uint8 if maxv == 255 else np.uint16
        L = rng.integers(0, maxv + 1, (hl, wl, C)).astype(dt)
        R = rng.integers(0, maxv + 1, (hr, wr, C)).astype(dt)
        got = rc.seam_row_costs(L, R, f)
        ref = brute_rows(L.tolist(), R.tolist(), f)
        assert got.shape == (len(ref),)
        for g, r in zip(got, ref):
            assert abs(g - r) <= 1e-12 * max(1.0, r)
        if ref:
            assert abs(rc.seam_cost(L, R, f) - sum(ref) / len(ref)) <= 1e-12 * max(1.0, max(ref))


def test_left_right_roles_are_not_symmetric():
    """Swapping the images changes the cost (which side is I- matters)."""
    rng = np.random.default_rng(3)
    L = rng.integers(0, 256, (16, 16, 3)).astype(np.uint8)
    R = rng.integers(0, 256, (16, 16, 3)).astype(np.uint8)
    assert rc.seam_cost(L, R, 8) != rc.seam_cost(R, L, 8)
    assert rc.seam_cost(L, R, 8) == pytest.approx(float(np.mean(brute_rows(L.tolist(), R.tolist(), 8))), rel=1e-12)


def test_undefined_cases():
    img = np.zeros((7, 40, 3), np.uint8)
    assert math.isnan(rc.seam_cost(img, img, 8))              # shorter than one box
    narrow = np.zeros((16, 15, 3), np.uint8)
    wide = np.zeros((16, 16, 3), np.uint8)
    assert math.isnan(rc.seam_cost(narrow, wide, 8))          # left narrower than two boxes
    assert math.isnan(rc.seam_cost(wide, narrow, 8))
    assert rc.seam_cost(wide, wide, 8) == 0.0
    assert math.isnan(rc.interior_cost(np.zeros((16, 31, 3), np.uint8), 8))   # halves 15 and 16 wide
    assert rc.interior_cost(np.zeros((16, 32, 3), np.uint8), 8) == 0.0


def test_mismatched_heights_use_the_top_rows_of_the_shorter():
    rng = np.random.default_rng(11)
    L = rng.integers(0, 256, (40, 24, 3)).astype(np.uint8)
    R = rng.integers(0, 256, (27, 24, 3)).astype(np.uint8)
    rows = rc.seam_row_costs(L, R, 8)
    assert rows.shape == (3,)
    assert np.array_equal(rows, rc.seam_row_costs(L[:24], R[:24], 8))


def test_interior_closed_forms():
    # A horizontal ramp continues across the centre: cost 0 (box means of a ramp are a ramp).
    x = np.arange(64, dtype=np.int64)
    ramp = np.broadcast_to((40 + 2 * x)[None, :, None], (24, 64, 3)).astype(np.uint8)
    assert rc.interior_cost(ramp, 8) == 0.0
    # Two tones u | v at the centre: d+ = d- = sqrt(C) |u - v|.
    for u, v, C in ((30, 200, 3), (90, 17, 1)):
        img = np.full((16, 48, C), u, np.uint8)
        img[:, 24:] = v
        assert rc.interior_cost(img, 8) == pytest.approx(math.sqrt(C) * abs(u - v), rel=1e-15)


def test_rig_enumerates_every_ring_seam():
    rng = np.random.default_rng(5)
    cams = [rc.Camera(32, 24, 3, 8, 0, 2), rc.Camera(40, 24, 3, 8, 0, 0), rc.Camera(24, 32, 3, 8, 0, 1),
            rc.Camera(48, 16, 1, 12, 1, 0), rc.Camera(32, 16, 1, 12, 1, 1), rc.Camera(16, 8, 3, 8, 2, 0)]
    frames = [rng.integers(0, (1 << c.bit_depth), (c.height, c.width, c.channels)).astype(
        np.uint8 if c.bit_depth == 8 else np.uint16) for c in cams]
    # Ring 0 by position: cam 1 (pos 0) -> cam 2 (pos 1) -> cam 0 (pos 2) -> back to cam 1.
    right_of = {1: 2, 2: 0, 0: 1, 3: 4, 4: 3, 5: 5}
    for closed in (True, False):
        r = rc.seam_costs(cams, rc.Options(closed_ring=closed), frames, 8)
        for k, cam in enumerate(cams):
            last = (k == 0) or (k == 4) or (k == 5)       # last position of its ring
            if last and not closed:
                assert math.isnan(r["seam"][k]) and r["seam_rows"][k].size == 0
            else:
                j = right_of[k]
                assert r["seam"][k] == rc.seam_cost(frames[k], frames[j], 8)
                assert np.array_equal(r["seam_rows"][k], rc.seam_row_costs(frames[k], frames[j], 8))
            expect_i = rc.interior_cost(frames[k], 8)
            assert (math.isnan(expect_i) and math.isnan(r["interior"][k])) or r["interior"][k] == expect_i
    # The one-camera ring faces itself: its seam is its own right edge against its own left edge.
    one = rc.seam_costs(cams[5:], rc.Options(), frames[5:], 8)
    assert one["seam"][0] == rc.seam_cost(frames[5], frames[5], 8)
