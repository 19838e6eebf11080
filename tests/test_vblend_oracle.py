"""Pins of the oracle's row-wise blend of adjacent blocks' maps (section 5:
convex combinations of the maps of adjacent blocks instead of one map per
block).  Independent checks: the row weights against exact rationals of the
block centres, rows at a centre taking that block's map exactly, maps equal
on every block leaving the plain result unchanged, identity maps leaving the
frame unchanged, and maps linear in the block index giving parameters that
follow the closed form of the blend."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ringcorr as rc


def centre(bounds, j):
    r0, r1 = bounds[j]
    return Fraction(r0 + r1 - 1, 2)


@pytest.mark.parametrize("H,NB", [(64, 4), (67, 5), (1080, 16), (1080, 64), (16, 16), (33, 32), (7, 1)])
def test_row_weights_against_rationals(H, NB):
    bounds = rc.block_bounds(H, NB)
    for r in range(H):
        a, b, v = rc.row_blend(H, NB, r)
        assert 0 <= v < 256 and 0 <= a <= b < NB
        j = rc.block_of_row(r, H, NB)
        assert j in (a, b)
        if a == b:
            assert v == 0
            # alone only before the first centre or from the last centre on
            assert (a == 0 and r <= centre(bounds, 0)) or (a == NB - 1 and r >= centre(bounds, NB - 1))
            continue
        assert b == a + 1 and centre(bounds, a) <= r < centre(bounds, b)
        exact = 256 * (Fraction(r) - centre(bounds, a)) / (centre(bounds, b) - centre(bounds, a))
        assert v == math.floor(exact + Fraction(1, 2))          # round half up


def test_blend_q16_closed_forms():
    for p in (-700000, -1, 0, 1, 65536, 8388607):
        for v in (0, 1, 128, 255):
            assert rc.blend_q16(p, p, v) == p                # equal parameters blend to themselves
    assert rc.blend_q16(0, 256, 128) == 128
    assert rc.blend_q16(0, 255, 128) == 128               # 127.5 + 0.5 floors to 128
    assert rc.blend_q16(-256, 0, 128) == -128
    assert rc.blend_q16(10, 20, 0) == 10


def random_frame(rng, H, W, C, bd):
    dt = np.uint8 if bd == 8 else np.uint16
    return rng.integers(0, 1 << bd, (H, W, C)).astype(dt)


@pytest.mark.parametrize("C,bd", [(3, 8), (1, 12)])
def test_equal_maps_on_every_block_match_the_plain_apply(C, bd):
    rng = np.random.default_rng([9, C, bd])
    cam = rc.Camera(23, 41, C, bd)
    nb = 6
    frame = random_frame(rng, cam.height, cam.width, C, bd)
    params = np.zeros((1, 2, nb, 3, 2))
    for s in (0, 1):
        for c in range(3):
            params[0, s, :, c] = (rng.uniform(0.6, 1.6), rng.uniform(-30, 30))
    lut8, qq = rc.build_luts([cam], rc.Options(n_blocks=nb), params)
    plain = rc.apply_camera(frame, cam, rc.Options(n_blocks=nb), lut8[0], qq[0])
    blended = rc.apply_camera(frame, cam, rc.Options(n_blocks=nb, vblend=True), lut8[0], qq[0])
    assert np.array_equal(plain, blended)


def test_identity_maps_leave_the_frame_unchanged():
    rng = np.random.default_rng(4)
    cam = rc.Camera(30, 20, 3, 8)
    frame = random_frame(rng, 20, 30, 3, 8)
    params = np.zeros((1, 2, 5, 3, 2))
    params[..., 0] = 1.0
    lut8, qq = rc.build_luts([cam], rc.Options(n_blocks=5), params)
    assert np.array_equal(rc.apply_camera(frame, cam, rc.Options(n_blocks=5, vblend=True), lut8[0], qq[0]), frame)


def test_rows_follow_the_blend_of_linear_block_parameters():
    """Offsets b_j = 8 j grey levels (a = 1) on both sides: a flat frame of
    value x corrected at the border column (weight 256) gives, row by row,
    x + the row's blended offset, rounded as the Q16 map rounds it."""
    H, W, nb = 40, 8, 4
    cam = rc.Camera(W, H, 1, 8)
    frame = np.full((H, W, 1), 100, np.uint8)
    params = np.zeros((1, 2, nb, 3, 2))
    params[..., 0] = 1.0
    for j in range(nb):
        params[0, :, j, :, 1] = 8.0 * j
    lut8, qq = rc.build_luts([cam], rc.Options(n_blocks=nb), params)
    out = rc.apply_camera(frame, cam, rc.Options(n_blocks=nb, vblend=True), lut8[0], qq[0])
    for r in range(H):
        a, b, v = rc.row_blend(H, nb, r)
        Bq = rc.blend_q16(8 * a * 65536, 8 * b * 65536, v)
        assert out[r, 0, 0] == (65536 * 100 + Bq + 32768) >> 16, r   # column 0: weight 256, the full map
        # ... which is the offset interpolated between the two block centres, to within rounding
        assert abs(Fraction(int(out[r, 0, 0])) - (100 + 8 * (a + Fraction(v, 256)))) <= Fraction(1, 2)


def test_short_frames_are_refused():
    cam = rc.Camera(8, 3, 3, 8)
    frame = np.zeros((3, 8, 3), np.uint8)
    with pytest.raises(ValueError):
        rc.apply_camera_vblend(frame, cam, rc.Options(n_blocks=4, vblend=True), np.zeros((2, 4, 3, 2), np.int64))
