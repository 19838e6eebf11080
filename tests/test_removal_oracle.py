"""Pins of the oracle's object removal and smoothing fallback (section 3.1's
two supplemental methods for moving objects, with the automatic choice
between them): a hand-worked seam (tests/golden/removal_worked.json),
brute-force kept sums, the threshold and kept-fraction boundaries, exact
recovery of the object-free estimate, the fallback's closed form, and the
reduction to the plain method when nothing moves."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ringcorr as rc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def two_gray(col0, col1):
    """Two 2x4 gray8 frames: camera 0's right band column and camera 1's left band column."""
    f0 = np.full((4, 2, 1), 50, np.uint8)
    f1 = np.full((4, 2, 1), 50, np.uint8)
    f0[:, 1, 0] = col0
    f1[:, 0, 0] = col1
    return [f0, f1]


CAMS2 = [rc.Camera(2, 4, 1, 8, 0, 0), rc.Camera(2, 4, 1, 8, 0, 1)]
OPTS2 = rc.Options(n_blocks=1, band_width=1, closed_ring=False)


def test_worked_removal_golden():
    g = golden("removal_worked.json")
    now = two_gray(g["now0"], g["now1"])
    prev = two_gray(g["prev0"], g["prev1"])
    kept = np.stack([rc.kept_band_sums(f, p, c, OPTS2, 20) for f, p, c in zip(now, prev, CAMS2)])
    full = np.stack([rc.band_stats(f, c, OPTS2)[1] for f, c in zip(now, CAMS2)])
    assert kept[0, 1, 0, 0].tolist() == g["kept_sums_0"] and kept[1, 0, 0, 0].tolist() == g["kept_sums_1"]
    assert full[0, 1, 0, 0].tolist() == g["full_sums_0"] and full[1, 0, 0, 0].tolist() == g["full_sums_1"]
    params, valid, method = rc.estimate_removal(CAMS2, OPTS2, full, kept, min_kept=0.25)
    assert method[0, 1, 0] == rc.METHOD_REMOVAL and method[1, 0, 0] == rc.METHOD_REMOVAL
    assert method[0, 0, 0] == rc.METHOD_NONE and method[1, 1, 0] == rc.METHOD_NONE   # chain ends
    a0, b0 = params[0, 1, 0, 0]
    a1, b1 = params[1, 0, 0, 0]
    assert abs(a0 - g["a0"]) <= 4e-16 * g["a0"] and abs(b0 - g["b0"]) <= 1e-13
    assert abs(a1 - g["a1"]) <= 4e-16 * g["a1"] and abs(b1 - g["b1"]) <= 1e-13
    # Without removal the same seam gives a different map (the object counts).
    plain, _ = rc.estimate(CAMS2, OPTS2, full)
    assert abs(plain[0, 1, 0, 0, 0] - 1.5) > 0.1


@pytest.mark.parametrize("had_state", [False, True])
def test_worked_fallback_golden(had_state):
    g = golden("removal_worked.json")
    now = two_gray(g["now0"], g["now1"])
    prev = two_gray(g["fallback_prev0"], g["prev1"])
    kept = np.stack([rc.kept_band_sums(f, p, c, OPTS2, 20) for f, p, c in zip(now, prev, CAMS2)])
    full = np.stack([rc.band_stats(f, c, OPTS2)[1] for f, c in zip(now, CAMS2)])
    assert kept[0, 1, 0, 0, 0] == 0
    prev_p = np.zeros((2, 2, 1, 3, 2))
    prev_p[..., 0] = 1.0
    prev_v = np.full((2, 2, 1, 3), 1 if had_state else 0, np.uint8)
    params, valid, method = rc.estimate_removal(CAMS2, OPTS2, full, kept, prev_p, prev_v, 0.25)
    assert method[0, 1, 0] == rc.METHOD_SMOOTHING and method[1, 0, 0] == rc.METHOD_SMOOTHING
    s0, s1 = math.sqrt(g["fallback_var0"]), math.sqrt(g["fallback_var1"])
    mu_s = (g["fallback_mu0"] + g["fallback_mu1"]) / 2
    for (k, side, mu, sd) in ((0, 1, g["fallback_mu0"], s0), (1, 0, g["fallback_mu1"], s1)):
        a_new = (s0 + s1) / 2 / sd
        b_new = mu_s - a_new * mu
        a_exp = 0.95 + 0.05 * a_new if had_state else a_new
        b_exp = 0.05 * b_new if had_state else b_new
        a, b = params[k, side, 0, 0]
        assert abs(a - a_exp) <= 1e-15 * a_exp and abs(b - b_exp) <= 1e-12 * max(1.0, abs(b_exp))
        assert valid[k, side, 0, 0] == 1


def brute_kept(frame, prev, cam, opts, tau):
    """Pixel-by-pixel loop: block by closed form, band by column range."""
    nb = opts.n_blocks
    out = np.zeros((2, nb, 3, 3), np.int64)
    (l0, l1), (r0, r1) = rc.band_columns(cam.width, opts.band_width)
    thr = tau * (1 << (cam.bit_depth - 8))
    for r in range(cam.height):
        j = rc.block_of_row(r, cam.height, nb)
        for col in range(cam.width):
            sides = [s for s, (a, b) in ((0, (l0, l1)), (1, (r0, r1))) if a <= col < b]
            if not sides:
                continue
            moving = prev is not None and max(abs(int(frame[r, col, c]) - int(prev[r, col, c]))
                                              for c in range(cam.channels)) > thr
            if moving:
                continue
            for s in sides:
                for c in range(cam.channels):
                    x = int(frame[r, col, c])
                    out[s, j, c] += (1, x, x * x)
    return out


@pytest.mark.parametrize("C,bd", [(3, 8), (1, 8), (1, 12), (1, 16)])
def test_kept_sums_bruteforce(C, bd):
    rng = np.random.default_rng(30 + C + bd)
    for (H, W, NB, B, tau) in [(7, 9, 3, 2, 20), (5, 3, 8, 1, 0), (11, 16, 4, 5, 40), (4, 1, 2, 3, 20)]:
        cam = rc.Camera(W, H, C, bd)
        opts = rc.Options(n_blocks=NB, band_width=B)
        dt = np.uint8 if bd == 8 else np.uint16
        maxv = (1 << bd) - 1
        frame = rng.integers(0, maxv + 1, (H, W, C)).astype(dt)
        # previous frame: mostly within a few multiples of tau of this one
        step = max(1, tau) << (bd - 8)
        prev = np.clip(frame.astype(np.int64) + rng.integers(-2 * step, 2 * step + 1, (H, W, C)), 0, maxv).astype(dt)
        got = rc.kept_band_sums(frame, prev, cam, opts, tau)
        assert np.array_equal(got, brute_kept(frame, prev, cam, opts, tau))
        assert np.array_equal(rc.kept_band_sums(frame, None, cam, opts, tau), rc.band_stats(frame, cam, opts)[1])


def test_threshold_boundary_and_bit_depth_scaling():
    base = np.full((1, 1, 3), 100, np.uint8)
    for d, moving in ((20, False), (21, True), (-20, False), (-21, True)):
        prev = base.copy()
        prev[0, 0, 1] = 100 + d
        assert bool(rc.moving_mask(base, prev, 8, 20)[0, 0]) == moving
    x = np.full((1, 1, 1), 5000, np.uint16)
    assert not rc.moving_mask(x, x + 320, 12, 20)[0, 0]         # 20 << 4 = 320
    assert rc.moving_mask(x, x + 321, 12, 20)[0, 0]
    y = np.full((1, 1, 1), 60000, np.uint16)
    assert not rc.moving_mask(y, y - 5120, 16, 20)[0, 0]        # 20 << 8 = 5120
    assert rc.moving_mask(y, y - 5121, 16, 20)[0, 0]


def test_kept_fraction_boundary():
    """Exactly min_kept of a band kept -> removal; one pixel fewer -> fallback."""
    cams = [rc.Camera(2, 8, 1, 8, 0, 0), rc.Camera(2, 8, 1, 8, 0, 1)]
    opts = rc.Options(n_blocks=1, band_width=1, closed_ring=False)
    rng = np.random.default_rng(3)
    now = [rng.integers(30, 200, (8, 2, 1)).astype(np.uint8) for _ in range(2)]
    for n_moving, expect in ((6, rc.METHOD_REMOVAL), (7, rc.METHOD_SMOOTHING)):
        prev = [f.copy() for f in now]
        prev[0][:n_moving, 1, 0] = (now[0][:n_moving, 1, 0].astype(np.int64) + 100) % 256   # |diff| >= 100 > 20
        kept = np.stack([rc.kept_band_sums(f, p, c, opts) for f, p, c in zip(now, prev, cams)])
        full = np.stack([rc.band_stats(f, c, opts)[1] for f, c in zip(now, cams)])
        _, _, method = rc.estimate_removal(cams, opts, full, kept, min_kept=0.25)
        assert method[0, 1, 0] == expect and method[1, 0, 0] == expect, (n_moving, method)


def row_uniform_scene(H, W, rng):
    """RGB frame whose rows are all equal (values vary with the column only)."""
    row = rng.integers(20, 230, (1, W, 3))
    return np.repeat(row, H, axis=0).astype(np.uint8)


@pytest.mark.parametrize("smoothing", [False, True])
def test_removal_recovers_the_object_free_estimate_exactly(smoothing):
    """A bright object enters the band of one block between two frames,
    covering whole band rows.  The band rows all hold the same multiset, so
    dropping the object's rows keeps every moment: the removal estimate equals, bit for bit, the estimate of
    the frame without the object, while the plain estimate does not."""
    rng = np.random.default_rng(21)
    H, W, NB = 32, 24, 4
    cams = [rc.Camera(W, H, 3, 8, 0, p) for p in range(3)]
    opts = rc.Options(n_blocks=NB, band_width=6, smoothing=smoothing)
    clean = [row_uniform_scene(H, W, rng) for _ in range(3)]
    now = [f.copy() for f in clean]
    now[1][10:14, W - 9:] = (250, 30, 30)            # whole rows of camera 1's right band, block 1 (rows 8..15)
    prev_p = np.zeros((3, 2, NB, 3, 2))
    prev_p[..., 0] = rng.uniform(0.8, 1.2, (3, 2, NB, 3))
    prev_p[..., 1] = rng.uniform(-5, 5, (3, 2, NB, 3))
    prev_v = np.ones((3, 2, NB, 3), np.uint8)
    ref = rc.frameset(cams, opts, clean, prev_p, prev_v)
    got = rc.frameset_removal(cams, opts, now, clean, prev_p, prev_v)
    assert np.array_equal(got["params"].view(np.uint64), ref["params"].view(np.uint64))
    assert np.all(got["method"][[0, 1, 2], :, :] != rc.METHOD_NONE)
    assert got["method"][1, 1, 1] == rc.METHOD_REMOVAL and got["method"][2, 0, 1] == rc.METHOD_REMOVAL
    plain = rc.frameset(cams, opts, now, prev_p, prev_v)
    assert not np.array_equal(plain["params"][1, 1, 1], ref["params"][1, 1, 1])


def test_fallback_sequence_closed_form():
    """An object covering a whole band block every frame (its colour changes
    by more than tau each frame) keeps the unit on the fallback:
    p_t = p_new + (1 - alpha)^t (p_0 - p_new) for constant bands."""
    rng = np.random.default_rng(22)
    H, W = 16, 16
    cams = [rc.Camera(W, H, 3, 8, 0, p) for p in range(2)]
    opts = rc.Options(n_blocks=1, band_width=4, closed_ring=False)
    base = [rng.integers(40, 200, (H, W, 3)).astype(np.uint8) for _ in range(2)]
    p0 = rc.frameset(cams, opts, base)["params"]               # first estimate, nothing moving
    frames = [f.copy() for f in base]
    prev = [f.copy() for f in base]
    params, valid = p0, np.ones((2, 2, 1, 3), np.uint8)
    seq = []
    for t in range(1, 6):
        colour = 40 if t % 2 else 120
        frames[0][:, W - 4:] = colour                          # camera 0's right band entirely covered
        r = rc.frameset_removal(cams, opts, frames, prev, params, valid)
        assert r["method"][0, 1, 0] == rc.METHOD_SMOOTHING
        params, valid = r["params"], r["valid"]
        prev = [f.copy() for f in frames]
        seq.append(params[0, 1, 0].copy())
    # The fit of the full bands alternates with the colour: check each step's recurrence.
    p_prev = p0[0, 1, 0]
    for t, p in enumerate(seq, start=1):
        full = rc.frameset(cams, opts, [np.where(np.arange(W)[None, :, None] >= W - 4,
                                                 40 if t % 2 else 120, base[0]).astype(np.uint8), base[1]])
        p_new = full["params"][0, 1, 0]
        exp = 0.95 * p_prev + 0.05 * p_new
        assert np.allclose(p, exp, rtol=1e-15, atol=1e-13)
        p_prev = p


def test_nothing_moving_reduces_to_the_plain_method():
    rng = np.random.default_rng(23)
    cams = [rc.Camera(40, 30, 3, 8, 0, p) for p in range(3)] + [rc.Camera(20, 12, 1, 12, 1, 0)]
    for smoothing in (False, True):
        opts = rc.Options(n_blocks=4, band_width=5, smoothing=smoothing)
        frames = [rng.integers(0, 256 if c.bit_depth == 8 else 4096, (c.height, c.width, c.channels))
                  .astype(np.uint8 if c.bit_depth == 8 else np.uint16) for c in cams]
        prev_p = rng.uniform(0.5, 2, (4, 2, 4, 3, 2))
        prev_v = rng.integers(0, 2, (4, 2, 4, 3)).astype(np.uint8)
        a = rc.frameset(cams, opts, frames, prev_p, prev_v)
        for prev_frames in (None, frames):
            b = rc.frameset_removal(cams, opts, frames, prev_frames, prev_p, prev_v)
            assert np.array_equal(a["params"].view(np.uint64), b["params"].view(np.uint64))
            assert np.array_equal(a["valid"], b["valid"])
            for x, y in zip(a["out"], b["out"]):
                assert np.array_equal(x, y)


def test_method_is_the_same_on_both_sides_of_every_seam():
    rng = np.random.default_rng(24)
    cams = [rc.Camera(24, 20, 3, 8, 0, p) for p in range(4)]
    opts = rc.Options(n_blocks=5, band_width=4)
    for trial in range(10):
        now = [rng.integers(0, 256, (20, 24, 3)).astype(np.uint8) for _ in range(4)]
        prev = [np.where(rng.random((20, 24, 1)) < rng.uniform(0, 1), (f.astype(int) + 60) % 256, f).astype(np.uint8)
                for f in now]
        kept = np.stack([rc.kept_band_sums(f, p, c, opts) for f, p, c in zip(now, prev, cams)])
        full = np.stack([rc.band_stats(f, c, opts)[1] for f, c in zip(now, cams)])
        _, _, method = rc.estimate_removal(cams, opts, full, kept)
        for k in range(4):
            for s in (0, 1):
                fk, fs = rc.facing(cams, opts, k, s)
                assert np.array_equal(method[k, s], method[fk, fs])
        assert set(np.unique(method)) <= {rc.METHOD_REMOVAL, rc.METHOD_SMOOTHING}
