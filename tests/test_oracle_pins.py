"""Pins of the CPU oracle against the paper and against mathematics.

Every check here reaches the oracle's result by another route: brute-force
loops over pixels, exact rational arithmetic (fractions.Fraction), closed
forms, invariants, and hand-worked values from tests/golden/.  A dropped
term, a wrong sign, a swapped side or an off-by-one block fails one of them.
No GPU and no compiled code is involved.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ringcorr as rc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def rhu(q: Fraction) -> int:
    """round half up of an exact rational."""
    return math.floor(q + Fraction(1, 2))


# ---------------------------------------------------------------- regions

def test_block_partition_bruteforce():
    for H in range(1, 41):
        for NB in range(1, 21):
            b = rc.block_bounds(H, NB)
            assert b[0][0] == 0 and b[-1][1] == H
            for j in range(NB - 1):
                assert b[j][1] == b[j + 1][0]
            sizes = [r1 - r0 for r0, r1 in b]
            assert max(sizes) - min(sizes) <= 1          # "blocks of identical size" up to one row
            for r in range(H):
                owners = [j for j, (r0, r1) in enumerate(b) if r0 <= r < r1]
                assert owners == [rc.block_of_row(r, H, NB)]


def test_band_columns():
    for W in range(1, 200):
        for B in (1, 2, 7, 32, 500):
            (l0, l1), (r0, r1) = rc.band_columns(W, B)
            bb = min(B, W // 2)
            assert (l0, l1, r0, r1) == (0, bb, W - bb, W)
            assert l1 <= r0                                   # bands never overlap


def test_facing_ring_and_chain():
    rng = np.random.default_rng(3)
    for m in (1, 2, 3, 14):
        pos = rng.permutation(m)
        cams = [rc.Camera(8, 8, ring=5, pos=int(p)) for p in pos]
        cams += [rc.Camera(8, 8, ring=1, pos=0)]            # another ring, never faced
        by_pos = {int(p): i for i, p in enumerate(pos)}
        closed = rc.Options(closed_ring=True)
        openc = rc.Options(closed_ring=False)
        for k in range(m):
            p = int(pos[k])
            assert rc.facing(cams, closed, k, rc.RIGHT) == (by_pos[(p + 1) % m], rc.LEFT)
            assert rc.facing(cams, closed, k, rc.LEFT) == (by_pos[(p - 1) % m], rc.RIGHT)
            for s in (rc.LEFT, rc.RIGHT):
                f = rc.facing(cams, closed, k, s)
                assert rc.facing(cams, closed, *f) == (k, s)   # facing is an involution
            assert (rc.facing(cams, openc, k, rc.RIGHT) is None) == (p == m - 1)
            assert (rc.facing(cams, openc, k, rc.LEFT) is None) == (p == 0)
        assert rc.facing(cams, closed, m, rc.LEFT) == (m, rc.RIGHT)   # ring of one faces itself


# ---------------------------------------------------------------- statistics

def brute_stats(frame, bit_depth, rows, cols):
    C = frame.shape[2]
    hist = [[0] * 256 for _ in range(3)]
    sums = [[0, 0, 0] for _ in range(3)]
    for r in rows:
        for col in cols:
            for c in range(C):
                v = int(frame[r, col, c])
                b = v if bit_depth == 8 else min(v // (1 << (bit_depth - 8)), 255)
                hist[c][b] += 1
                sums[c][0] += 1
                sums[c][1] += v
                sums[c][2] += v * v
    return np.array(hist), np.array(sums)


@pytest.mark.parametrize("bit_depth,C", [(8, 3), (8, 1), (10, 1), (12, 1), (16, 1)])
def test_region_stats_bruteforce(bit_depth, C):
    rng = np.random.default_rng(bit_depth * 10 + C)
    for (H, W) in [(1, 1), (2, 3), (5, 4), (13, 17), (17, 13)]:
        dt = np.uint8 if bit_depth == 8 else np.uint16
        f = rng.integers(0, 1 << bit_depth, (H, W, C)).astype(dt)
        h, s = rc.region_stats(f, bit_depth)
        bh, bs = brute_stats(f, bit_depth, range(H), range(W))
        assert np.array_equal(h, bh) and np.array_equal(s, bs)


def test_band_stats_bruteforce_per_pixel_classification():
    """Classify every pixel by the closed-form block index and band test, then count."""
    rng = np.random.default_rng(11)
    for (H, W, NB, B) in [(13, 17, 4, 3), (9, 5, 16, 32), (30, 40, 7, 6), (4, 1, 2, 2)]:
        f = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
        cam = rc.Camera(W, H)
        opts = rc.Options(n_blocks=NB, band_width=B)
        hist, sums = rc.band_stats(f, cam, opts)
        bb = min(B, W // 2)
        ref_h = np.zeros_like(hist)
        ref_s = np.zeros_like(sums)
        for r in range(H):
            j = ((r + 1) * NB - 1) // H
            for col in range(W):
                sides = []
                if col < bb:
                    sides.append(0)
                if col >= W - bb:
                    sides.append(1)
                for s in sides:
                    for c in range(3):
                        v = int(f[r, col, c])
                        ref_h[s, j, c, v] += 1
                        ref_s[s, j, c] += (1, v, v * v)
        assert np.array_equal(hist, ref_h) and np.array_equal(sums, ref_s)


def test_hist_moment_identities_u8():
    rng = np.random.default_rng(5)
    f = rng.integers(0, 256, (37, 53, 3)).astype(np.uint8)
    h, s = rc.region_stats(f, 8)
    v = np.arange(256)
    for c in range(3):
        assert h[c].sum() == s[c, 0] == 37 * 53
        assert (v * h[c]).sum() == s[c, 1]
        assert (v * v * h[c]).sum() == s[c, 2]


def test_whole_is_union_of_disjoint_tiling():
    rng = np.random.default_rng(6)
    f = rng.integers(0, 1 << 12, (31, 29, 1)).astype(np.uint16)
    h, s = rc.whole_stats(f, rc.Camera(29, 31, 1, 12))
    ys = [0, 7, 8, 20, 31]
    xs = [0, 1, 15, 29]
    th, ts = np.zeros_like(h), np.zeros_like(s)
    for a, b in zip(ys[:-1], ys[1:]):
        for c0, c1 in zip(xs[:-1], xs[1:]):
            hh, ss = rc.region_stats(f[a:b, c0:c1], 12)
            th += hh
            ts += ss
    assert np.array_equal(h, th) and np.array_equal(s, ts)


# ---------------------------------------------------------------- estimate

def test_worked_fit_golden():
    g = golden("affine_fit_worked.json")
    own, fac = tuple(g["own_sums"]), tuple(g["facing_sums"])
    a, b = rc.fit_side(own, fac, 0.125, 8.0)
    a2, b2 = rc.fit_side(fac, own, 0.125, 8.0)
    assert abs(a - g["a_own"]) < 1e-14 and abs(b - g["b_own"]) < 1e-12
    assert abs(a2 - g["a_facing"]) < 1e-14 and abs(b2 - g["b_facing"]) < 1e-12
    assert (rc.q16(a), rc.q16(b)) == tuple(g["q16_own"])
    assert (rc.q16(a2), rc.q16(b2)) == tuple(g["q16_facing"])
    lut_p, lut_q = rc.lut_u8(a, b), rc.lut_u8(a2, b2)
    for x, v in g["lut_own"].items():
        assert lut_p[int(x)] == v
    for x, v in g["lut_facing"].items():
        assert lut_q[int(x)] == v


def mirrored_pair_rig(H=64, W=48, NB=4, seed=0):
    """Two identical cameras, each mirror-symmetric left/right: every facing band
    pair holds the same multiset of samples."""
    rng = np.random.default_rng(seed)
    half = rng.integers(20, 230, (H, W // 2, 3)).astype(np.uint8)
    f = np.concatenate([half, half[:, ::-1]], axis=1)
    cams = [rc.Camera(W, H, pos=0), rc.Camera(W, H, pos=1)]
    return cams, rc.Options(n_blocks=NB, band_width=8), [f, f.copy()]


def test_identity_on_equal_bands():
    cams, opts, frames = mirrored_pair_rig()
    r = rc.frameset(cams, opts, frames)
    assert np.all(r["params"][..., 0] == 1.0) and np.all(r["params"][..., 1] == 0.0)
    assert np.all(r["lut8"] == np.arange(256, dtype=np.uint8))
    for f, o in zip(frames, r["out"]):
        assert np.array_equal(f, o)


def test_gain_recovery_integer_gains_exact():
    """Facing bands s and 2 s: a_P = 1.5, a_Q = 0.75, b = 0, corrected bands equal."""
    rng = np.random.default_rng(1)
    s = rng.integers(16, 97, (40, 8, 3)).astype(np.int64)
    P, Q = s.astype(np.uint8), (2 * s).astype(np.uint8)
    hp, sp = rc.region_stats(P, 8)
    hq, sq = rc.region_stats(Q, 8)
    for c in range(3):
        aP, bP = rc.fit_side(tuple(sp[c]), tuple(sq[c]), 0.125, 8.0)
        aQ, bQ = rc.fit_side(tuple(sq[c]), tuple(sp[c]), 0.125, 8.0)
        assert abs(aP - 1.5) <= 4e-16 * 1.5 and abs(aQ - 0.75) <= 4e-16
        assert abs(bP) < 1e-12 and abs(bQ) < 1e-12
        lp, lq = rc.lut_u8(aP, bP), rc.lut_u8(aQ, bQ)
        cp = lp[P[:, :, c]]
        cq = lq[Q[:, :, c]]
        assert np.array_equal(cp, cq)
        assert np.array_equal(cp.astype(np.int64), (3 * s[:, :, c] + 1) // 2)   # round_half_up(1.5 s)


def test_gain_recovery_requantised():
    """Bands of one scene under gains gP, gQ: a_P / a_Q = gQ / gP up to uint8 re-quantisation."""
    rng = np.random.default_rng(2)
    for trial in range(20):
        s = rng.uniform(16.0, 96.0, (200, 16, 3))         # continuous scene, no clipping
        gP, gQ = rng.uniform(0.5, 2.0, 2)
        P = np.rint(gP * s).astype(np.uint8)
        Q = np.rint(gQ * s).astype(np.uint8)
        _, sp = rc.region_stats(P, 8)
        _, sq = rc.region_stats(Q, 8)
        for c in range(3):
            aP, bP = rc.fit_side(tuple(sp[c]), tuple(sq[c]), 0.125, 8.0)
            aQ, bQ = rc.fit_side(tuple(sq[c]), tuple(sp[c]), 0.125, 8.0)
            # rounding to integers perturbs each sigma by ~1/(24 g^2 sigma^2) relative
            assert abs(aP / aQ - gQ / gP) < 1e-3 * (gQ / gP)
            assert abs(aP - (gP + gQ) / (2 * gP)) < 1e-3 * aP
            assert abs(bP) < 0.6 and abs(bQ) < 0.6


def test_fit_invariants_and_bruteforce_moments():
    rng = np.random.default_rng(4)
    for trial in range(200):
        n1, n2 = rng.integers(1, 60, 2)
        P = rng.integers(0, 256, n1)
        Q = rng.integers(0, 256, n2)
        own = (len(P), int(P.sum()), int((P * P).sum()))
        fac = (len(Q), int(Q.sum()), int((Q * Q).sum()))
        a, b = rc.fit_side(own, fac, 1e-9, 1e9)
        a2, b2 = rc.fit_side(fac, own, 1e-9, 1e9)
        mu_s = (P.mean() + Q.mean()) / 2
        sd_s = (P.std() + Q.std()) / 2
        if P.std() > 0:
            assert abs(a * P.std() - sd_s) <= 1e-12 * max(sd_s, 1)
            cp = a * P.astype(float) + b              # the unrounded map applied to the band
            assert abs(cp.mean() - mu_s) < 1e-9 and abs(cp.std() - sd_s) < 1e-9
        else:
            assert a == 1.0
        assert abs((a * P.mean() + b) - mu_s) < 1e-9
        if P.std() > 0 and Q.std() > 0:
            assert abs(a * P.std() - a2 * Q.std()) < 1e-9
            assert abs((a * P.mean() + b) - (a2 * Q.mean() + b2)) < 1e-9


def test_fit_clamp_and_empty():
    assert rc.fit_side((0, 0, 0), (4, 100, 3000), 0.125, 8) is None
    assert rc.fit_side((4, 100, 3000), (0, 0, 0), 0.125, 8) is None
    # flat own band: a = 1, b moves the mean
    a, b = rc.fit_side((4, 40, 400), (4, 100, 3000), 0.125, 8)
    assert a == 1.0 and b == (10 + 25) / 2 - 10
    # huge contrast ratio is clamped, and b is computed after the clamp
    a, b = rc.fit_side((2, 201, 20201), (2, 200, 25000), 0.125, 8)   # sigma 0.5 vs 50
    assert a == 8.0 and abs(b - ((100.5 + 100.0) / 2 - 8.0 * 100.5)) < 1e-12


def test_ema_golden_and_closed_form():
    g = golden("ema_worked.json")
    alpha = g["alpha"]
    seq = [g["first"]]
    for _ in range(len(g["sequence"]) - 1):
        seq.append(rc.ema(seq[-1], g["new"], alpha))
    assert np.allclose(seq, g["sequence"], rtol=0, atol=1e-14)
    p, p0, pn = 0.7, 0.7, 1.9
    for t in range(1, 200):
        p = rc.ema(p, pn, 0.05)
        assert abs(p - (pn + (1 - 0.05) ** t * (p0 - pn))) < 1e-12
    q = 1.2345
    for _ in range(50):
        assert abs(rc.ema(q, q, 0.05) - q) <= 2 * np.spacing(q)   # constant input stays constant


def test_estimate_state_machine():
    """First estimate is taken as is, then smoothed; empty bands keep the previous map."""
    cams = [rc.Camera(16, 4, pos=0), rc.Camera(16, 4, pos=1)]
    opts = rc.Options(n_blocks=1, band_width=2, smoothing=True)
    K = 2
    sums0 = np.zeros((K, 2, 1, 3, 3), np.int64)
    sums0[..., :] = (4, 100, 3000)
    sums0[1, 0, 0, :] = (4, 240, 16400)                     # camera 1 left band faces camera 0 right
    p, v = rc.estimate(cams, opts, sums0)
    assert p[0, 1, 0, 0, 0] == pytest.approx(1.5, abs=1e-14) and v.all()
    p1, v1 = rc.estimate(cams, opts, sums0, p, v)
    assert p1[0, 1, 0, 0, 0] == pytest.approx(1.5, abs=1e-14)
    sums_e = sums0.copy()
    sums_e[0, 1] = 0                                        # camera 0 right band empty
    p2, v2 = rc.estimate(cams, opts, sums_e, p1, v1)
    assert np.array_equal(p2[0, 1], p1[0, 1]) and np.array_equal(p2[1, 0], p1[1, 0])
    p3, v3 = rc.estimate(cams, opts, sums_e)                 # no history: identity, not valid
    assert np.all(p3[0, 1, ..., 0] == 1.0) and np.all(p3[0, 1, ..., 1] == 0.0) and not v3[0, 1].any()
    po, vo = rc.estimate(cams, rc.Options(n_blocks=1, band_width=2, closed_ring=False), sums0)
    assert np.all(po[0, 0, ..., 0] == 1.0) and np.all(po[0, 0, ..., 1] == 0.0) and vo[0, 0].all()
    assert np.all(po[1, 1, ..., 0] == 1.0) and vo[1, 1].all()


# ---------------------------------------------------------------- LUT, weights, blend

def test_q16_and_lut_against_rationals():
    rng = np.random.default_rng(7)
    cases = [(1.0, 0.0), (1.5, 5.0), (0.75, -2.5), (0.125, 300.0), (8.0, -2000.0), (1.0, 0.5 / 65536)]
    cases += [(float(a), float(b)) for a, b in zip(rng.uniform(0.125, 8, 300), rng.uniform(-300, 300, 300))]
    for a, b in cases:
        A = round(Fraction(a) * 65536)          # Fraction rounds half to even
        Bq = round(Fraction(b) * 65536)
        assert (rc.q16(a), rc.q16(b)) == (A, Bq)
        lut = rc.lut_u8(a, b)
        for x in range(256):
            ref = min(max(rhu(Fraction(A * x + Bq, 65536)), 0), 255)
            assert lut[x] == ref
        if a > 0:
            assert np.all(np.diff(lut.astype(int)) >= 0)      # monotone map


def test_lut_identity():
    assert np.array_equal(rc.lut_u8(1.0, 0.0), np.arange(256))


def test_blend_exhaustive():
    x = np.arange(256)[:, None, None]
    w = np.arange(257)[None, :, None]
    L = np.arange(256)[None, None, :]
    y = rc.blend(x, L, w)
    num = (256 - w) * x + w * L                       # exact numerator over 256
    ref = np.floor_divide(2 * num + 256, 512)         # round half up of num / 256
    assert np.array_equal(y, ref)
    assert np.all((y >= np.minimum(x, L)) & (y <= np.maximum(x, L)))
    assert np.array_equal(y[:, 0, :], np.broadcast_to(x[:, 0, :], (256, 256)))
    assert np.array_equal(y[:, 256, :], np.broadcast_to(L[:, 0, :], (256, 256)))
    rng = np.random.default_rng(8)
    for _ in range(3000):
        xi, wi, li = int(rng.integers(256)), int(rng.integers(257)), int(rng.integers(256))
        exact = Fraction(256 - wi, 256) * xi + Fraction(wi, 256) * li
        assert rc.blend(xi, li, wi) == rhu(exact)


def test_weights_golden():
    g = golden("weights_worked.json")
    for W, ws in g["cases"].items():
        w, side = rc.column_weights(int(W))
        assert list(w) == ws
    for W, s in g["side"].items():
        assert list(rc.column_weights(int(W))[1]) == s


def test_weights_against_rationals():
    for W in list(range(1, 130)) + [640, 1920, 4096]:
        w, side = rc.column_weights(W)
        h = W // 2
        for col in range(W):
            if col < h:
                ref, sref = rhu(Fraction(256 * (h - col), h)), 0
            elif col >= W - h:
                ref, sref = rhu(Fraction(256 * (h - (W - 1 - col)), h)), 1
            else:
                ref, sref = 0, -1
            assert (w[col], side[col]) == (ref, sref)
        assert np.array_equal(w, w[::-1])                    # the two halves mirror each other
        if W >= 2:
            assert w[0] == 256 and w[-1] == 256


def test_weights_table_golden():
    """The per-camera table the tables step writes: one row per camera of
    W_max entries, each camera's own weights then zeros (hand-worked)."""
    g = golden("weights_table_worked.json")
    cams = [rc.Camera(w, 4, pos=i) for i, w in enumerate(g["widths"])]
    t = rc.weights_table(cams)
    assert t.dtype == np.uint16 and t.shape == (3, 8)
    assert t.tolist() == g["table"]


def test_weights_table_rows_against_rationals():
    """Rows of uneven rigs: row k, columns < W_k, is round_half_up(256 d / h)
    by exact rationals (d counted from the centre), every later entry is 0;
    row order follows the camera list, not ring position."""
    widths = [17, 1, 64, 2, 33, 7]
    cams = [rc.Camera(w, 3, ring=i % 2, pos=i // 2) for i, w in enumerate(widths)]
    t = rc.weights_table(cams)
    assert t.shape == (len(widths), max(widths))
    for k, W in enumerate(widths):
        h = W // 2
        for col in range(max(widths)):
            if col >= W:
                ref = 0
            elif col < h:
                ref = rhu(Fraction(256 * (h - col), h))
            elif col >= W - h:
                ref = rhu(Fraction(256 * (col - (W - h) + 1), h))
            else:
                ref = 0
            assert int(t[k, col]) == ref, (k, col)


@pytest.mark.parametrize("bit_depth", [8, 12])
def test_apply_bruteforce(bit_depth):
    """Per-pixel loop: block by closed form, weight by rationals, map by rationals."""
    rng = np.random.default_rng(9 + bit_depth)
    for (H, W, NB) in [(7, 9, 3), (5, 2, 8), (6, 1, 2), (11, 16, 4)]:
        C = 3 if bit_depth == 8 else 1
        cam = rc.Camera(W, H, C, bit_depth)
        opts = rc.Options(n_blocks=NB)
        maxv = (1 << bit_depth) - 1
        f = rng.integers(0, maxv + 1, (H, W, C)).astype(np.uint8 if bit_depth == 8 else np.uint16)
        params = np.zeros((1, 2, NB, 3, 2))
        params[..., 0] = rng.uniform(0.5, 2.0, (1, 2, NB, 3))
        params[..., 1] = rng.uniform(-20, 20, (1, 2, NB, 3)) * (1 if bit_depth == 8 else 16)
        lut8, qq = rc.build_luts([cam], opts, params)
        out = rc.apply_camera(f, cam, opts, lut8[0], qq[0])
        h = W // 2
        for r in range(H):
            j = ((r + 1) * NB - 1) // H
            for col in range(W):
                if col < h:
                    s, w = 0, rhu(Fraction(256 * (h - col), h))
                elif col >= W - h:
                    s, w = 1, rhu(Fraction(256 * (h - (W - 1 - col)), h))
                else:
                    s, w = 0, 0
                for c in range(C):
                    x = int(f[r, col, c])
                    a, b = params[0, s, j, c]
                    A, Bq = round(Fraction(a) * 65536), round(Fraction(b) * 65536)
                    fx = min(max(rhu(Fraction(A * x + Bq, 65536)), 0), maxv)
                    y = rhu(Fraction(256 - w, 256) * x + Fraction(w, 256) * fx)
                    assert out[r, col, c] == y, (H, W, NB, r, col, c)


# ---------------------------------------------------------------- seam cost

def test_seam_cost_golden():
    g = golden("seam_cost_worked.json")
    n, f, amp = g["size"], g["factor"], g["checker_amplitude"]
    chk = np.fromfunction(lambda r, c: ((r + c) % 2) * 2 - 1, (n, n)) * amp   # zero mean per 8x8 box

    def img(vals):
        a = np.zeros((n, n, 3))
        for i, v in enumerate(vals):
            a[:, i * f:(i + 1) * f, :] = v
        return a + chk[:, :, None]
    cost = rc.seam_cost(img(g["left_box_values"]), img(g["right_box_values"]), f)
    assert abs(cost - g["cost"]) < 1e-12


def test_seam_cost_closed_forms():
    H, W = 64, 48
    ramp = np.arange(2 * W, dtype=np.float64)[None, :, None] * np.array([1.0, 2.0, -0.5])
    ramp = np.broadcast_to(ramp, (H, 2 * W, 3)) + 40
    assert abs(rc.seam_cost(ramp[:, :W], ramp[:, W:], 1)) < 1e-12
    assert abs(rc.seam_cost(ramp[:, :W], ramp[:, W:], 8)) < 1e-12       # box means of a ramp are a ramp
    for u, v in [(10, 200), (100, 100), (255, 0)]:
        L = np.full((H, W, 3), float(u))
        R = np.full((H, W, 3), float(v))
        assert abs(rc.seam_cost(L, R, 8) - math.sqrt(3) * abs(u - v)) < 1e-9
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 255, (H, 2 * W, 3))
    assert rc.interior_cost(img, 8) == rc.seam_cost(img[:, :W], img[:, W:], 8)
