"""Pins of the oracle's cross-channel 3x3 maps (section 5's 3x3 linear maps
across the colour channels; readings R-x3-* in oracle/crossmap.py).
Independent checks: cross sums against pixel loops, the Cholesky factor
against numpy's, the fitted map transporting the own band's mean and
covariance onto the shared ones (checked with numpy matrix algebra), the
per-channel fit recovered for uncorrelated channels and on every fallback,
exact scaling of bands that are multiples of each other, the Q16 map and its
blend against exact rationals per pixel, and identity maps."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import crossmap as cm
from oracle import ringcorr as rc


def sums_of(pix):
    v = pix.astype(np.int64).reshape(-1, 3)
    s = np.array([[v.shape[0], int(v[:, c].sum()), int((v[:, c] * v[:, c]).sum())] for c in range(3)], np.int64)
    return s, cm.cross_sums(pix)


def test_cross_sums_against_loops():
    rng = np.random.default_rng(1)
    cam = rc.Camera(19, 13, 3, 8)
    opts = rc.Options(n_blocks=3, band_width=4)
    f = rng.integers(0, 256, (13, 19, 3)).astype(np.uint8)
    got = cm.band_cross(f, cam, opts)
    for j, (r0, r1) in enumerate(rc.block_bounds(13, 3)):
        for s, (c0, c1) in enumerate(rc.band_columns(19, 4)):
            ref = [0, 0, 0]
            for r in range(r0, r1):
                for c in range(c0, c1):
                    p = [int(v) for v in f[r, c]]
                    ref[0] += p[0] * p[1]
                    ref[1] += p[0] * p[2]
                    ref[2] += p[1] * p[2]
            assert got[s, j].tolist() == ref


@pytest.mark.parametrize("seed", range(5))
def test_cholesky_against_numpy(seed):
    rng = np.random.default_rng([2, seed])
    A = rng.normal(size=(3, 3)) * rng.uniform(1, 40)
    C = A @ A.T + np.eye(3) * 0.1
    L = np.array(cm.cholesky3(C.tolist()))
    assert np.allclose(L, np.linalg.cholesky(C), rtol=1e-12, atol=1e-12)
    assert cm.cholesky3([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]]) is None   # indefinite
    assert cm.cholesky3([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]) is None


def correlated_band(rng, n, mean, mix):
    z = rng.normal(size=(n, 3))
    return np.clip(np.rint(mean + z @ mix.T), 0, 255).astype(np.uint8).reshape(n, 1, 3)


@pytest.mark.parametrize("seed", range(6))
def test_map_transports_mean_and_covariance(seed):
    rng = np.random.default_rng([3, seed])
    own = correlated_band(rng, 3000, rng.uniform(60, 120, 3), rng.uniform(-1, 1, (3, 3)) * 4 + np.eye(3) * 12)
    fac = correlated_band(rng, 2500, rng.uniform(60, 160, 3), rng.uniform(-1, 1, (3, 3)) * 4 + np.eye(3) * 15)
    so, xo = sums_of(own)
    sf, xf = sums_of(fac)
    M, t = cm.fit_cross(so, xo, sf, xf, 1 / 8, 8.0)
    M, t = np.array(M), np.array(t)
    assert np.count_nonzero(M - np.diag(np.diag(M))) > 0          # the 3x3 fit, not the fallback
    mo, Co = np.array(cm.mean_cov(so, xo)[0]), np.array(cm.mean_cov(so, xo)[1])
    mf, Cf = np.array(cm.mean_cov(sf, xf)[0]), np.array(cm.mean_cov(sf, xf)[1])
    Ls = (np.linalg.cholesky(Co) + np.linalg.cholesky(Cf)) / 2
    assert np.allclose(M @ Co @ M.T, Ls @ Ls.T, rtol=1e-9, atol=1e-9)
    assert np.allclose(M @ mo + t, (mo + mf) / 2, rtol=1e-12, atol=1e-9)
    assert np.allclose(M @ np.linalg.cholesky(Co), Ls, rtol=1e-12, atol=1e-12)    # M L_own = L*
    # mean and covariance of the samples themselves, by numpy
    x = own.reshape(-1, 3).astype(np.float64)
    assert np.allclose(x.mean(0), mo) and np.allclose(np.cov(x.T, bias=True), Co, rtol=1e-9)


def test_uncorrelated_channels_give_the_per_channel_fit():
    # sums whose cross terms are exactly n mu_a mu_b: zero covariance
    n = 64
    so = np.array([[n, 64 * 50, 64 * 2600], [n, 64 * 80, 64 * 6500], [n, 64 * 100, 64 * 10100]], np.int64)
    sf = np.array([[n, 64 * 70, 64 * 5000], [n, 64 * 60, 64 * 3700], [n, 64 * 90, 64 * 8200]], np.int64)
    xo = np.array([64 * 50 * 80, 64 * 50 * 100, 64 * 80 * 100], np.int64)
    xf = np.array([64 * 70 * 60, 64 * 70 * 90, 64 * 60 * 90], np.int64)
    M, t = cm.fit_cross(so, xo, sf, xf, 1 / 8, 8.0)
    for c in range(3):
        a, b = rc.fit_side(tuple(int(v) for v in so[c]), tuple(int(v) for v in sf[c]), 1 / 8, 8.0)
        assert abs(M[c][c] - a) <= 1e-15 * a and abs(t[c] - b) <= 1e-12 * max(1.0, abs(b))
        for d in range(3):
            if d != c:
                assert M[c][d] == 0.0


def test_multiples_scale_exactly():
    rng = np.random.default_rng(4)
    own = correlated_band(rng, 1000, np.array([40.0, 50.0, 60.0]), np.array([[6, 2, 0], [1, 7, 2], [0, 2, 5.0]]))
    fac = (own.astype(np.int64) * 2)
    so, xo = sums_of(own)
    sf, xf = sums_of(fac)
    M, t = cm.fit_cross(so, xo, sf, xf, 1 / 8, 8.0)
    assert np.allclose(np.array(M), 1.5 * np.eye(3), rtol=0, atol=1e-14)
    assert np.allclose(t, 0.0, atol=1e-11)


def test_fallbacks_take_the_per_channel_fit():
    rng = np.random.default_rng(5)
    flat = np.full((200, 1, 3), 90, np.uint8)                       # zero covariance: no Cholesky factor
    other = correlated_band(rng, 300, np.array([70.0, 90.0, 110.0]), np.eye(3) * 9)
    for own, fac, amax in ((flat, other, 8.0), (other, flat, 8.0), (other, other.astype(np.int64) * 4, 2.0)):
        so, xo = sums_of(own)
        sf, xf = sums_of(fac)
        M, t = cm.fit_cross(so, xo, sf, xf, 1 / 8, amax)
        for c in range(3):
            a, b = rc.fit_side(tuple(int(v) for v in so[c]), tuple(int(v) for v in sf[c]), 1 / 8, amax)
            assert (M[c][c], t[c]) == (a, b)
            assert all(M[c][d] == 0.0 for d in range(3) if d != c)
    empty = np.zeros((3, 3), np.int64)
    assert cm.fit_cross(empty, np.zeros(3, np.int64), *sums_of(other), 1 / 8, 8.0) is None


def test_q16_map_and_blend_against_rationals():
    rng = np.random.default_rng(6)
    cam = rc.Camera(9, 4, 3, 8)
    opts = rc.Options(n_blocks=2, band_width=2)
    frame = rng.integers(0, 256, (4, 9, 3)).astype(np.uint8)
    params = np.zeros((1, 2, 2, 12))
    params[..., :9] = rng.uniform(-0.6, 1.6, (1, 2, 2, 9))
    params[..., 9:] = rng.uniform(-40, 40, (1, 2, 2, 3))
    q = cm.build_cross([cam], opts, params)
    out = cm.apply_camera_cross(frame, cam, opts, q[0])
    w, side = rc.column_weights(9)
    for r in range(4):
        j = rc.block_of_row(r, 4, 2)
        for col in range(9):
            x = [int(v) for v in frame[r, col]]
            if side[col] < 0:
                assert out[r, col].tolist() == x
                continue
            qq = q[0, side[col], j]
            for c in range(3):
                assert qq[3 * c] == round(Fraction(params[0, side[col], j, 3 * c]) * 65536)
                v = Fraction(sum(int(qq[3 * c + d]) * x[d] for d in range(3)) + int(qq[9 + c]) + 32768, 65536)
                f = min(max(v.numerator // v.denominator, 0), 255)
                y = Fraction((256 - int(w[col])) * x[c] + int(w[col]) * f + 128, 256)
                assert out[r, col, c] == y.numerator // y.denominator


def test_identity_maps_and_frameset_shapes():
    rng = np.random.default_rng(7)
    cams = [rc.Camera(24, 16, 3, 8, 0, p) for p in range(3)]
    opts = rc.Options(n_blocks=2, band_width=4)
    frames = [rng.integers(0, 256, (16, 24, 3)).astype(np.uint8) for _ in cams]
    q = cm.build_cross(cams, opts, np.tile(np.array(cm.IDENTITY), (3, 2, 2, 1)))
    for k in range(3):
        assert np.array_equal(cm.apply_camera_cross(frames[k], cams[k], opts, q[k]), frames[k])
    r = cm.frameset_cross(cams, opts, frames)
    assert r["params"].shape == (3, 2, 2, 12) and r["valid"].all()
    open_opts = rc.Options(n_blocks=2, band_width=4, closed_ring=False)
    r2 = cm.frameset_cross(cams, open_opts, frames)
    assert r2["params"][0, 0].tolist() == [cm.IDENTITY] * 2       # outer side faces nothing
    with pytest.raises(ValueError):
        cm.estimate_cross([rc.Camera(8, 8, 1, 8)], opts, np.zeros((1, 2, 2, 3, 3)), np.zeros((1, 2, 2, 3)))


def test_smoothing_blends_every_parameter():
    rng = np.random.default_rng(8)
    cams = [rc.Camera(24, 16, 3, 8, 0, p) for p in range(2)]
    opts = rc.Options(n_blocks=2, band_width=4, smoothing=True)
    f0 = [rng.integers(0, 256, (16, 24, 3)).astype(np.uint8) for _ in cams]
    f1 = [rng.integers(0, 256, (16, 24, 3)).astype(np.uint8) for _ in cams]
    r0 = cm.frameset_cross(cams, opts, f0)
    r1 = cm.frameset_cross(cams, opts, f1, r0["params"], r0["valid"])
    fresh = cm.frameset_cross(cams, rc.Options(n_blocks=2, band_width=4), f1)
    for idx in np.ndindex(r1["params"].shape):
        assert r1["params"][idx] == rc.ema(float(r0["params"][idx]), float(fresh["params"][idx]), 0.05)
