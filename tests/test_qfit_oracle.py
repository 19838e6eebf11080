"""Pins of the oracle's quantile least-squares fit (the affine map that makes
the two band distributions agree, section 3.1, fitted on quantiles instead of
the two moments).  Independent checks: quantiles against sorted samples with
exact rationals, the fitted line against numpy's least-squares solver on the
same quantile pairs, bands that are exact affine images of each other (the
moment fit's map, in closed form), identical and constant bands, 12- and
16-bit bin centres, and the estimate's dispatch (the removal path refuses the
quantile fit)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ringcorr as rc

M = rc.QFIT_LEVELS


def hist_of(values):
    return np.bincount(np.asarray(values, np.int64), minlength=rc.NBINS).astype(np.int64)


def sorted_quantiles(values):
    """Level-i quantile as the ceil(p_i n)-th smallest sample, p_i = (2i+1)/(2M)."""
    v = sorted(int(x) for x in values)
    n = len(v)
    return [v[math.ceil(Fraction(2 * i + 1, 2 * M) * n) - 1] for i in range(M)]


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 7), (2, 64), (3, 65), (4, 2144), (5, 10000)])
def test_quantile_bins_against_sorted_samples(seed, n):
    rng = np.random.default_rng([77, seed])
    vals = np.clip(rng.normal(rng.uniform(40, 200), rng.uniform(1, 40), n), 0, 255).astype(np.int64)
    assert rc.quantile_bins(hist_of(vals)) == sorted_quantiles(vals)


@pytest.mark.parametrize("seed", range(6))
def test_fit_matches_numpy_least_squares(seed):
    rng = np.random.default_rng([78, seed])
    own = np.clip(rng.normal(90, 20, 3000), 0, 255).astype(np.int64)
    fac = np.clip(rng.gamma(4.0, 12.0, 2500) + 30, 0, 255).astype(np.int64)
    a, b = rc.fit_side_quantile(hist_of(own), hist_of(fac), 8, 1 / 8, 8.0)
    x = np.array(sorted_quantiles(own), np.float64)
    y = (x + np.array(sorted_quantiles(fac), np.float64)) / 2
    A = np.stack([x, np.ones_like(x)], axis=1)
    (ref_a, ref_b), *_ = np.linalg.lstsq(A, y, rcond=None)
    assert abs(a - ref_a) <= 1e-12 * abs(ref_a)
    assert abs(b - ref_b) <= 1e-9 * max(1.0, abs(ref_b))


def test_affine_images_give_the_moment_fit_in_closed_form():
    rng = np.random.default_rng(5)
    own = rng.integers(10, 100, 1500)
    # facing band = 2 x: both fits give a = 3/2, b = 0 exactly
    a, b = rc.fit_side_quantile(hist_of(own), hist_of(2 * own), 8, 1 / 8, 8.0)
    assert (a, b) == (1.5, 0.0)
    am, bm = rc.fit_side(tuple(int(v) for v in (own.size, own.sum(), (own * own).sum())),
                         tuple(int(v) for v in (own.size, (2 * own).sum(), (4 * own * own).sum())), 1 / 8, 8.0)
    assert abs(am - 1.5) < 1e-15 and abs(bm) < 1e-12
    # facing band = x + 10: a = 1, b = 5 exactly; the facing side gets a = 1, b = -5
    assert rc.fit_side_quantile(hist_of(own), hist_of(own + 10), 8, 1 / 8, 8.0) == (1.0, 5.0)
    assert rc.fit_side_quantile(hist_of(own + 10), hist_of(own), 8, 1 / 8, 8.0) == (1.0, -5.0)


def test_identical_and_empty_and_constant_bands():
    rng = np.random.default_rng(6)
    h = hist_of(rng.integers(0, 256, 999))
    assert rc.fit_side_quantile(h, h, 8, 1 / 8, 8.0) == (1.0, 0.0)
    assert rc.fit_side_quantile(h, np.zeros(256, np.int64), 8, 1 / 8, 8.0) is None
    assert rc.fit_side_quantile(np.zeros(256, np.int64), h, 8, 1 / 8, 8.0) is None
    const = hist_of([77] * 50)
    a, b = rc.fit_side_quantile(const, h, 8, 1 / 8, 8.0)
    qf = rc.quantile_bins(h)
    assert a == 1.0
    assert b == float(Fraction(77 * M + sum(qf), 2 * M) - 77)


def test_clamp_binds_before_b():
    own = hist_of(list(range(100, 110)) * 10)          # spread 9
    fac = hist_of(list(range(0, 250, 25)) * 10)        # spread 225
    a, b = rc.fit_side_quantile(own, fac, 8, 1 / 8, 2.0)
    assert a == 2.0
    qo, qf = rc.quantile_bins(own), rc.quantile_bins(fac)
    mu_o = Fraction(sum(qo), M)
    mu_s = Fraction(sum(qo) + sum(qf), 2 * M)
    assert b == float(mu_s) - 2.0 * float(mu_o)


@pytest.mark.parametrize("bd", [10, 12, 16])
def test_wide_samples_use_bin_centres(bd):
    sh = bd - 8
    rng = np.random.default_rng([79, bd])
    bins = rng.integers(20, 200, 800)
    own = hist_of(bins)
    fac = hist_of(bins + 3)                               # three bins up: 3 * 2^sh sample units
    a, b = rc.fit_side_quantile(own, fac, bd, 1 / 8, 8.0)
    assert a == 1.0 and b == 1.5 * (1 << sh)
    assert rc.bin_centre2(0, bd) == (1 << sh) - 1 and rc.bin_centre2(255, bd) == 2 * (255 << sh) + (1 << sh) - 1
    assert rc.bin_centre2(17, 8) == 34


def test_estimate_dispatches_on_the_fit_option():
    rng = np.random.default_rng(8)
    cams = [rc.Camera(40, 24, 3, 8, 0, p) for p in range(3)]
    frames = [rng.integers(0, 256, (24, 40, 3)).astype(np.uint8) for _ in cams]
    opts = rc.Options(n_blocks=2, band_width=6, fit="quantile")
    r = rc.frameset(cams, opts, frames)
    for k in range(3):
        for s in (0, 1):
            fk, fs = rc.facing(cams, opts, k, s)
            for j in range(2):
                for c in range(3):
                    ref = rc.fit_side_quantile(r["band_hist"][k, s, j, c], r["band_hist"][fk, fs, j, c], 8,
                                               opts.a_min, opts.a_max)
                    assert tuple(r["params"][k, s, j, c]) == ref
    with pytest.raises(ValueError):
        rc.estimate(cams, opts, r["band_sums"])             # no histograms
    with pytest.raises(ValueError):
        rc.estimate_removal(cams, opts, r["band_sums"], r["band_sums"])
    with pytest.raises(ValueError):
        rc.estimate(cams, rc.Options(fit="median"), r["band_sums"])
