"""Oracle for the exposure / white-balance correction of a ring of cameras.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain, slow and exact.

The method is the one of section 3.1 of the paper ("White balance and exposure
correction"):

* narrow bands on both sides of every seam are assumed to share one colour
  spectrum (the local constancy prior);
* a shared spectrum is estimated per seam by averaging the two facing bands;
* each camera side gets one affine map f_c(x) = a_c x + b_c per colour
  channel that sends its band onto the shared spectrum; a map depends only on
  the two adjacent streams;
* the map is blended convexly from the identity at the image centre to f_c at
  the border, over half of each image;
* the stream is split vertically into blocks of equal size, one map per block;
* optional exponential smoothing E = (1 - alpha) E_prev + alpha E_new with
  alpha = 0.05 (the blending equation of section 3.1).

Where the paper is silent the readings are fixed here (and listed with their
reasons in the design notes of the repository):

R-ring    camera at ring position p meets position p+1 (closed ring by
          default, the last meeting the first; open chain optional, where the
          two outer sides get the identity map).
R-block   block j covers rows [floor(j H / NB), floor((j+1) H / NB)).
R-band    band width B' = min(B, floor(W / 2)); left band = columns [0, B'),
          right band = columns [W - B', W).
R-bins    uint8 sample v -> bin v; uint16 sample v of bit depth d ->
          bin min(v >> (d - 8), 255).
R-mid     shared spectrum = the "midway" distribution: mean of the two means
          and mean of the two standard deviations.
R-fit     a = sigma* / sigma_own (a = 1 when the own variance is 0), clamped to
          [a_min, a_max]; b = mu* - a mu_own, computed after the clamp.  No
          estimate when either band is empty: keep the previous map (identity
          if there is none).
R-ema     smoothing blends (a, b) pointwise, as two products and one sum;
          the first estimate is taken as is.
R-q16     A = round_half_even(a * 65536), Bq = round_half_even(b * 65536);
          f(x) = clamp((A x + Bq + 32768) >> 16) with >> a floor shift.
R-weight  h = floor(W / 2); left column col < h has Q8 weight
          round_half_up(256 (h - col) / h); right column col >= W - h has
          round_half_up(256 (col - (W - h) + 1) / h); the centre column of an
          odd width has weight 0.
R-apply   y = ((256 - w) x + w f(x) + 128) >> 8, i.e. the exact convex
          combination rounded half up.
R-vblend  optional (section 5: convex combinations of the maps of adjacent
          blocks): with doubled block centres C_j = r0_j + r1_j - 1, row r of
          block j blends block j with its neighbour on r's side of the centre,
          j - 1 if 2r < C_j, else j + 1 (alone at the first and last centre):
          between the blocks a < b, v = round_half_up(256 (2r - C_a) /
          (C_b - C_a)) and each Q16 parameter of the row is floor(((256 - v)
          P_a + v P_b + 128) / 256) (A and Bq alike, per side and channel); the
          row's map is then evaluated and blended with the identity as in
          R-apply.  Needs blocks of at least one row (H >= NB).
R-qfit    optional (the map should make the main characteristics of the two
          distributions agree, section 3.1; a least-squares fit of quantiles
          instead of the two moments): with M = 64 levels p_i = (2i + 1) /
          (2M), the level-i quantile of a band histogram h with n samples is
          the smallest bin v with 2M cum_h(v) >= (2i + 1) n; x_i and f_i are
          the bin centres (in sample units) of the own and the facing band's
          quantiles, the shared spectrum's quantiles are y_i = (x_i + f_i) / 2
          (the midway distribution: the average of the two quantile
          functions), and (a, b) is the least-squares line of y on x:
          a = cov(x, y) / var(x) from exact integer sums (a = 1 when every x_i
          is equal), clamped to [a_min, a_max], b = mean(y) - a mean(x).  For
          two bands whose samples are affine images of each other it gives
          the moment fit's map.  Plain estimate only (standard and smoothing
          modes).
R-seam    seam gradient cost (section 4.2): box means of factor x factor
          blocks, the two box columns on each side of the seam aligned with
          it, Euclidean norm over the channels in sample units; the interior
          reference is the same cost at a virtual seam at column floor(W/2).
R-seam-rows  the rows of a seam are the boxes of the shorter image from the
          top; with no row, or an image narrower than two boxes, the cost is
          undefined (NaN).

Every floating-point step is one IEEE binary64 operation on Python floats
(no fused multiply-add), so the result is reproducible to the last bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NBINS = 256
CSLOTS = 3          # channel slots of every per-camera statistics array
LEFT, RIGHT = 0, 1  # camera sides


@dataclass(frozen=True)
class Camera:
    """Geometry of one camera.  bit_depth 8 means uint8 samples, 9..16 uint16."""
    width: int
    height: int
    channels: int = 3
    bit_depth: int = 8
    ring: int = 0
    pos: int = 0


@dataclass(frozen=True)
class Options:
    n_blocks: int = 16          # vertical blocks (section 3.1: 16 and 64 tested)
    band_width: int = 32        # B, clamped to floor(W / 2)
    closed_ring: bool = True
    smoothing: bool = False     # exponential smoothing of section 3.1
    ema_alpha: float = 0.05     # alpha of the blending equation of section 3.1
    a_min: float = 0.125
    a_max: float = 8.0
    vblend: bool = False        # blend the maps of adjacent blocks row by row (R-vblend)
    fit: str = "moments"        # "moments" (R-fit) or "quantile" (R-qfit)


# --------------------------------------------------------------------------
# Regions (section 3.1: bands along the seam, vertical blocks, half images)
# --------------------------------------------------------------------------

def block_bounds(height: int, n_blocks: int) -> list[tuple[int, int]]:
    """Rows [r0, r1) of every vertical block (reading R-block)."""
    return [(j * height // n_blocks, (j + 1) * height // n_blocks) for j in range(n_blocks)]


def block_of_row(row: int, height: int, n_blocks: int) -> int:
    """Index of the block that holds `row` (closed form of R-block)."""
    return ((row + 1) * n_blocks - 1) // height


def band_columns(width: int, band_width: int) -> tuple[tuple[int, int], tuple[int, int]]:
    """Column ranges of the left and right bands (reading R-band)."""
    b = min(band_width, width // 2)
    return (0, b), (width - b, width)


def ring_order(cams: list[Camera], ring: int) -> list[int]:
    """Camera indices of one ring sorted by ring position."""
    return [i for _, i in sorted((c.pos, i) for i, c in enumerate(cams) if c.ring == ring)]


def facing(cams: list[Camera], opts: Options, k: int, side: int):
    """(camera, side) whose band faces `side` of camera k across a seam, or None.

    Right side of position p meets the left side of position p + 1 (reading
    R-ring).  A one-camera closed ring faces itself.
    """
    order = ring_order(cams, cams[k].ring)
    m, p = len(order), order.index(k)
    if side == RIGHT:
        q = p + 1
        if q == m:
            if not opts.closed_ring:
                return None
            q = 0
        return order[q], LEFT
    q = p - 1
    if q < 0:
        if not opts.closed_ring:
            return None
        q = m - 1
    return order[q], RIGHT


# --------------------------------------------------------------------------
# Statistics (section 3.1: intensity distributions of the narrow bands)
# --------------------------------------------------------------------------

def sample_bins(values: np.ndarray, bit_depth: int) -> np.ndarray:
    """Histogram bin of every sample (reading R-bins)."""
    v = values.astype(np.int64)
    if bit_depth == 8:
        return v
    return np.minimum(v >> (bit_depth - 8), NBINS - 1)


def region_stats(pix: np.ndarray, bit_depth: int) -> tuple[np.ndarray, np.ndarray]:
    """256-bin histogram and exact (n, S1, S2) of each channel of a region.

    pix has shape (rows, cols, C).  Returns hist int64 [CSLOTS][256] and sums
    int64 [CSLOTS][3] = (count, sum of samples, sum of squared samples);
    channel slots >= C stay zero.
    """
    hist = np.zeros((CSLOTS, NBINS), np.int64)
    sums = np.zeros((CSLOTS, 3), np.int64)
    for c in range(pix.shape[2]):
        v = pix[:, :, c].astype(np.int64).ravel()
        hist[c] = np.bincount(sample_bins(v, bit_depth), minlength=NBINS)
        sums[c, 0] = v.size
        sums[c, 1] = int(v.sum())
        sums[c, 2] = int((v * v).sum())
    return hist, sums


def band_stats(frame: np.ndarray, cam: Camera, opts: Options) -> tuple[np.ndarray, np.ndarray]:
    """Statistics of every (side, block) band of one camera.

    Returns hist [2][NB][CSLOTS][256] and sums [2][NB][CSLOTS][3].
    """
    nb = opts.n_blocks
    hist = np.zeros((2, nb, CSLOTS, NBINS), np.int64)
    sums = np.zeros((2, nb, CSLOTS, 3), np.int64)
    cols = band_columns(cam.width, opts.band_width)
    for j, (r0, r1) in enumerate(block_bounds(cam.height, nb)):
        for s in (LEFT, RIGHT):
            c0, c1 = cols[s]
            hist[s, j], sums[s, j] = region_stats(frame[r0:r1, c0:c1, :], cam.bit_depth)
    return hist, sums


def whole_stats(frame: np.ndarray, cam: Camera) -> tuple[np.ndarray, np.ndarray]:
    """Statistics of the whole frame: hist [CSLOTS][256], sums [CSLOTS][3]."""
    return region_stats(frame, cam.bit_depth)


# --------------------------------------------------------------------------
# Estimate (section 3.1: shared spectrum and per-channel affine fit)
# --------------------------------------------------------------------------

def moments(n: int, s1: int, s2: int) -> tuple[float, float, float]:
    """Mean, variance and standard deviation from exact sums (binary64)."""
    nf = float(n)
    mu = float(s1) / nf
    ex2 = float(s2) / nf
    mu2 = mu * mu
    var = ex2 - mu2
    if var < 0.0:
        var = 0.0
    return mu, var, math.sqrt(var)


def fit_side(own: tuple[int, int, int], fac: tuple[int, int, int],
             a_min: float, a_max: float):
    """Affine map (a, b) that sends the own band onto the shared spectrum.

    own, fac are (n, S1, S2) of one channel of the own and the facing band.
    Returns None when either band is empty (reading R-fit).
    """
    if own[0] == 0 or fac[0] == 0:
        return None
    mu_o, var_o, sd_o = moments(*own)
    mu_f, _, sd_f = moments(*fac)
    mu_s = (mu_o + mu_f) / 2.0            # shared spectrum (reading R-mid)
    sd_s = (sd_o + sd_f) / 2.0
    a = 1.0 if var_o == 0.0 else sd_s / sd_o
    a = min(max(a, a_min), a_max)
    am = a * mu_o
    b = mu_s - am
    return a, b


QFIT_LEVELS = 64


def quantile_bins(hist: np.ndarray, levels: int = QFIT_LEVELS) -> list[int]:
    """Bin of the level-i quantile of a histogram, i = 0 .. levels - 1: the
    smallest bin v whose cumulative count reaches (2i + 1) / (2 levels) of the
    total (reading R-qfit).  Exact integers."""
    h = np.asarray(hist, np.int64)
    n = int(h.sum())
    cum2m = 2 * levels * np.cumsum(h)                       # 2M cum(v), exact int64
    need = (2 * np.arange(levels, dtype=np.int64) + 1) * n  # (2i + 1) n
    # smallest v with 2M cum(v) >= need: the left insertion point in the sorted cum2m
    return [int(v) for v in np.searchsorted(cum2m, need, side="left")]


def bin_centre2(v: int, bit_depth: int) -> int:
    """Twice the centre of bin v in sample units (bins of 2^(d - 8) samples
    for bit depth d > 8; the bin itself for 8-bit samples)."""
    sh = 0 if bit_depth == 8 else bit_depth - 8
    return ((2 * v) << sh) + (1 << sh) - 1


def fit_side_quantile(own_hist: np.ndarray, fac_hist: np.ndarray, bit_depth: int,
                      a_min: float, a_max: float):
    """Affine map (a, b) by the least-squares fit of the shared spectrum's
    quantiles on the own band's (reading R-qfit).  own_hist, fac_hist: one
    channel's 256-bin histograms.  None when either band is empty."""
    if int(own_hist.sum()) == 0 or int(fac_hist.sum()) == 0:
        return None
    M = QFIT_LEVELS
    x2 = [bin_centre2(v, bit_depth) for v in quantile_bins(own_hist)]    # 2 x_i
    f2 = [bin_centre2(v, bit_depth) for v in quantile_bins(fac_hist)]    # 2 f_i
    sx, sf = sum(x2), sum(f2)
    sxx = sum(x * x for x in x2)
    sxf = sum(x * f for x, f in zip(x2, f2))
    # With y_i = (x_i + f_i) / 2: M sum(x y) - sum(x) sum(y) = num / 8 and
    # M sum(x^2) - sum(x)^2 = den / 4 in the doubled integers.
    num = M * (sxx + sxf) - sx * (sx + sf)
    den = M * sxx - sx * sx
    a = 1.0 if den == 0 else float(num) / (2.0 * float(den))
    a = min(max(a, a_min), a_max)
    mu_o = float(sx) / float(2 * M)
    mu_s = float(sx + sf) / float(4 * M)
    am = a * mu_o
    b = mu_s - am
    return a, b


def ema(prev: float, new: float, alpha: float) -> float:
    """One step of the exponential smoothing of section 3.1 (reading R-ema)."""
    keep = 1.0 - alpha
    t_prev = keep * prev
    t_new = alpha * new
    return t_prev + t_new


def estimate(cams: list[Camera], opts: Options, band_sums: np.ndarray,
             prev_params: np.ndarray | None = None, prev_valid: np.ndarray | None = None,
             band_hist: np.ndarray | None = None):
    """Per (camera, side, block, channel) affine maps for one frame-set.

    band_sums: [K][2][NB][CSLOTS][3].  prev_params f64 [K][2][NB][CSLOTS][2],
    prev_valid u8 [K][2][NB][CSLOTS] (1 = the unit holds an estimate).
    band_hist [K][2][NB][CSLOTS][256]: needed by the quantile fit (R-qfit).
    Returns (params, valid) of the same shapes.
    """
    if opts.fit not in ("moments", "quantile"):
        raise ValueError(f"unknown fit {opts.fit!r}")
    if opts.fit == "quantile" and band_hist is None:
        raise ValueError("the quantile fit needs the band histograms")
    K, nb = len(cams), opts.n_blocks
    if prev_params is None:
        prev_params = np.zeros((K, 2, nb, CSLOTS, 2), np.float64)
        prev_params[..., 0] = 1.0
    if prev_valid is None:
        prev_valid = np.zeros((K, 2, nb, CSLOTS), np.uint8)
    params = np.zeros((K, 2, nb, CSLOTS, 2), np.float64)
    valid = np.zeros((K, 2, nb, CSLOTS), np.uint8)
    for k, cam in enumerate(cams):
        for s in (LEFT, RIGHT):
            fc = facing(cams, opts, k, s)
            for j in range(nb):
                for c in range(CSLOTS):
                    if c >= cam.channels:
                        params[k, s, j, c] = (1.0, 0.0)
                        continue
                    if fc is None:
                        params[k, s, j, c] = (1.0, 0.0)
                        valid[k, s, j, c] = 1
                        continue
                    own = tuple(int(v) for v in band_sums[k, s, j, c])
                    fac = tuple(int(v) for v in band_sums[fc[0], fc[1], j, c])
                    if opts.fit == "quantile":
                        new = fit_side_quantile(band_hist[k, s, j, c], band_hist[fc[0], fc[1], j, c],
                                                cam.bit_depth, opts.a_min, opts.a_max)
                    else:
                        new = fit_side(own, fac, opts.a_min, opts.a_max)
                    had = bool(prev_valid[k, s, j, c])
                    if new is None:
                        if had:
                            params[k, s, j, c] = prev_params[k, s, j, c]
                            valid[k, s, j, c] = 1
                        else:
                            params[k, s, j, c] = (1.0, 0.0)
                        continue
                    a, b = new
                    if opts.smoothing and had:
                        a = ema(float(prev_params[k, s, j, c, 0]), a, opts.ema_alpha)
                        b = ema(float(prev_params[k, s, j, c, 1]), b, opts.ema_alpha)
                    params[k, s, j, c] = (a, b)
                    valid[k, s, j, c] = 1
    return params, valid


# --------------------------------------------------------------------------
# Object removal with the smoothing fallback (section 3.1, the two
# supplemental methods for moving objects; section 4.1 prefers removal when
# enough of the block remains)
# --------------------------------------------------------------------------
#
# R-move    a pixel is moving when its thresholded absolute difference to the
#           previous frame of the same camera exceeds tau on some channel:
#           max_c |x_t - x_{t-1}| > tau << (bit_depth - 8), tau in 8-bit
#           units (tau = 20 by default).  Without a previous frame nothing
#           moves.
# R-kept    removal drops the moving pixels from the band statistics: the
#           kept sums (n, S1, S2) of a band count only the pixels that do
#           not move.
# R-select  per seam unit, the removal fit (kept sums of both facing bands,
#           then the context's temporal mode) is used when at least a
#           fraction min_kept (0.25 by default) of each band's pixels is
#           kept, the fraction computed in binary64 as kept_n / n; otherwise
#           the smoothing fallback: the fit of the full bands blended as
#           E = (1 - alpha) E_prev + alpha E_new (the first estimate taken as
#           is).  Both sides of a seam see the same two fractions, so they
#           take the same method.

REMOVAL_TAU = 20
REMOVAL_MIN_KEPT = 0.25
METHOD_NONE, METHOD_REMOVAL, METHOD_SMOOTHING = 0, 1, 2


def moving_mask(frame: np.ndarray, prev: np.ndarray | None, bit_depth: int, tau: int) -> np.ndarray:
    """bool (rows, cols): the pixels whose difference to `prev` exceeds the threshold (R-move)."""
    if prev is None:
        return np.zeros(frame.shape[:2], bool)
    d = np.abs(frame.astype(np.int64) - prev.astype(np.int64)).max(axis=2)
    return d > (tau << (bit_depth - 8))


def kept_band_sums(frame: np.ndarray, prev: np.ndarray | None, cam: Camera, opts: Options,
                   tau: int = REMOVAL_TAU) -> np.ndarray:
    """(n, S1, S2) of the kept pixels of every (side, block) band, [2][NB][CSLOTS][3] (R-kept)."""
    nb = opts.n_blocks
    out = np.zeros((2, nb, CSLOTS, 3), np.int64)
    moving = moving_mask(frame, prev, cam.bit_depth, tau)
    cols = band_columns(cam.width, opts.band_width)
    for j, (r0, r1) in enumerate(block_bounds(cam.height, nb)):
        for s in (LEFT, RIGHT):
            c0, c1 = cols[s]
            keep = ~moving[r0:r1, c0:c1]
            for c in range(cam.channels):
                v = frame[r0:r1, c0:c1, c].astype(np.int64)[keep]
                out[s, j, c] = (v.size, int(v.sum()), int((v * v).sum()))
    return out


def estimate_removal(cams: list[Camera], opts: Options, band_sums: np.ndarray, kept_sums: np.ndarray,
                     prev_params: np.ndarray | None = None, prev_valid: np.ndarray | None = None,
                     min_kept: float = REMOVAL_MIN_KEPT):
    """Per unit: the removal fit or the smoothing fallback (R-select).

    Returns (params, valid, method); method u8 [K][2][NB] is METHOD_REMOVAL,
    METHOD_SMOOTHING, or METHOD_NONE where no new estimate was made (no facing
    band, or an empty band).  The fits are the moment fit (R-fit) only.
    """
    if opts.fit != "moments":
        raise ValueError("object removal keeps only the moments of the kept pixels")
    K, nb = len(cams), opts.n_blocks
    if prev_params is None:
        prev_params = np.zeros((K, 2, nb, CSLOTS, 2), np.float64)
        prev_params[..., 0] = 1.0
    if prev_valid is None:
        prev_valid = np.zeros((K, 2, nb, CSLOTS), np.uint8)
    params = np.zeros((K, 2, nb, CSLOTS, 2), np.float64)
    valid = np.zeros((K, 2, nb, CSLOTS), np.uint8)
    method = np.zeros((K, 2, nb), np.uint8)
    for k, cam in enumerate(cams):
        for s in (LEFT, RIGHT):
            fc = facing(cams, opts, k, s)
            for j in range(nb):
                m = METHOD_NONE
                if fc is not None:
                    n_own, n_fac = int(band_sums[k, s, j, 0, 0]), int(band_sums[fc[0], fc[1], j, 0, 0])
                    if n_own > 0 and n_fac > 0:
                        kn_own, kn_fac = int(kept_sums[k, s, j, 0, 0]), int(kept_sums[fc[0], fc[1], j, 0, 0])
                        f_own = float(kn_own) / float(n_own)
                        f_fac = float(kn_fac) / float(n_fac)
                        ok = kn_own > 0 and kn_fac > 0 and f_own >= min_kept and f_fac >= min_kept
                        m = METHOD_REMOVAL if ok else METHOD_SMOOTHING
                method[k, s, j] = m
                for c in range(CSLOTS):
                    if c >= cam.channels:
                        params[k, s, j, c] = (1.0, 0.0)
                        continue
                    if fc is None:
                        params[k, s, j, c] = (1.0, 0.0)
                        valid[k, s, j, c] = 1
                        continue
                    had = bool(prev_valid[k, s, j, c])
                    if m == METHOD_NONE:
                        if had:
                            params[k, s, j, c] = prev_params[k, s, j, c]
                            valid[k, s, j, c] = 1
                        else:
                            params[k, s, j, c] = (1.0, 0.0)
                        continue
                    src = kept_sums if m == METHOD_REMOVAL else band_sums
                    own = tuple(int(v) for v in src[k, s, j, c])
                    fac = tuple(int(v) for v in src[fc[0], fc[1], j, c])
                    a, b = fit_side(own, fac, opts.a_min, opts.a_max)
                    smooth = opts.smoothing if m == METHOD_REMOVAL else True
                    if smooth and had:
                        a = ema(float(prev_params[k, s, j, c, 0]), a, opts.ema_alpha)
                        b = ema(float(prev_params[k, s, j, c, 1]), b, opts.ema_alpha)
                    params[k, s, j, c] = (a, b)
                    valid[k, s, j, c] = 1
    return params, valid, method


# --------------------------------------------------------------------------
# LUTs and column weights (section 3.1: the map and its convex blend)
# --------------------------------------------------------------------------

def q16(value: float) -> int:
    """round_half_even(value * 65536) as an exact integer (reading R-q16)."""
    return int(round(value * 65536.0))


def affine_fixed(A: int, Bq: int, x: int, max_value: int) -> int:
    """f(x) = clamp((A x + Bq + 32768) >> 16, 0, max_value) in exact integers."""
    y = (A * x + Bq + 32768) >> 16
    return min(max(y, 0), max_value)


def lut_u8(a: float, b: float) -> np.ndarray:
    """256-entry uint8 table of the affine map (a, b)."""
    A, Bq = q16(a), q16(b)
    return np.array([affine_fixed(A, Bq, x, 255) for x in range(NBINS)], np.uint8)


def build_luts(cams: list[Camera], opts: Options, params: np.ndarray):
    """lut8 u8 [K][2][NB][CSLOTS][256] (uint8 cameras only) and q16 i64 [K][2][NB][CSLOTS][2]."""
    K, nb = len(cams), opts.n_blocks
    lut8 = np.zeros((K, 2, nb, CSLOTS, NBINS), np.uint8)
    qq = np.zeros((K, 2, nb, CSLOTS, 2), np.int64)
    for k, cam in enumerate(cams):
        for s in (LEFT, RIGHT):
            for j in range(nb):
                for c in range(CSLOTS):
                    a, b = float(params[k, s, j, c, 0]), float(params[k, s, j, c, 1])
                    qq[k, s, j, c] = (q16(a), q16(b))
                    if cam.bit_depth == 8:
                        lut8[k, s, j, c] = lut_u8(a, b)
    return lut8, qq


def column_weights(width: int) -> tuple[np.ndarray, np.ndarray]:
    """Q8 weight and side (0 left, 1 right, -1 centre) of every column (reading R-weight)."""
    h = width // 2
    w = np.zeros(width, np.int64)
    side = np.full(width, -1, np.int64)
    for col in range(width):
        if col < h:
            side[col] = LEFT
            w[col] = ((h - col) * 256 + h // 2) // h
        elif col >= width - h:
            side[col] = RIGHT
            w[col] = ((col - width + h + 1) * 256 + h // 2) // h
    return w, side


def weights_table(cams: list[Camera]) -> np.ndarray:
    """u16 [K][W_max] column weights, zero beyond each camera's width."""
    wmax = max(c.width for c in cams)
    t = np.zeros((len(cams), wmax), np.uint16)
    for k, cam in enumerate(cams):
        t[k, :cam.width] = column_weights(cam.width)[0]
    return t


# --------------------------------------------------------------------------
# Apply (section 3.1: identity at the centre, f_c at the border)
# --------------------------------------------------------------------------

def blend(x: np.ndarray, fx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y = ((256 - w) x + w f(x) + 128) >> 8 in exact integers (reading R-apply)."""
    return ((256 - w) * x + w * fx + 128) >> 8


def row_blend(height: int, n_blocks: int, row: int) -> tuple[int, int, int]:
    """(block a, block b, Q8 weight v of b) of one row under R-vblend; a == b
    with v = 0 where the row takes one block's map."""
    bounds = block_bounds(height, n_blocks)
    j = block_of_row(row, height, n_blocks)
    cj = bounds[j][0] + bounds[j][1] - 1
    if 2 * row < cj:
        a, b = j - 1, j
    else:
        a, b = j, j + 1
    if a < 0 or b >= n_blocks:
        return j, j, 0
    ca = bounds[a][0] + bounds[a][1] - 1
    cb = bounds[b][0] + bounds[b][1] - 1
    v = ((2 * row - ca) * 512 + (cb - ca)) // (2 * (cb - ca))
    return a, b, v


def blend_q16(pa: int, pb: int, v: int) -> int:
    """floor(((256 - v) pa + v pb + 128) / 256) in exact integers (R-vblend)."""
    return ((256 - v) * pa + v * pb + 128) >> 8


def apply_camera_vblend(frame: np.ndarray, cam: Camera, opts: Options, q16_cam: np.ndarray) -> np.ndarray:
    """Corrected copy of one frame with the maps of adjacent blocks blended row
    by row (R-vblend).  q16_cam [2][NB][CSLOTS][2]."""
    if cam.height < opts.n_blocks:
        raise ValueError("blending adjacent blocks needs blocks of at least one row")
    out = frame.copy()
    w, side = column_weights(cam.width)
    maxv = (1 << cam.bit_depth) - 1
    for r in range(cam.height):
        a, b, v = row_blend(cam.height, opts.n_blocks, r)
        for s in (LEFT, RIGHT):
            cols = np.nonzero(side == s)[0]
            if cols.size == 0:
                continue
            for c in range(cam.channels):
                A = blend_q16(int(q16_cam[s, a, c, 0]), int(q16_cam[s, b, c, 0]), v)
                Bq = blend_q16(int(q16_cam[s, a, c, 1]), int(q16_cam[s, b, c, 1]), v)
                x = frame[r, cols, c].astype(np.int64)
                fx = np.clip((A * x + Bq + 32768) >> 16, 0, maxv)
                out[r, cols, c] = blend(x, fx, w[cols]).astype(frame.dtype)
    return out


def apply_camera(frame: np.ndarray, cam: Camera, opts: Options,
                 lut8_cam: np.ndarray, q16_cam: np.ndarray) -> np.ndarray:
    """Corrected copy of one frame.  lut8_cam [2][NB][CSLOTS][256], q16_cam [2][NB][CSLOTS][2]."""
    if opts.vblend:
        return apply_camera_vblend(frame, cam, opts, q16_cam)
    out = frame.copy()
    w, side = column_weights(cam.width)
    maxv = (1 << cam.bit_depth) - 1
    for j, (r0, r1) in enumerate(block_bounds(cam.height, opts.n_blocks)):
        for s in (LEFT, RIGHT):
            cols = np.nonzero(side == s)[0]
            if cols.size == 0 or r1 == r0:
                continue
            ws = w[cols][None, :]
            for c in range(cam.channels):
                x = frame[r0:r1][:, cols, c].astype(np.int64)
                if cam.bit_depth == 8:
                    fx = lut8_cam[s, j, c].astype(np.int64)[x]
                else:
                    A, Bq = int(q16_cam[s, j, c, 0]), int(q16_cam[s, j, c, 1])
                    fx = np.clip((A * x + Bq + 32768) >> 16, 0, maxv)
                out[r0:r1, cols[0]:cols[-1] + 1, c] = blend(x, fx, ws).astype(frame.dtype)
    return out


# --------------------------------------------------------------------------
# One frame-set end to end
# --------------------------------------------------------------------------

def frameset(cams: list[Camera], opts: Options, frames: list[np.ndarray],
             prev_params: np.ndarray | None = None, prev_valid: np.ndarray | None = None) -> dict:
    """Statistics -> estimate -> LUTs -> apply for one synchronized frame-set.

    Whole-frame statistics are of the input frames.
    """
    K, nb = len(cams), opts.n_blocks
    bh = np.zeros((K, 2, nb, CSLOTS, NBINS), np.int64)
    bs = np.zeros((K, 2, nb, CSLOTS, 3), np.int64)
    wh = np.zeros((K, CSLOTS, NBINS), np.int64)
    ws = np.zeros((K, CSLOTS, 3), np.int64)
    for k, (cam, f) in enumerate(zip(cams, frames)):
        bh[k], bs[k] = band_stats(f, cam, opts)
        wh[k], ws[k] = whole_stats(f, cam)
    params, valid = estimate(cams, opts, bs, prev_params, prev_valid, band_hist=bh)
    lut8, qq = build_luts(cams, opts, params)
    outs = [apply_camera(f, cam, opts, lut8[k], qq[k]) for k, (cam, f) in enumerate(zip(cams, frames))]
    return dict(band_hist=bh, band_sums=bs, whole_hist=wh, whole_sums=ws, params=params,
                valid=valid, lut8=lut8, q16=qq, weights=weights_table(cams), out=outs)


def frameset_removal(cams: list[Camera], opts: Options, frames: list[np.ndarray],
                     prev_frames: list[np.ndarray] | None, prev_params: np.ndarray | None = None,
                     prev_valid: np.ndarray | None = None, tau: int = REMOVAL_TAU,
                     min_kept: float = REMOVAL_MIN_KEPT) -> dict:
    """frameset() with object removal and the smoothing fallback: the band
    statistics of the whole bands, the kept sums against the previous frames
    (None: nothing moves), the estimate by R-select, tables and apply."""
    r = frameset(cams, opts, frames, prev_params, prev_valid)
    kept = np.stack([kept_band_sums(f, None if prev_frames is None else prev_frames[k], cam, opts, tau)
                     for k, (cam, f) in enumerate(zip(cams, frames))])
    params, valid, method = estimate_removal(cams, opts, r["band_sums"], kept, prev_params, prev_valid, min_kept)
    lut8, qq = build_luts(cams, opts, params)
    outs = [apply_camera(f, cam, opts, lut8[k], qq[k]) for k, (cam, f) in enumerate(zip(cams, frames))]
    r.update(kept_sums=kept, params=params, valid=valid, method=method, lut8=lut8, q16=qq, out=outs)
    return r


# --------------------------------------------------------------------------
# Seam gradient cost (section 4.2, the gradient-cost equation)
# --------------------------------------------------------------------------

def box_downsample(img: np.ndarray, factor: int, from_right: bool) -> np.ndarray:
    """Mean of non-overlapping factor x factor boxes (binary64).

    Rows are taken from the top; columns from the right edge when from_right
    (so that the last box column touches the seam), else from the left edge.
    """
    h = img.shape[0] // factor * factor
    wc = img.shape[1] // factor * factor
    sub = img[:h, img.shape[1] - wc:] if from_right else img[:h, :wc]
    sub = sub.astype(np.float64)
    r, cc = h // factor, wc // factor
    return sub.reshape(r, factor, cc, factor, img.shape[2]).mean(axis=(1, 3))


def seam_row_costs(left: np.ndarray, right: np.ndarray, factor: int = 8) -> np.ndarray:
    """(d+ + d-)/2 for every downsampled row of the seam between `left` and `right`.

    d+ = |(I+_1 - I+_0) - (I+_0 - I-_0)|, d- = |(I-_-1 - I-_0) - (I-_0 - I+_0)|,
    with |.| the Euclidean norm over the colour channels, after box
    downsampling by `factor` in both directions (R-seam).  The rows are the
    boxes of the shorter image from the top (R-seam-rows); empty when either
    image is narrower than two boxes or shorter than one.
    """
    n = min(left.shape[0], right.shape[0]) // factor
    if n == 0 or left.shape[1] < 2 * factor or right.shape[1] < 2 * factor:
        return np.zeros(0, np.float64)
    lft = box_downsample(left[:n * factor, left.shape[1] - 2 * factor:], factor, True)
    rgt = box_downsample(right[:n * factor, :2 * factor], factor, False)
    im1, im0 = lft[:, 0, :], lft[:, 1, :]
    ip0, ip1 = rgt[:, 0, :], rgt[:, 1, :]
    d_plus = np.sqrt((((ip1 - ip0) - (ip0 - im0)) ** 2).sum(axis=1))
    d_minus = np.sqrt((((im1 - im0) - (im0 - ip0)) ** 2).sum(axis=1))
    return (d_plus + d_minus) / 2.0


def seam_cost(left: np.ndarray, right: np.ndarray, factor: int = 8) -> float:
    """The gradient cost of section 4.2: the mean over rows of (d+ + d-)/2
    (seam_row_costs); NaN when no row is defined."""
    r = seam_row_costs(left, right, factor)
    return float(r.mean()) if r.size else math.nan


def interior_rows(img: np.ndarray, factor: int = 8) -> np.ndarray:
    """Row costs at a virtual seam in the middle of one image: columns
    [0, W/2) on the left, [W/2, W) on the right (section 4.2's reference)."""
    m = img.shape[1] // 2
    return seam_row_costs(img[:, :m], img[:, m:], factor)


def interior_cost(img: np.ndarray, factor: int = 8) -> float:
    """The same cost at a virtual seam in the middle of one image (section 4.2)."""
    r = interior_rows(img, factor)
    return float(r.mean()) if r.size else math.nan


def seam_costs(cams: list[Camera], opts: Options, frames: list[np.ndarray], factor: int = 8) -> dict:
    """The cost of every seam of the rig and the interior reference of every camera.

    seam[k]: the seam between camera k (left image) and the camera its right
    side faces (R-ring), NaN without one; interior[k]: the virtual seam in
    the middle of camera k.  seam_rows[k] / interior_rows[k] hold the row
    values behind each mean.
    """
    K = len(cams)
    seam = np.full(K, math.nan)
    interior = np.full(K, math.nan)
    s_rows, i_rows = [], []
    for k in range(K):
        fc = facing(cams, opts, k, RIGHT)
        r = seam_row_costs(frames[k], frames[fc[0]], factor) if fc is not None else np.zeros(0)
        s_rows.append(r)
        if r.size:
            seam[k] = float(r.mean())
        ri = interior_rows(frames[k], factor)
        i_rows.append(ri)
        if ri.size:
            interior[k] = float(ri.mean())
    return dict(seam=seam, interior=interior, seam_rows=s_rows, interior_rows=i_rows)
