"""Oracle of the cross-channel 3x3 linear maps (section 5 names 3x3 linear
maps across the colour channels as an improvement over one affine map per
channel).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain, slow and exact.

Readings (the paper gives the idea only):

R-x3-stats  per band of an RGB camera, besides (n, S1, S2) per channel, the
            exact cross sums S_RG, S_RB, S_GB of the products of a pixel's
            channel samples.
R-x3-fit    with mu = S1 / n and the covariance C_cd = S_cd / n - mu_c mu_d
            (binary64; the diagonal is the variance of R-fit, clamped at 0),
            L_own and L_fac are the Cholesky factors (lower triangular,
            positive diagonal) of the own and the facing band's covariance;
            the shared spectrum has mean mu* = (mu_own + mu_fac) / 2 and the
            factor L* = (L_own + L_fac) / 2 (entry by entry: the
            generalisation of sigma* = (sigma_own + sigma_fac) / 2 of R-mid);
            the map is y = M x + t with M = L* L_own^-1 (solved row by row
            against L_own from the last column to the first) and
            t = mu* - M mu_own, which sends a band with the own mean and
            covariance to one with mean mu* and covariance L* L*^T.  Each
            operation is one binary64 operation in the order written in
            fit_cross.  Fallback: when either covariance has a pivot <= 0, or
            a diagonal entry of M lies outside [a_min, a_max], or an
            off-diagonal entry exceeds a_max in magnitude (or is NaN), M and t
            are the per-channel fits of R-fit (a diagonal M).  No estimate
            when either band is empty (the unit keeps its state, identity if
            none); identity without a facing band.
R-x3-ema    smoothing blends the twelve parameters (M row-major, then t)
            pointwise as R-ema does.
R-x3-q16    A_rc = round_half_even(M_rc 65536), B_r = round_half_even(t_r
            65536); f_r(x) = clamp((A_r0 x_0 + A_r1 x_1 + A_r2 x_2 + B_r +
            32768) >> 16, 0, 255) in exact integers; then R-weight and
            R-apply per channel: y_r = ((256 - w) x_r + w f_r(x) + 128) >> 8.

Only 8-bit RGB cameras take these maps.
"""
from __future__ import annotations

import math

import numpy as np

from . import ringcorr as rc

NPARAM = 12          # M row-major (9), then t (3)
PAIRS = ((0, 1), (0, 2), (1, 2))


def cross_sums(pix: np.ndarray) -> np.ndarray:
    """(S_RG, S_RB, S_GB) of a region of an RGB image (rows, cols, 3), exact (R-x3-stats)."""
    v = pix.astype(np.int64).reshape(-1, 3)
    return np.array([int((v[:, a] * v[:, b]).sum()) for a, b in PAIRS], np.int64)


def band_cross(frame: np.ndarray, cam: rc.Camera, opts: rc.Options) -> np.ndarray:
    """Cross sums of every (side, block) band of one RGB camera: [2][NB][3]."""
    nb = opts.n_blocks
    out = np.zeros((2, nb, 3), np.int64)
    cols = rc.band_columns(cam.width, opts.band_width)
    for j, (r0, r1) in enumerate(rc.block_bounds(cam.height, nb)):
        for s in (rc.LEFT, rc.RIGHT):
            c0, c1 = cols[s]
            out[s, j] = cross_sums(frame[r0:r1, c0:c1, :])
    return out


def mean_cov(sums: np.ndarray, cross: np.ndarray):
    """Mean vector and covariance (3x3 list) of a band from its exact sums:
    sums [3][3] = (n, S1, S2) per channel, cross = (S_RG, S_RB, S_GB)."""
    n = float(int(sums[0][0]))
    mu = [float(int(sums[c][1])) / n for c in range(3)]
    cov = [[0.0] * 3 for _ in range(3)]
    for c in range(3):
        ex = float(int(sums[c][2])) / n
        m2 = mu[c] * mu[c]
        v = ex - m2
        cov[c][c] = v if v > 0.0 else 0.0
    for i, (a, b) in enumerate(PAIRS):
        ex = float(int(cross[i])) / n
        m2 = mu[a] * mu[b]
        cov[a][b] = cov[b][a] = ex - m2
    return mu, cov


def cholesky3(cov):
    """Lower-triangular L with L L^T = cov (binary64, fixed order), or None
    when a pivot is not positive."""
    if not cov[0][0] > 0.0:
        return None
    l00 = math.sqrt(cov[0][0])
    l10 = cov[1][0] / l00
    l20 = cov[2][0] / l00
    p11 = cov[1][1] - l10 * l10
    if not p11 > 0.0:
        return None
    l11 = math.sqrt(p11)
    l21 = (cov[2][1] - l20 * l10) / l11
    p22 = (cov[2][2] - l20 * l20) - l21 * l21
    if not p22 > 0.0:
        return None
    l22 = math.sqrt(p22)
    return [[l00, 0.0, 0.0], [l10, l11, 0.0], [l20, l21, l22]]


def solve_right(Ls, L):
    """M with M L = Ls for lower-triangular L (row by row, last column first)."""
    M = [[0.0] * 3 for _ in range(3)]
    for r in range(3):
        m2 = Ls[r][2] / L[2][2]
        m1 = (Ls[r][1] - m2 * L[2][1]) / L[1][1]
        m0 = ((Ls[r][0] - m1 * L[1][0]) - m2 * L[2][0]) / L[0][0]
        M[r] = [m0, m1, m2]
    return M


def fit_cross(own_sums, own_cross, fac_sums, fac_cross, a_min: float, a_max: float):
    """(M, t) of the own side (reading R-x3-fit), or None when a band is empty."""
    if int(own_sums[0][0]) == 0 or int(fac_sums[0][0]) == 0:
        return None
    mu_o, cov_o = mean_cov(own_sums, own_cross)
    mu_f, cov_f = mean_cov(fac_sums, fac_cross)
    Lo, Lf = cholesky3(cov_o), cholesky3(cov_f)
    ok = Lo is not None and Lf is not None
    if ok:
        Ls = [[(Lo[r][c] + Lf[r][c]) / 2.0 for c in range(3)] for r in range(3)]
        M = solve_right(Ls, Lo)
        for r in range(3):
            for c in range(3):
                m = M[r][c]
                good = (a_min <= m <= a_max) if r == c else (-a_max <= m <= a_max)
                ok = ok and good
    if not ok:
        M = [[0.0] * 3 for _ in range(3)]
        t = [0.0] * 3
        for c in range(3):
            a, b = rc.fit_side(tuple(int(v) for v in own_sums[c]), tuple(int(v) for v in fac_sums[c]), a_min, a_max)
            M[c][c] = a
            t[c] = b
        return M, t
    mu_s = [(mu_o[c] + mu_f[c]) / 2.0 for c in range(3)]
    t = []
    for r in range(3):
        mx = (M[r][0] * mu_o[0] + M[r][1] * mu_o[1]) + M[r][2] * mu_o[2]
        t.append(mu_s[r] - mx)
    return M, t


def flat(M, t) -> list[float]:
    return [M[r][c] for r in range(3) for c in range(3)] + list(t)


IDENTITY = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0]


def estimate_cross(cams, opts: rc.Options, band_sums: np.ndarray, cross: np.ndarray,
                   prev: np.ndarray | None = None, prev_valid: np.ndarray | None = None):
    """Per (camera, side, block) cross-channel maps: params f64 [K][2][NB][12]
    (M row-major, then t) and valid u8 [K][2][NB] (R-x3-fit, R-x3-ema).
    band_sums [K][2][NB][3][3], cross [K][2][NB][3]."""
    K, nb = len(cams), opts.n_blocks
    if any(c.channels != 3 or c.bit_depth != 8 for c in cams):
        raise ValueError("cross-channel maps need 8-bit RGB cameras")
    if prev is None:
        prev = np.tile(np.array(IDENTITY), (K, 2, nb, 1))
    if prev_valid is None:
        prev_valid = np.zeros((K, 2, nb), np.uint8)
    params = np.tile(np.array(IDENTITY), (K, 2, nb, 1))
    valid = np.zeros((K, 2, nb), np.uint8)
    for k in range(K):
        for s in (rc.LEFT, rc.RIGHT):
            fc = rc.facing(cams, opts, k, s)
            for j in range(nb):
                if fc is None:
                    valid[k, s, j] = 1
                    continue
                had = bool(prev_valid[k, s, j])
                new = fit_cross(band_sums[k, s, j], cross[k, s, j], band_sums[fc[0], fc[1], j],
                                cross[fc[0], fc[1], j], opts.a_min, opts.a_max)
                if new is None:
                    if had:
                        params[k, s, j] = prev[k, s, j]
                        valid[k, s, j] = 1
                    continue
                p = flat(*new)
                if opts.smoothing and had:
                    p = [rc.ema(float(prev[k, s, j, i]), p[i], opts.ema_alpha) for i in range(NPARAM)]
                params[k, s, j] = p
                valid[k, s, j] = 1
    return params, valid


def build_cross(cams, opts: rc.Options, params: np.ndarray) -> np.ndarray:
    """q3 i64 [K][2][NB][12] = round_half_even(params * 65536) (R-x3-q16)."""
    q = np.zeros(params.shape, np.int64)
    for idx in np.ndindex(params.shape):
        q[idx] = rc.q16(float(params[idx]))
    return q


def map_pixel(q: np.ndarray, x) -> list[int]:
    """f(x) of one pixel under the Q16 map q [12] (R-x3-q16)."""
    out = []
    for r in range(3):
        y = (int(q[3 * r]) * int(x[0]) + int(q[3 * r + 1]) * int(x[1]) + int(q[3 * r + 2]) * int(x[2])
             + int(q[9 + r]) + 32768) >> 16
        out.append(min(max(y, 0), 255))
    return out


def apply_camera_cross(frame: np.ndarray, cam: rc.Camera, opts: rc.Options, q_cam: np.ndarray) -> np.ndarray:
    """Corrected frame of one camera with its maps q_cam [2][NB][12] (vectorised
    over pixels, exact int64)."""
    w, side = rc.column_weights(cam.width)
    x = frame.astype(np.int64)
    out = frame.copy()
    for j, (r0, r1) in enumerate(rc.block_bounds(cam.height, opts.n_blocks)):
        for s in (rc.LEFT, rc.RIGHT):
            cols = np.nonzero(side == s)[0]
            if cols.size == 0 or r1 <= r0:
                continue
            q = q_cam[s, j].astype(np.int64)
            xs = x[r0:r1, cols, :]
            ww = w[cols][None, :]
            for r in range(3):
                f = (q[3 * r] * xs[..., 0] + q[3 * r + 1] * xs[..., 1] + q[3 * r + 2] * xs[..., 2] + q[9 + r]
                     + 32768) >> 16
                f = np.clip(f, 0, 255)
                out[r0:r1, cols, r] = rc.blend(xs[..., r], f, ww).astype(frame.dtype)
    return out


def frameset_cross(cams, opts: rc.Options, frames, prev=None, prev_valid=None) -> dict:
    """Statistics -> cross-channel estimate -> Q16 maps -> apply for one frame-set."""
    K, nb = len(cams), opts.n_blocks
    bs = np.zeros((K, 2, nb, rc.CSLOTS, 3), np.int64)
    cr = np.zeros((K, 2, nb, 3), np.int64)
    wh = np.zeros((K, rc.CSLOTS, rc.NBINS), np.int64)
    ws = np.zeros((K, rc.CSLOTS, 3), np.int64)
    for k, (cam, f) in enumerate(zip(cams, frames)):
        _, bs[k] = rc.band_stats(f, cam, opts)
        cr[k] = band_cross(f, cam, opts)
        wh[k], ws[k] = rc.whole_stats(f, cam)
    params, valid = estimate_cross(cams, opts, bs, cr, prev, prev_valid)
    q = build_cross(cams, opts, params)
    outs = [apply_camera_cross(f, cam, opts, q[k]) for k, (cam, f) in enumerate(zip(cams, frames))]
    return dict(band_sums=bs, cross=cr, whole_hist=wh, whole_sums=ws, params=params, valid=valid, q3=q,
                weights=rc.weights_table(cams), out=outs)
