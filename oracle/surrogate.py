"""Oracle for the learned surrogate of the estimate.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper has no
network; the surrogate is specified by the project: a small MLP that maps the
normalised 64-bin histograms of a unit's surroundings to that unit's affine
maps, trained on the plain estimator's output, with the plain estimator as
fallback.  Everything here is binary64 unless a step says otherwise.

Unit        (camera k, side s, block j) of an RGB camera.
Features    576 = 3 regions x 3 channels x 64 bins, region-major, then channel,
            then bin.  Regions: 0 the whole frame of camera k as passed in (the
            previous frame-set's at inference), 1 the unit's own band, 2 the
            facing band of the same block (zeros without one).  Each 64-bin
            histogram sums 4 adjacent 256-bins, times 64, divided by the
            region's sample count (a density relative to a flat histogram, so
            that inputs are of order one; zeros when the count is 0), computed
            in binary64 and rounded once to float32.
Targets     6 = (a_R, a_G, a_B, b_R/255, b_G/255, b_B/255) of the plain
            estimate of the unit (before any temporal smoothing).
Network     576 -> 256 (ReLU) -> 256 (ReLU) -> 6, y = x W + b per layer.
Loss        mean over the N x 6 outputs of (y - target)^2.
Optimizer   Adam with bias correction.
Fallback    residual r = max_c max(|a^_c - a_c|, |b^n_c - b_c / 255|) against
            the plain estimate of the same unit; the network's output is used
            iff every output is finite and r <= tol (all three channels of the
            unit together); otherwise the plain estimate.  The decision is
            taken on the predictions as given (float32 from the device), and a
            used prediction becomes (a, b) = (double(a^), 255 * double(b^n)).
"""
from __future__ import annotations

import numpy as np

from . import ringcorr as rc

IN, HID, OUT = 576, 256, 6
BINS = 64


# ----------------------------------------------------------------------------- features

def merge64(h256: np.ndarray) -> np.ndarray:
    """Sum of 4 adjacent bins of a 256-bin histogram (exact integers)."""
    h = np.asarray(h256, dtype=np.int64)
    return np.array([h[4 * i] + h[4 * i + 1] + h[4 * i + 2] + h[4 * i + 3] for i in range(BINS)], np.int64)


def region_features(h3x256: np.ndarray) -> np.ndarray:
    """192 float32 features of one region: per channel, 64 * merged bins / count."""
    out = np.zeros((3, BINS), np.float32)
    for c in range(3):
        n = int(np.asarray(h3x256[c], dtype=np.int64).sum())
        if n == 0:
            continue
        m = merge64(h3x256[c])
        out[c] = np.array([np.float32(float(v) * 64.0 / float(n)) for v in m], np.float32)
    return out.ravel()


def unit_features(cams, opts, band_hist, whole_hist, k: int, s: int, j: int) -> np.ndarray:
    fc = rc.facing(cams, opts, k, s)
    regions = [whole_hist[k], band_hist[k, s, j]]
    regions.append(band_hist[fc[0], fc[1], j] if fc is not None else np.zeros((3, 256), np.int64))
    return np.concatenate([region_features(r) for r in regions]).astype(np.float32)


def all_features(cams, opts, band_hist, whole_hist) -> np.ndarray:
    """Features of every (camera, side, block), [K * 2 * NB][576]; rows of
    non-RGB cameras are zero."""
    K, nb = len(cams), opts.n_blocks
    X = np.zeros((K * 2 * nb, IN), np.float32)
    for k, cam in enumerate(cams):
        if cam.channels != 3:
            continue
        for s in (0, 1):
            for j in range(nb):
                X[(k * 2 + s) * nb + j] = unit_features(cams, opts, band_hist, whole_hist, k, s, j)
    return X


# ----------------------------------------------------------------------------- plain estimate, split

NONE, NEW, IDENTITY, UNUSED = 0, 1, 2, 3   # status of a (camera, side, block, channel) unit


def estimate_new(cams, opts, band_sums):
    """The plain estimate of every unit before the temporal step.

    Returns p_new f64 [K][2][NB][3][2] and status i32 [K][2][NB][3]:
    NEW (an estimate), NONE (an empty band: keep the state), IDENTITY (no
    facing band), UNUSED (channel slot beyond the camera's channels).
    """
    K, nb = len(cams), opts.n_blocks
    p = np.zeros((K, 2, nb, 3, 2), np.float64)
    p[..., 0] = 1.0
    st = np.zeros((K, 2, nb, 3), np.int32)
    for k, cam in enumerate(cams):
        for s in (0, 1):
            fc = rc.facing(cams, opts, k, s)
            for j in range(nb):
                for c in range(3):
                    if c >= cam.channels:
                        st[k, s, j, c] = UNUSED
                    elif fc is None:
                        st[k, s, j, c] = IDENTITY
                    else:
                        own = tuple(int(v) for v in band_sums[k, s, j, c])
                        fac = tuple(int(v) for v in band_sums[fc[0], fc[1], j, c])
                        r = rc.fit_side(own, fac, opts.a_min, opts.a_max)
                        if r is None:
                            st[k, s, j, c] = NONE
                        else:
                            st[k, s, j, c] = NEW
                            p[k, s, j, c] = r
    return p, st


def temporal(opts, p_new, status, prev_params, prev_valid):
    """The state update of the estimate (same rules as ringcorr.estimate)."""
    params = prev_params.copy()
    valid = prev_valid.copy()
    it = np.ndindex(*status.shape)
    for idx in it:
        st = status[idx]
        if st == UNUSED:
            params[idx] = (1.0, 0.0)
            valid[idx] = 0
        elif st == IDENTITY:
            params[idx] = (1.0, 0.0)
            valid[idx] = 1
        elif st == NONE:
            if not prev_valid[idx]:
                params[idx] = (1.0, 0.0)
        else:
            a, b = float(p_new[idx][0]), float(p_new[idx][1])
            if opts.smoothing and prev_valid[idx]:
                a = rc.ema(float(prev_params[idx][0]), a, opts.ema_alpha)
                b = rc.ema(float(prev_params[idx][1]), b, opts.ema_alpha)
            params[idx] = (a, b)
            valid[idx] = 1
    return params, valid


def targets(p_new_unit: np.ndarray) -> np.ndarray:
    """(a_R, a_G, a_B, b_R/255, b_G/255, b_B/255) of one unit's [3][2] parameters."""
    return np.array([p_new_unit[0, 0], p_new_unit[1, 0], p_new_unit[2, 0],
                     p_new_unit[0, 1] / 255.0, p_new_unit[1, 1] / 255.0, p_new_unit[2, 1] / 255.0], np.float64)


# ----------------------------------------------------------------------------- network

def forward(P: dict, X: np.ndarray):
    """Y and the hidden activations (binary64)."""
    X = np.asarray(X, np.float64)
    Z1 = X @ P["w1"] + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["w2"] + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ P["w3"] + P["b3"]
    return Y, H1, H2


def mse(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean((np.asarray(Y, np.float64) - np.asarray(T, np.float64)) ** 2))


def backward(P: dict, X: np.ndarray, H1: np.ndarray, H2: np.ndarray, Y: np.ndarray, T: np.ndarray) -> dict:
    """Gradients of mse(forward(P, X), T) with respect to every parameter."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    dY = 2.0 * (np.asarray(Y, np.float64) - np.asarray(T, np.float64)) / (n * OUT)
    g = {"w3": H2.T @ dY, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ P["w3"].T) * (H2 > 0)
    g["w2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["w2"].T) * (H1 > 0)
    g["w1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam(P: dict, G: dict, M: dict, V: dict, step: int, lr: float, beta1: float, beta2: float, eps: float):
    """One Adam step (step counts from 1), returns new (P, M, V)."""
    P2, M2, V2 = {}, {}, {}
    for name in P:
        m = beta1 * M[name] + (1.0 - beta1) * G[name]
        v = beta2 * V[name] + (1.0 - beta2) * G[name] * G[name]
        mh = m / (1.0 - beta1 ** step)
        vh = v / (1.0 - beta2 ** step)
        P2[name] = P[name] - lr * mh / (np.sqrt(vh) + eps)
        M2[name], V2[name] = m, v
    return P2, M2, V2


# ----------------------------------------------------------------------------- fallback

def residual(pred6, p_unit: np.ndarray) -> float:
    """max over channels of |a^ - a| and |b^n - b / 255| (pred given as float32)."""
    pr = np.asarray(pred6, np.float32).astype(np.float64)
    r = 0.0
    for c in range(3):
        r = max(r, abs(pr[c] - p_unit[c, 0]), abs(pr[3 + c] - p_unit[c, 1] / 255.0))
    return r


def select(pred, p_new, status, cams, tol: float):
    """Per unit (camera, side, block): use the network's prediction or the plain estimate.

    pred float32 [K*2*NB][6]; p_new, status from estimate_new.  Returns the
    chosen p_new' (same shape), used u8 [K*2*NB] and residual f32 [K*2*NB].
    Only RGB units whose three channels all hold a NEW estimate are eligible.
    """
    K, _, nb = status.shape[:3]
    tol64 = float(np.float32(tol))          # the threshold travels as float32
    out = p_new.copy()
    used = np.zeros(K * 2 * nb, np.uint8)
    res = np.full(K * 2 * nb, np.inf, np.float32)
    for k in range(K):
        if cams[k].channels != 3:
            continue
        for s in (0, 1):
            for j in range(nb):
                u = (k * 2 + s) * nb + j
                if not np.all(status[k, s, j] == NEW):
                    continue
                pr = np.asarray(pred[u], np.float32)
                if not np.all(np.isfinite(pr)):
                    continue
                r = residual(pr, p_new[k, s, j])
                res[u] = np.float32(r)
                if r <= tol64:
                    used[u] = 1
                    for c in range(3):
                        out[k, s, j, c] = (float(pr[c]), 255.0 * float(pr[3 + c]))
    return out, used, res
