"""Evaluation of the correction around a moving object (section 4.1's
comparison of the standard correction, object removal and exponential
smoothing with 16 and 64 vertical blocks, reproduced on synthetic scenes).

The paper shows the effect as images: with the standard correction the block
next to a vehicle that has just crossed a seam is discoloured; object removal
looks natural while enough of the block remains; smoothing looks natural but
lags.  Here the same scene is rendered twice, with and without the object
(identical noise and gains), both are corrected with the same method, and the
discolouration is the mean absolute difference between the two corrected
results over the background pixels (not covered by the object in either
rendering) of the correction domains that face the seam - the seam-side half
of each of the two cameras - in the rows of the vertical blocks the object
overlaps.  Zero means the object left the background's correction untouched.

Evaluation only: no step of the correction method is computed here.
"""
from __future__ import annotations

import numpy as np


def affected_rows(height: int, n_blocks: int, y0: int, h: int) -> np.ndarray:
    """bool [height]: the rows of every vertical block (floor partition of
    the rows into n_blocks) that overlaps rows [y0, y0 + h)."""
    rows = np.zeros(height, bool)
    for j in range(n_blocks):
        a, b = j * height // n_blocks, (j + 1) * height // n_blocks
        if a < y0 + h and b > y0:
            rows[a:b] = True
    return rows


def seam_halves_mask(height: int, width_left: int, width_right: int, rows: np.ndarray):
    """Masks of the left camera's right half and the right camera's left half
    restricted to `rows`: (mask_left [H][W_left], mask_right [H][W_right])."""
    ml = np.zeros((height, width_left), bool)
    mr = np.zeros((height, width_right), bool)
    ml[:, width_left // 2:] = True
    mr[:, :width_right // 2] = True
    ml[~rows] = False
    mr[~rows] = False
    return ml, mr


def discolouration(pairs) -> float:
    """Mean absolute difference over the masked background samples.

    pairs: iterable of (in_obj, in_ref, out_obj, out_ref, mask) per camera,
    arrays [H][W][C] (mask [H][W]); a pixel counts when the mask holds and
    the two inputs are equal in every channel (the object covers neither)."""
    total, count = 0, 0
    for in_o, in_r, out_o, out_r, mask in pairs:
        bg = mask & np.all(in_o == in_r, axis=2)
        d = np.abs(out_o.astype(np.int64) - out_r.astype(np.int64))
        total += int(d[bg].sum())
        count += int(bg.sum()) * in_o.shape[2]
    return total / count if count else 0.0
