"""Oracle for the difference approach of the attention mechanisms.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Section 3.3 lists
three attention mechanisms that decide where the detector looks; the second,
the difference approach, finds significant local changes by thresholding the
absolute difference of two consecutive frames (the same thresholded
difference that section 3.1's object removal uses), then slides a window
across the binary image and selects every window whose number of on-pixels
exceeds a threshold.  The detector itself is not part of this project.

Readings where the paper is silent:

R-on      a pixel is on when max over channels |I_t - I_{t-1}| exceeds
          tau << (bit_depth - 8), tau in 8-bit units (as R-move of the
          correction oracle).
R-cells   on-pixels are counted per cell of c x c pixels aligned to the top
          left corner; the cells of the last row and column are cut by the
          frame's border.
R-window  a window is m x m cells; windows start at every cell (stride one
          cell) and lie inside the cell grid; a window's count is the sum of
          its cells' counts and it is selected when the count exceeds theta.

Every quantity is an exact integer.
"""
from __future__ import annotations

import numpy as np

from .ringcorr import moving_mask


def on_pixels(frame: np.ndarray, prev: np.ndarray, bit_depth: int, tau: int) -> np.ndarray:
    """bool [H][W]: the thresholded frame difference (R-on)."""
    return moving_mask(frame, prev, bit_depth, tau)


def cell_counts(on: np.ndarray, cell: int) -> np.ndarray:
    """int64 [ceil(H/c)][ceil(W/c)]: on-pixels per cell (R-cells)."""
    H, W = on.shape
    hc, wc = -(-H // cell), -(-W // cell)
    pad = np.zeros((hc * cell, wc * cell), np.int64)
    pad[:H, :W] = on
    return pad.reshape(hc, cell, wc, cell).sum(axis=(1, 3))


def window_counts(cells: np.ndarray, m: int) -> np.ndarray:
    """int64 [Hc - m + 1][Wc - m + 1]: on-pixels of every window of m x m
    cells (R-window); empty when the cell grid is smaller than a window."""
    hc, wc = cells.shape
    if hc < m or wc < m:
        return np.zeros((max(hc - m + 1, 0), max(wc - m + 1, 0)), np.int64)
    out = np.zeros((hc - m + 1, wc - m + 1), np.int64)
    for dy in range(m):
        for dx in range(m):
            out += cells[dy:dy + hc - m + 1, dx:dx + wc - m + 1]
    return out


def attention(frame: np.ndarray, prev: np.ndarray, bit_depth: int, tau: int, cell: int, m: int,
              theta: int) -> dict:
    """Everything the difference approach computes for one camera."""
    on = on_pixels(frame, prev, bit_depth, tau)
    cells = cell_counts(on, cell)
    win = window_counts(cells, m)
    return dict(on=on, cells=cells, windows=win, selected=win > theta)
