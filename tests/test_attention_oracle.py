"""Pins of the oracle's difference approach (section 3.3, attention
mechanisms): on-pixels of the thresholded frame difference, counts per cell
and per sliding window, selected windows.  Independent checks: pure-Python
loops on tiny frames, the threshold boundary and its bit-depth scaling, and a
moving square whose counts are known in closed form."""
import numpy as np
import pytest

from oracle import attention as at


def brute(frame, prev, bd, tau, cell, m, theta):
    H, W, C = frame.shape
    thr = tau << (bd - 8)
    on = [[max(abs(int(frame[r, x, c]) - int(prev[r, x, c])) for c in range(C)) > thr for x in range(W)]
          for r in range(H)]
    hc, wc = -(-H // cell), -(-W // cell)
    cells = [[sum(on[r][x] for r in range(i * cell, min(H, (i + 1) * cell))
                  for x in range(j * cell, min(W, (j + 1) * cell))) for j in range(wc)] for i in range(hc)]
    win = [[sum(cells[i + a][j + b] for a in range(m) for b in range(m)) for j in range(wc - m + 1)]
           for i in range(hc - m + 1)]
    return on, cells, win


@pytest.mark.parametrize("shape,C,bd,cell,m", [((7, 9), 3, 8, 2, 2), ((13, 11), 1, 8, 4, 3), ((16, 16), 1, 12, 4, 1),
                                               ((9, 20), 3, 8, 3, 4), ((5, 5), 1, 16, 8, 1), ((6, 6), 3, 8, 2, 5)])
def test_against_loops(shape, C, bd, cell, m):
    rng = np.random.default_rng([3, *shape, C, bd])
    dt = np.uint8 if bd == 8 else np.uint16
    prev = rng.integers(0, 1 << bd, (*shape, C)).astype(dt)
    step = rng.integers(-60 << (bd - 8), (60 << (bd - 8)) + 1, (*shape, C))
    frame = np.clip(prev.astype(np.int64) + step * (rng.random((*shape, 1)) < 0.4), 0, (1 << bd) - 1).astype(dt)
    r = at.attention(frame, prev, bd, 20, cell, m, 3)
    on, cells, win = brute(frame, prev, bd, 20, cell, m, 3)
    assert np.array_equal(r["on"], np.array(on, bool))
    assert np.array_equal(r["cells"], np.array(cells, np.int64).reshape(r["cells"].shape))
    assert np.array_equal(r["windows"], np.array(win, np.int64).reshape(r["windows"].shape))
    assert np.array_equal(r["selected"], r["windows"] > 3)


def test_threshold_boundary_and_bit_depth():
    prev = np.full((1, 4, 3), 100, np.uint8)
    frame = prev.copy()
    frame[0, 0, 1] = 120      # difference 20 = tau: off
    frame[0, 1, 2] = 121      # 21: on
    frame[0, 2, 0] = 79       # 21 down: on
    assert at.on_pixels(frame, prev, 8, 20).tolist() == [[False, True, True, False]]
    p16 = np.full((1, 2, 1), 30000, np.uint16)
    f16 = p16.copy()
    f16[0, 0, 0] = 30000 + (20 << 8)         # exactly tau at 16 bits: off
    f16[0, 1, 0] = 30000 + (20 << 8) + 1
    assert at.on_pixels(f16, p16, 16, 20).tolist() == [[False, True]]


def test_moving_square_closed_form():
    """A bright 24x24 square moves 8 px to the right on a flat grey frame:
    the on-pixels are the two 24x8 strips it uncovers and covers."""
    H, W = 64, 96
    prev = np.full((H, W, 3), 60, np.uint8)
    frame = prev.copy()
    prev[16:40, 32:56] = 220
    frame[16:40, 40:64] = 220
    r = at.attention(frame, prev, 8, 20, 8, 2, 100)
    assert int(r["on"].sum()) == 2 * 24 * 8
    cells = r["cells"]
    assert cells.shape == (8, 12)
    # strips: columns 32..39 (cell column 4) and 56..63 (cell column 7), rows 16..39 (cell rows 2..4)
    expect = np.zeros((8, 12), np.int64)
    expect[2:5, 4] = 64
    expect[2:5, 7] = 64
    assert np.array_equal(cells, expect)
    # 2x2-cell windows: a window holds one strip column over two cell rows at most
    assert r["windows"].max() == 128 and int((r["windows"] > 100).sum()) == 2 * 2 * 2


def test_window_larger_than_grid_is_empty():
    on = np.ones((10, 10), bool)
    assert at.window_counts(at.cell_counts(on, 4), 4).shape == (0, 0)
