"""Pins of the surrogate oracle: finite differences for every gradient, Adam
closed forms, feature structure by brute force, the split estimate against
the combined one, and the fallback rule."""
import numpy as np
import pytest

from oracle import ringcorr as rc
from oracle import surrogate as sg


def rand_params(rng, scale=0.05):
    return {"w1": rng.normal(0, scale, (sg.IN, sg.HID)), "b1": rng.normal(0, scale, sg.HID),
            "w2": rng.normal(0, scale, (sg.HID, sg.HID)), "b2": rng.normal(0, scale, sg.HID),
            "w3": rng.normal(0, scale, (sg.HID, sg.OUT)), "b3": rng.normal(0, scale, sg.OUT)}


def test_merge_and_region_features_bruteforce():
    rng = np.random.default_rng(0)
    h = rng.integers(0, 50, (3, 256))
    h[1] = 0
    f = sg.region_features(h).reshape(3, 64)
    for c in range(3):
        n = h[c].sum()
        for b in range(64):
            ref = 0.0 if n == 0 else np.float32(64 * sum(int(h[c, 4 * b + i]) for i in range(4)) / n)
            assert f[c, b] == ref
    assert abs(f[0].astype(np.float64).sum() - 64.0) < 64e-5 and np.all(f[1] == 0)
    flat = np.full((3, 256), 5, np.int64)
    assert np.all(sg.region_features(flat) == 1.0)            # a flat histogram has density 1 everywhere
    one = np.zeros((3, 256), np.int64)
    one[2, 21] = 7
    g = sg.region_features(one).reshape(3, 64)
    assert g[2, 5] == 64.0 and g.sum() == 64.0


def test_unit_feature_layout_and_facing():
    cams = [rc.Camera(16, 8, pos=p) for p in range(3)]
    opts = rc.Options(n_blocks=2, band_width=4, closed_ring=False)
    bh = np.zeros((3, 2, 2, 3, 256), np.int64)
    wh = np.zeros((3, 3, 256), np.int64)
    wh[1, :, 10] = 1                      # whole frame of camera 1 -> bin 2
    bh[1, 1, 0, :, 100] = 1               # own band -> bin 25
    bh[2, 0, 0, :, 200] = 1               # facing band (camera 2 left) -> bin 50
    x = sg.unit_features(cams, opts, bh, wh, 1, 1, 0).reshape(3, 3, 64)
    for c in range(3):
        assert x[0, c, 2] == 64 and x[1, c, 25] == 64 and x[2, c, 50] == 64
    assert x.sum() == 9 * 64
    x_end = sg.unit_features(cams, opts, bh, wh, 2, 1, 0).reshape(3, 3, 64)   # open chain end: no facing band
    assert np.all(x_end[2] == 0)
    X = sg.all_features(cams + [rc.Camera(8, 8, 1, 12, ring=1)], opts, np.concatenate([bh, bh[:1]]),
                        np.concatenate([wh, wh[:1]]))
    assert X.shape == (4 * 2 * 2, 576) and np.all(X[12:] == 0)


@pytest.mark.parametrize("smoothing", [False, True])
def test_split_estimate_equals_combined(smoothing):
    rng = np.random.default_rng(5)
    cams = [rc.Camera(40, 30, pos=p) for p in range(3)] + [rc.Camera(20, 10, 1, 12, ring=4, pos=0)]
    opts = rc.Options(n_blocks=4, band_width=5, smoothing=smoothing, closed_ring=True)
    prev_p = rng.uniform(0.5, 2, (4, 2, 4, 3, 2))
    prev_v = rng.integers(0, 2, (4, 2, 4, 3)).astype(np.uint8)
    sums = np.zeros((4, 2, 4, 3, 3), np.int64)
    for idx in np.ndindex(4, 2, 4, 3):
        n = int(rng.integers(0, 4)) * 5
        v = rng.integers(0, 256, n)
        sums[idx] = (n, v.sum(), (v * v).sum())
    ref_p, ref_v = rc.estimate(cams, opts, sums, prev_p, prev_v)
    p_new, st = sg.estimate_new(cams, opts, sums)
    got_p, got_v = sg.temporal(opts, p_new, st, prev_p, prev_v)
    assert np.array_equal(got_p.view(np.uint64), ref_p.view(np.uint64)) and np.array_equal(got_v, ref_v)


def test_gradients_against_central_differences():
    rng = np.random.default_rng(1)
    P = rand_params(rng)
    X = rng.uniform(0, 0.1, (8, sg.IN))
    T = rng.normal(0, 1, (8, sg.OUT))
    Y, H1, H2 = sg.forward(P, X)
    G = sg.backward(P, X, H1, H2, Y, T)
    h = 1e-6
    for name, arr in P.items():
        for _ in range(6):
            idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
            old = arr[idx]
            arr[idx] = old + h
            lp = sg.mse(sg.forward(P, X)[0], T)
            arr[idx] = old - h
            lm = sg.mse(sg.forward(P, X)[0], T)
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, G[name][idx])


def test_forward_bruteforce_one_sample():
    rng = np.random.default_rng(2)
    P = rand_params(rng, 0.1)
    x = rng.uniform(0, 0.2, sg.IN)
    Y, _, _ = sg.forward(P, x[None, :])
    h1 = [max(0.0, sum(x[i] * P["w1"][i, j] for i in range(sg.IN)) + P["b1"][j]) for j in range(sg.HID)]
    h2 = [max(0.0, sum(h1[i] * P["w2"][i, j] for i in range(sg.HID)) + P["b2"][j]) for j in range(sg.HID)]
    y = [sum(h2[i] * P["w3"][i, o] for i in range(sg.HID)) + P["b3"][o] for o in range(sg.OUT)]
    assert np.allclose(Y[0], y, rtol=1e-12, atol=1e-12)


def test_mse_and_adam_closed_forms():
    Y = np.array([[1.0, 2, 3, 4, 5, 6]])
    T = np.zeros((1, 6))
    assert sg.mse(Y, T) == (1 + 4 + 9 + 16 + 25 + 36) / 6
    P = {"w": np.array([1.0, -2.0, 3.0])}
    G = {"w": np.array([0.5, -4.0, 0.0])}
    M = {"w": np.zeros(3)}
    V = {"w": np.zeros(3)}
    lr, eps = 1e-3, 1e-8
    P1, M1, V1 = sg.adam(P, G, M, V, 1, lr, 0.9, 0.999, eps)
    assert np.allclose(P1["w"], P["w"] - lr * G["w"] / (np.abs(G["w"]) + eps), rtol=0, atol=1e-15)
    P2, _, _ = sg.adam(P1, G, M1, V1, 2, lr, 0.9, 0.999, eps)      # constant gradient: same step again
    assert np.allclose(P2["w"], P1["w"] - lr * G["w"] / (np.abs(G["w"]) + eps), rtol=0, atol=1e-12)


def test_select_rule():
    cams = [rc.Camera(8, 8, pos=0), rc.Camera(8, 8, pos=1), rc.Camera(8, 8, 1, 12, ring=3)]
    nb = 1
    p_new = np.zeros((3, 2, nb, 3, 2))
    p_new[..., 0] = 1.25
    p_new[..., 1] = 12.75
    st = np.full((3, 2, nb, 3), sg.NEW, np.int32)
    st[1, 1, 0, 2] = sg.NONE                       # one channel without an estimate
    exact = np.array([1.25, 1.25, 1.25, 0.05, 0.05, 0.05], np.float32)
    pred = np.tile(exact, (3 * 2 * nb, 1))
    pred[1] = exact + np.float32(2e-3)             # camera 0 right: residual 2e-3 > tol
    pred[2, 4] = np.nan                            # camera 1 left: not finite
    out, used, res = sg.select(pred, p_new, st, cams, 1e-3)
    assert list(used) == [1, 0, 0, 0, 0, 0]
    assert res[0] == np.float32(abs(np.float64(np.float32(0.05)) - 0.05))
    assert out[0, 0, 0, 0, 1] == 255.0 * float(np.float32(0.05)) and out[0, 1, 0, 0, 1] == 12.75
    edge = pred.copy()
    edge[0, 0] = np.float32(1.25) + np.float32(9.5367431640625e-4)   # residual just under 1e-3 -> used
    assert sg.select(edge, p_new, st, cams, 1e-3)[1][0] == 1


def test_targets_order_and_scale_hand_cases():
    """Hand-worked: the unit's [channel][a, b] parameters become (a_R, a_G,
    a_B, b_R/255, b_G/255, b_B/255), gains first in channel order, offsets
    in grey levels divided by 255."""
    p = np.array([[1.5, 51.0], [2.0, -25.5], [0.5, 255.0]])
    assert sg.targets(p).tolist() == [1.5, 2.0, 0.5, 0.2, -0.1, 1.0]
    q = np.array([[1.0, 0.0], [1.0, 0.0], [1.0, 0.0]])
    assert sg.targets(q).tolist() == [1.0, 1.0, 1.0, 0.0, 0.0, 0.0]
    r = np.array([[0.125, -12.75], [8.0, 25.5], [3.0, 127.5]])       # offsets exact in binary
    assert sg.targets(r).tolist() == [0.125, 8.0, 3.0, -0.05, 0.1, 0.5]


def test_targets_of_known_gains():
    """Closed form: a seam whose two bands are one scene under gains gP and
    gQ = 2 gP (integer samples, no clipping) has a_P = 1.5 and b_P = 0 in
    every channel, so the own unit's target is (1.5, 1.5, 1.5, 0, 0, 0) and
    the facing unit's (0.75, 0.75, 0.75, 0, 0, 0) - with the offset term
    unscaled by 255 this would not tell them apart, with the order swapped
    the first three would be 0."""
    rng = np.random.default_rng(11)
    s = rng.integers(16, 97, (16, 8, 3)).astype(np.int64)
    cams = [rc.Camera(16, 16, pos=0), rc.Camera(16, 16, pos=1)]
    opts = rc.Options(n_blocks=1, band_width=8, closed_ring=False)
    frames = [np.zeros((16, 16, 3), np.uint8) for _ in range(2)]
    frames[0][:, 8:] = s.astype(np.uint8)           # right band of camera 0
    frames[1][:, :8] = (2 * s).astype(np.uint8)     # left band of camera 1 (facing it)
    bs = np.stack([rc.band_stats(f, c, opts)[1] for f, c in zip(frames, cams)])
    p_new, st = sg.estimate_new(cams, opts, bs)
    assert np.all(st[0, 1, 0] == sg.NEW) and np.all(st[1, 0, 0] == sg.NEW)
    t_own = sg.targets(p_new[0, 1, 0])
    t_fac = sg.targets(p_new[1, 0, 0])
    assert np.allclose(t_own, [1.5, 1.5, 1.5, 0, 0, 0], rtol=0, atol=1e-12)
    assert np.allclose(t_fac, [0.75, 0.75, 0.75, 0, 0, 0], rtol=0, atol=1e-12)


def test_targets_as_prediction_have_zero_residual_and_restore_the_estimate():
    """A network that outputs exactly the targets (as float32) is within the
    float32 rounding of the plain estimate under the fallback rule's residual,
    and a used prediction gives back (a, 255 b/255) of the estimate."""
    rng = np.random.default_rng(12)
    cams = [rc.Camera(8, 8, pos=0), rc.Camera(8, 8, pos=1)]
    p_new = np.zeros((2, 2, 1, 3, 2))
    p_new[..., 0] = rng.uniform(0.5, 2.0, (2, 2, 1, 3))
    p_new[..., 1] = rng.uniform(-40.0, 40.0, (2, 2, 1, 3))
    st = np.full((2, 2, 1, 3), sg.NEW, np.int32)
    pred = np.array([sg.targets(p_new[k, s, 0]) for k in range(2) for s in range(2)], np.float32)
    for u in range(4):
        k, s = divmod(u, 2)
        r = sg.residual(pred[u], p_new[k, s, 0])
        assert r <= 2.0 ** -23 * 4            # one float32 rounding of values below 4 in magnitude
    out, used, _ = sg.select(pred, p_new, st, cams, 1e-6)
    assert used.tolist() == [1, 1, 1, 1]
    assert np.allclose(out[..., 0], p_new[..., 0], rtol=2.0 ** -23, atol=0)
    assert np.allclose(out[..., 1], p_new[..., 1], rtol=0, atol=255 * 2.0 ** -24 * 1.0)
