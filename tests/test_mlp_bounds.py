"""CPU checks of the element-wise bars the GPU surrogate tests apply
(tests/mlp_bounds.py): a float32 forward and backward computed on the host
(numpy's float32 products, another summation order than the device's) passes
them, and each planted mistake - a dropped bias, a transposed operand, a
wrong ReLU mask, one gradient element off by 0.1 % in a region where the
gradient is small - fails them.  The last one passes a per-tensor norm check
at 1e-4, which is why the GPU tests compare element by element."""
import numpy as np
import pytest

from tests import mlp_bounds as mb


def params(rng):
    P = {"w1": rng.normal(0, 0.06, (576, 256)), "b1": rng.normal(0, 0.05, 256),
         "w2": rng.normal(0, 0.09, (256, 256)), "b2": rng.normal(0, 0.05, 256),
         "w3": rng.normal(0, 0.09, (256, 6)), "b3": rng.normal(0, 0.05, 6)}
    return {k: v.astype(np.float32) for k, v in P.items()}


def f32_forward(P, X, drop_b1=False):
    Z1 = X @ P["w1"] + (0 if drop_b1 else P["b1"])
    H1 = np.maximum(Z1, np.float32(0))
    H2 = np.maximum(H1 @ P["w2"] + P["b2"], np.float32(0))
    Y = H2 @ P["w3"] + P["b3"]
    return H1.astype(np.float32), H2.astype(np.float32), Y.astype(np.float32)


def f32_backward(P, X, H1, H2, Y, T):
    n = Y.shape[0]
    dY = (np.float32(2.0 / (n * 6)) * (Y - T)).astype(np.float32)
    dZ2 = ((dY @ P["w3"].T) * (H2 > 0)).astype(np.float32)
    dZ1 = ((dZ2 @ P["w2"].T) * (H1 > 0)).astype(np.float32)
    g = {"w3": H2.T @ dY, "b3": dY.sum(axis=0, dtype=np.float32), "w2": H1.T @ dZ2,
         "b2": dZ2.sum(axis=0, dtype=np.float32), "w1": X.T @ dZ1, "b1": dZ1.sum(axis=0, dtype=np.float32)}
    return dY, dZ2, dZ1, {k: v.astype(np.float32) for k, v in g.items()}


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(8)
    P = params(rng)
    n = 96
    X = rng.uniform(0, 2.0, (n, 576)).astype(np.float32)
    X[:, rng.integers(0, 576, 150)] = 0.0
    T = rng.normal(1.0, 0.3, (n, 6)).astype(np.float32)
    H1, H2, Y = f32_forward(P, X)
    dY, dZ2, dZ1, g = f32_backward(P, X, H1, H2, Y, T)
    return P, X, T, H1, H2, Y, dY, dZ2, dZ1, g


def test_float32_host_results_pass(case):
    P, X, T, H1, H2, Y, dY, dZ2, dZ1, g = case
    mb.check_forward_layers(P, X, H1, H2, Y)
    mb.check_forward_end_to_end(P, X, H1, H2, Y)
    mb.check_backward_layers(P, X, H1, H2, Y, T, dY, dZ2, dZ1, g)
    mb.check_backward_end_to_end(P, X, H1, H2, Y, T, g)


def test_dropped_bias_fails(case):
    P, X, T, *_ = case
    H1, H2, Y = f32_forward(P, X, drop_b1=True)
    with pytest.raises(AssertionError, match="H1"):
        mb.check_forward_end_to_end(P, X, H1, H2, Y)


def test_transposed_operand_fails(case):
    P, X, T, H1, H2, Y, dY, dZ2, dZ1, g = case
    bad = dict(g)
    bad["w2"] = g["w2"].T.copy()
    with pytest.raises(AssertionError, match="grad w2"):
        mb.check_backward_end_to_end(P, X, H1, H2, Y, T, bad)


def test_wrong_mask_fails(case):
    P, X, T, H1, H2, Y, dY, dZ2, dZ1, g = case
    wrong = ((dY @ P["w3"].T) * (H1 > 0)).astype(np.float32)      # mask of the other layer
    with pytest.raises(AssertionError, match="dZ2"):
        mb.check_backward_layers(P, X, H1, H2, Y, T, dY, wrong, dZ1, g)


def test_one_small_gradient_element_off_fails_but_passes_a_norm_check(case):
    P, X, T, H1, H2, Y, dY, dZ2, dZ1, g = case
    ref = mb.backward_ref(P, X, H1, H2, Y, T)[3]["w1"]
    mag = np.abs(ref)
    i = tuple(int(v) for v in np.argwhere(mag > np.percentile(mag[mag > 0], 5))[0])
    bad = dict(g)
    bad["w1"] = g["w1"].copy()
    bad["w1"][i] = np.float32(bad["w1"][i] * 1.001 + np.sign(ref[i]) * 1e-3 * np.abs(ref).max() * 1e-2)
    rel = np.linalg.norm(bad["w1"].astype(np.float64) - ref) / np.linalg.norm(ref)
    assert rel < 1e-4                              # a per-tensor norm check would not see it
    with pytest.raises(AssertionError, match="grad w1"):
        mb.check_backward_end_to_end(P, X, H1, H2, Y, T, bad)
