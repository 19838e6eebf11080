"""Element-wise bars for float32 results of the surrogate network against the
binary64 oracle.

Every float32 value the device produces for the network is a sum of K
products (plus a bias) of float32 inputs.  Whatever the summation order (the
tile kernels split K over waves and add the partial tiles in LDS), such a
sum computed in float32 differs from the exact one by at most
gamma_{K+1} * (sum |a_i b_i| + |bias|), gamma_n = n u / (1 - n u) with
u = 2^-24 (the classical rounding-error bound of a floating-point dot
product).  A result passes when

    |device - reference| <= 1e-4 |reference| + floor

element by element: 1e-4 relative is the parameter bar of the method, and
the floor is that rounding bound, carried through the layers when the
reference starts from the oracle's own binary64 activations (an input that
is off by e contributes at most e |W| to a product, and ReLU and the fixed
masks do not enlarge a difference).  The bounds are computed in binary64.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24    # unit roundoff of float32
REL = 1e-4          # relative part of the bar


def gamma(n: int) -> float:
    return n * U32 / (1.0 - n * U32)


def f64(a) -> np.ndarray:
    return np.asarray(a, np.float64)


def check(name: str, got, ref, floor) -> None:
    """|got - ref| <= REL |ref| + floor for every element."""
    g, r = f64(got), f64(ref)
    assert g.shape == r.shape, (name, g.shape, r.shape)
    assert np.all(np.isfinite(g)), f"{name}: non-finite values"
    lim = REL * np.abs(r) + f64(floor)
    bad = np.abs(g - r) > lim
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        raise AssertionError(f"{name}: {int(bad.sum())} of {bad.size} elements outside the bar; first at {list(i)}: "
                             f"device {g[i]!r} reference {r[i]!r} bar {lim[i]!r}")


def product_floor(A, B, bias=None) -> np.ndarray:
    """Rounding bound of the float32 product A B (+ bias), K = A.shape[1]."""
    A, B = np.abs(f64(A)), np.abs(f64(B))
    s = A @ B
    if bias is not None:
        s = s + np.abs(f64(bias))
    return gamma(A.shape[1] + 1) * s


def forward_ref(P, X):
    """Binary64 forward with the pre-activations (oracle arithmetic, ReLU)."""
    X = f64(X)
    Z1 = X @ f64(P["w1"]) + f64(P["b1"])
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ f64(P["w2"]) + f64(P["b2"])
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ f64(P["w3"]) + f64(P["b3"])
    return H1, H2, Y


def check_forward_layers(P, X, H1, H2, Y) -> None:
    """Each layer of the device's forward from the device's own input to it."""
    X, H1g, H2g = f64(X), f64(H1), f64(H2)
    r1 = np.maximum(X @ f64(P["w1"]) + f64(P["b1"]), 0.0)
    check("H1 (layer)", H1, r1, product_floor(X, P["w1"], P["b1"]))
    r2 = np.maximum(H1g @ f64(P["w2"]) + f64(P["b2"]), 0.0)
    check("H2 (layer)", H2, r2, product_floor(H1g, P["w2"], P["b2"]))
    r3 = H2g @ f64(P["w3"]) + f64(P["b3"])
    check("Y (layer)", Y, r3, product_floor(H2g, P["w3"], P["b3"]))


def check_forward_end_to_end(P, X, H1, H2, Y) -> None:
    """The device's activations against the oracle's binary64 forward from X,
    with the rounding bound of every earlier layer carried through."""
    H1o, H2o, Yo = forward_ref(P, X)
    W2, W3 = np.abs(f64(P["w2"])), np.abs(f64(P["w3"]))
    F1 = product_floor(X, P["w1"], P["b1"])
    check("H1", H1, H1o, F1)
    F2 = product_floor(H1o + F1, P["w2"], P["b2"]) + F1 @ W2
    check("H2", H2, H2o, F2)
    FY = product_floor(H2o + F2, P["w3"], P["b3"]) + F2 @ W3
    check("Y", Y, Yo, FY)


def backward_ref(P, X, H1, H2, Y, T):
    """Binary64 backward of the mean squared error from the given forward
    activations (the masks are the activations' own, H > 0)."""
    X, H1, H2, Y, T = f64(X), f64(H1), f64(H2), f64(Y), f64(T)
    n, out = Y.shape
    dY = 2.0 * (Y - T) / (n * out)
    dZ2 = (dY @ f64(P["w3"]).T) * (H2 > 0)
    dZ1 = (dZ2 @ f64(P["w2"]).T) * (H1 > 0)
    g = {"w3": H2.T @ dY, "b3": dY.sum(axis=0), "w2": H1.T @ dZ2, "b2": dZ2.sum(axis=0),
         "w1": X.T @ dZ1, "b1": dZ1.sum(axis=0)}
    return dY, dZ2, dZ1, g


def check_backward_layers(P, X, H1, H2, Y, T, dY, dZ2, dZ1, grads) -> None:
    """Each product of the device's backward from the device's own inputs to it."""
    X, H1, H2, Y, T = f64(X), f64(H1), f64(H2), f64(Y), f64(T)
    dYg, dZ2g, dZ1g = f64(dY), f64(dZ2), f64(dZ1)
    n, out = Y.shape
    c = 2.0 / (n * out)
    check("dY (layer)", dYg, c * (Y - T), gamma(3) * c * (np.abs(Y) + np.abs(T)))
    m2, m1 = (H2 > 0), (H1 > 0)
    check("dZ2 (layer)", dZ2g, (dYg @ f64(P["w3"]).T) * m2, product_floor(dYg, f64(P["w3"]).T) * m2)
    check("dZ1 (layer)", dZ1g, (dZ2g @ f64(P["w2"]).T) * m1, product_floor(dZ2g, f64(P["w2"]).T) * m1)
    ones = np.ones((1, n))
    for name, A, D in (("w3", H2, dYg), ("w2", H1, dZ2g), ("w1", X, dZ1g)):
        check(f"grad {name} (layer)", grads[name], A.T @ D, product_floor(A.T, D))
        b = "b" + name[1]
        check(f"grad {b} (layer)", grads[b], (ones @ D)[0], product_floor(ones, D)[0])


def check_backward_end_to_end(P, X, H1, H2, Y, T, grads) -> None:
    """Every gradient against the oracle's binary64 backward evaluated at the
    device's forward activations (so that both take the same ReLU masks), with
    the rounding bound of every earlier product carried through."""
    X, H1, H2, Y, T = f64(X), f64(H1), f64(H2), f64(Y), f64(T)
    dY, dZ2, dZ1, g = backward_ref(P, X, H1, H2, Y, T)
    n, out = Y.shape
    c = 2.0 / (n * out)
    W2T, W3T = f64(P["w2"]).T, f64(P["w3"]).T
    FdY = gamma(3) * c * (np.abs(Y) + np.abs(T))
    FdZ2 = (product_floor(np.abs(dY) + FdY, W3T) + FdY @ np.abs(W3T)) * (H2 > 0)
    FdZ1 = (product_floor(np.abs(dZ2) + FdZ2, W2T) + FdZ2 @ np.abs(W2T)) * (H1 > 0)
    ones = np.ones((1, n))
    for name, A, D, FD in (("w3", H2, dY, FdY), ("w2", H1, dZ2, FdZ2), ("w1", X, dZ1, FdZ1)):
        check(f"grad {name}", grads[name], g[name], product_floor(A.T, np.abs(D) + FD) + np.abs(A.T) @ FD)
        b = "b" + name[1]
        check(f"grad {b}", grads[b], g[b], (product_floor(ones, np.abs(D) + FD) + ones @ FD)[0])
