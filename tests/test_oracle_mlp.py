"""Pins of the FP64 numpy network reference used to check the warm-start kernels:
central finite differences of the loss for every weight and bias gradient, GELU and its
derivative at points where the normal distribution is tabulated, and Adam against its
closed form for a constant gradient."""
import math

import numpy as np

from oracle import mlp


def small_net(rng, dims=(6, 5, 4, 3)):
    W = [rng.normal(0, 0.5, (a, b)) for a, b in zip(dims[:-1], dims[1:])]
    b = [rng.normal(0, 0.1, d) for d in dims[1:]]
    return W, b


def test_gelu_known_values():
    """GELU(z) = z Phi(z) at points where the standard normal CDF is tabulated (Abramowitz
    and Stegun, Table 26.1; values to 16+ digits): Phi(0.5) = 0.6914624612740131,
    Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208, Phi(3) = 0.9986501019683699,
    Phi(-z) = 1 - Phi(z).  The derivative Phi(z) + z phi(z) at z = 1 and 2 uses the
    tabulated density phi(1) = 0.24197072451914337, phi(2) = 0.05399096651318806."""
    table = {-3.0: -0.0040496940948902836, -1.0: -0.15865525393145707, 0.0: 0.0,
             0.5: 0.34573123063700655, 1.0: 0.8413447460685429, 2.0: 1.9544997361036416,
             3.0: 2.9959503059051097}
    z = np.array(sorted(table))
    want = np.array([table[v] for v in z])
    got = mlp.gelu(z)
    assert np.all(np.abs(got - want) <= 4e-16 * np.maximum(1.0, np.abs(want))), got - want
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    dtab = {0.0: 0.5, 1.0: 1.0833154705876863, 2.0: 1.0852318010781969}
    zd = np.array(sorted(dtab))
    assert np.allclose(mlp.gelu_grad(zd), [dtab[v] for v in zd], rtol=0, atol=2e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    W, b = small_net(rng)
    x = rng.normal(size=(7, 6))
    y = rng.normal(size=(7, 3))

    def loss(W, b):
        out, _ = mlp.forward(x, W, b)
        return mlp.mse(out, y)[0]

    out, cache = mlp.forward(x, W, b)
    _, dout = mlp.mse(out, y)
    grads = mlp.backward(dout, W, cache)
    h = 1e-6
    for l in range(len(W)):
        for idx in [(0, 0), (1, 2), (W[l].shape[0] - 1, W[l].shape[1] - 1)]:
            Wp = [w.copy() for w in W]; Wp[l][idx] += h
            Wm = [w.copy() for w in W]; Wm[l][idx] -= h
            fd = (loss(Wp, b) - loss(Wm, b)) / (2 * h)
            assert abs(grads[l][0][idx] - fd) < 1e-7 * max(1.0, abs(fd))
        for k in [0, b[l].shape[0] - 1]:
            bp = [v.copy() for v in b]; bp[l][k] += h
            bm = [v.copy() for v in b]; bm[l][k] -= h
            fd = (loss(W, bp) - loss(W, bm)) / (2 * h)
            assert abs(grads[l][1][k] - fd) < 1e-7 * max(1.0, abs(fd))


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2, so each
    # step moves w by -lr * g / (|g| + eps)
    w = np.array([1.0, -2.0]); g = np.array([0.3, -0.7]); m = np.zeros(2); v = np.zeros(2)
    for step in range(1, 6):
        w_new, m, v = mlp.adam_step(w, g, m, v, step, lr=1e-2)
        assert np.allclose(w_new - w, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        w = w_new


def test_bf16_rounding():
    # bf16 keeps 7 fraction bits: the spacing at 1.0 is 2^-7
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-3], np.float32)
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # halfway, ties to the even neighbour 1.0
    assert r[2] == 1.0 + 2 ** -6          # halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert r[3] == 1.0 + 2 ** -7          # above halfway rounds up
    r = r[[0, 1, 2, 4, 5]]
    assert abs(r[3] + 3.140625) < 1e-12
    assert abs(r[4] - 1e-3) / 1e-3 < 2 ** -8
