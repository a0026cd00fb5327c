"""Plain FP64 numpy reference of the warm-start network (forward, backward, one Adam step).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: used by the tests to check the GPU kernels'
outputs and gradients.  It shares no code with the GPU path.

Network: x -> [W1, b1] -> GELU -> [W2, b2] -> GELU -> [W3, b3] -> GELU -> [W4, b4] -> y,
row-major activations [batch][features], weights [in][out], exact erf GELU
0.5 z (1 + erf(z / sqrt 2)), mean-squared-error loss over all outputs.
"""
from __future__ import annotations

import math

import numpy as np

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest even) and return them as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(x, weights, biases):
    """Returns (output, list of (input, pre-activation) per layer)."""
    cache = []
    a = x
    L = len(weights)
    for l, (W, b) in enumerate(zip(weights, biases)):
        z = a @ W + b
        cache.append((a, z))
        a = gelu(z) if l < L - 1 else z
    return a, cache


def mse(pred, target):
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(dout, weights, cache):
    """Gradients (dW, db) per layer for d loss / d output = dout."""
    L = len(weights)
    grads = [None] * L
    g = dout
    for l in range(L - 1, -1, -1):
        a, z = cache[l]
        dz = g * gelu_grad(z) if l < L - 1 else g
        grads[l] = (a.T @ dz, dz.sum(axis=0))
        g = dz @ weights[l].T
    return grads


def adam_step(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
