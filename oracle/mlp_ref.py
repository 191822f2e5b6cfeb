"""Reference forms of the cost-model perceptron (TEST INFRASTRUCTURE ONLY).

Plain numpy in FP64: a 3-layer perceptron x[12] -> 64 -> 64 -> 2 with ReLU
after both hidden layers and the loss L = 1/(2B) sum_{b,j} (y[b,j] -
t[b,j])^2, its gradient by the chain rule, and one Adam step (Kingma & Ba,
ICLR 2015). Parameter layout: W1[12][64], b1[64], W2[64][64], b2[64],
W3[64][2], b3[2] (row-major, W[k][j] multiplies input k into output j).

`bf16=True` mirrors the GPU's rounding points: both inputs of every matrix
product are rounded to BF16 (round to nearest even) first; the products and
sums are then exact or FP64 here (FP32 accumulation on the GPU), and the
biases, ReLU and bias gradients stay unrounded.
"""
from __future__ import annotations

import numpy as np

IN, W, OUT = 12, 64, 2
SHAPES = [("W1", (IN, W)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (W, OUT)),
          ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(a):
    """Round to BF16 (nearest even) through FP32, returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, rnd):
    return (bf16(a) @ bf16(b)) if rnd else (a @ b)


def forward(p, x, bf16_inputs=False):
    """Returns (z1, z2, y)."""
    q = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = _mm(x, q["W1"], bf16_inputs) + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _mm(h1, q["W2"], bf16_inputs) + q["b2"]
    h2 = np.maximum(z2, 0.0)
    y = _mm(h2, q["W3"], bf16_inputs) + q["b3"]
    return z1, z2, y


def loss(p, x, t, bf16_inputs=False):
    _, _, y = forward(p, x, bf16_inputs)
    return 0.5 * float(np.sum((y - np.asarray(t, dtype=np.float64)) ** 2)) / len(x)


def backward(p, x, t, bf16_inputs=False):
    """Gradient of loss() with respect to the packed parameters."""
    q = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    B = len(x)
    z1, z2, y = forward(p, x, bf16_inputs)
    h1, h2 = np.maximum(z1, 0.0), np.maximum(z2, 0.0)
    dy = (y - np.asarray(t, dtype=np.float64)) / B
    r = bf16_inputs
    g = {}
    g["W3"] = _mm(h2.T, dy, r)
    g["b3"] = dy.sum(axis=0)
    dz2 = _mm(dy, q["W3"].T, r) * (z2 > 0)
    g["W2"] = _mm(h1.T, dz2, r)
    g["b2"] = dz2.sum(axis=0)
    dz1 = _mm(dz2, q["W2"].T, r) * (z1 > 0)
    g["W1"] = _mm(x.T, dz1, r)
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed: int):
    """He-uniform weights, zero biases (FP64)."""
    g = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[0])
            d[name] = g.uniform(-lim, lim, size=shp)
        else:
            d[name] = np.zeros(shp)
    return pack(d)
