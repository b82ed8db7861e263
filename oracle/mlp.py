"""FP64 reference of the surrogate MLP (dense layers, exact-erf GELU hidden
activations, linear output, mean-squared-error loss) and of Adam.

TEST INFRASTRUCTURE ONLY.

Parameters are one flat vector, layer by layer: W_l [out_l, in_l] row-major
then b_l [out_l].  With ``bf16=True`` the operands of every matrix product
are rounded to bfloat16 first, exactly where the GPU rounds them (layer
inputs and weights in the forward pass; the upstream gradient and the
saved activations / weights in the backward pass); products and sums are
then FP64, so the GPU's only extra error is its FP32 accumulation.

Pinned by: central finite differences of the FP64 loss (bf16=False), and
an Adam step written from the update rule of Kingma & Ba (ICLR 2015).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import bf16_round


def shapes(n_in: int, hidden: int, layers: int, n_out: int):
    dims = [n_in] + [hidden] * layers + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def unpack(theta: np.ndarray, shp):
    out, o = [], 0
    for (r, c) in shp:
        W = theta[o:o + r * c].reshape(r, c)
        o += r * c
        b = theta[o:o + r]
        o += r
        out.append((W, b))
    assert o == len(theta)
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _r(x, bf16):
    return bf16_round(x).astype(np.float64) if bf16 else np.asarray(x, dtype=np.float64)


def forward(theta, X, shp, bf16=False):
    """Returns (Y, cache) with cache = list of (input, pre-activation)."""
    layers = unpack(np.asarray(theta, dtype=np.float64), shp)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = _r(a, bf16) @ _r(W, bf16).T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a, cache


def loss_and_grad(theta, X, T, shp, bf16=False):
    """MSE loss mean((Y - T)^2) over all entries and its gradient."""
    theta = np.asarray(theta, dtype=np.float64)
    layers = unpack(theta, shp)
    Y, cache = forward(theta, X, shp, bf16)
    B, O = Y.shape
    loss = float(np.mean((Y - T) ** 2))
    dz = 2.0 * (Y - T) / (B * O)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        a_in, _ = cache[li]
        gW = _r(dz, bf16).T @ _r(a_in, bf16)
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            _, z_prev = cache[li - 1]
            da = _r(dz, bf16) @ _r(W, bf16)
            dz = da * gelu_grad(z_prev)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
