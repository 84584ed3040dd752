"""Reference multilayer-perceptron surrogate (oracle; test infrastructure only).

Sec. 1 names machine-learning surrogates of the forward model as a way to faster
retrievals; here the surrogate maps the retrieval parameters to the standardised binned
spectrum and serves as stage 1 of delayed acceptance. Written in FP64 numpy from the
definitions: dense layers z_i = h_i W_i^T + b_i, SiLU hidden activations
silu(z) = z / (1 + e^-z), a linear output layer, the mean-squared error, back-propagation
by the chain rule, and Adam (Kingma & Ba 2015) with bias correction. ``bf16`` rounds to
the bfloat16 format (1 sign, 8 exponent, 7 fraction bits) to nearest, ties to even, from
the bit pattern of the FP32 value, so a test can feed the oracle the same BF16 operands
the matrix cores see.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Nearest bfloat16 value of FP32(x), ties to even, returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def scale_input(params, lo, hi, width: int | None = None) -> np.ndarray:
    """Parameters mapped onto [0, 1] by the prior box, zero-padded to ``width`` columns."""
    params = np.atleast_2d(np.asarray(params, np.float64))
    x = (params - lo) / (hi - lo)
    if width is not None and width > x.shape[1]:
        x = np.hstack([x, np.zeros((x.shape[0], width - x.shape[1]))])
    return x


def forward(h0, weights, biases, round_bf16: bool = False):
    """Forward pass. Returns (zs, hs, out): hs[i] is layer i's input, zs[i] its
    pre-activation; out = zs[-1]. With round_bf16 the layer inputs and weights are
    rounded to BF16 before each product (as the matrix cores consume them)."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    hs, zs = [r(h0)], []
    for i, (w, b) in enumerate(zip(weights, biases)):
        z = hs[-1] @ r(w).T + b
        zs.append(z)
        if i < len(weights) - 1:
            hs.append(r(silu(z)))
    return zs, hs, zs[-1]


def mse(out, target) -> float:
    """Mean over all elements of (out - target)^2."""
    d = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d))


def mse_grad(out, target) -> np.ndarray:
    d = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    return 2.0 * d / d.size


def backward(weights, zs, hs, dout, round_bf16: bool = False):
    """Gradients (gW, gb) of a scalar loss with d loss / d out = dout, by the chain rule
    through the linear output layer and the SiLU hidden layers. With round_bf16 the
    back-propagated gradients and the weights are rounded to BF16 before each product."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    n = len(weights)
    gw, gb = [None] * n, [None] * n
    dz = r(dout)
    for i in range(n - 1, -1, -1):
        gw[i] = dz.T @ hs[i]
        gb[i] = dz.sum(0)
        if i > 0:
            dz = r((dz @ r(weights[i])) * silu_grad(zs[i - 1]))
    return gw, gb


def adam(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (bias-corrected moments); returns the new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def surrogate_chi2(out, mean, scale, data, err) -> np.ndarray:
    """chi^2 of the unstandardised prediction mean + scale * out against the data."""
    pred = mean + scale * np.atleast_2d(np.asarray(out, np.float64))
    return np.sum(((pred - data) / err) ** 2, axis=1)
