"""FP64 oracle for the learned closure (features, MLP forward/backward, Adam, fallback).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The paper contains no machine learning; everything
here follows the interface chosen for the learned closure, whose readings are:

* inputs (14): g = Delta * G (G_ij = d_j ut_i, 9 components, row-major) and five
  invariants of g with s = (g + g^T)/2, r = (g - g^T)/2:
  tr(s^2), tr(r^2), tr(s^3), tr(s r^2), tr(s^2 r^2). Scaling G by the filter width makes
  the inputs comparable across grids and widths.
* target (6): tau_c / rho_bar for c in xx xy xz yy yz zz.
* network 14 -> 64 -> 64 -> 64 -> 6, GELU (tanh form) after the three hidden layers.
* BF16 round-to-nearest-even is applied where the GPU feeds the matrix cores: layer
  inputs, weights and the upstream gradients of each backward product; accumulation,
  biases, GELU and Adam stay in higher precision (FP64 here).
* loss: mean squared error over batch and the 6 standardised outputs.

Parameter packing (9670 floats): W1 (64x14), b1, W2 (64x64), b2, W3 (64x64), b3,
W4 (6x64), b4, each W row-major (out, in).
"""
from __future__ import annotations

import math

import numpy as np

SIZES = (14, 64, 64, 64, 6)
N_PARAMS = sum(SIZES[i] * SIZES[i + 1] + SIZES[i + 1] for i in range(4))
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.

    The value is first taken to FP32 (the GPU's operand type), then its low 16 bits are
    rounded away: add 0x7FFF plus the lowest kept bit, then clear the low half.
    """
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = rounded.view(np.float32).astype(np.float64)
    # NaN stays NaN (the rounding above could carry a NaN payload into Inf)
    return np.where(np.isnan(f), np.nan, out)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    out, o = [], 0
    for l in range(4):
        fi, fo = SIZES[l], SIZES[l + 1]
        W = p[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = p[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for (W, b) in layers])


def init_params(seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, numpy PCG64 seed."""
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(4):
        fi, fo = SIZES[l], SIZES[l + 1]
        bound = 1.0 / math.sqrt(fi)
        layers.append((rng.uniform(-bound, bound, (fo, fi)), rng.uniform(-bound, bound, fo)))
    return pack(layers).astype(np.float32)


def gelu(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * x * (1.0 + t)


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


# --------------------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------------------
def features_from_grad(G, delta: float):
    """G: (..., 3, 3) with G[..., i, j] = d_j ut_i. Returns (..., 14)."""
    g = np.asarray(G, dtype=np.float64) * delta
    gt = np.swapaxes(g, -1, -2)
    s = 0.5 * (g + gt)
    r = 0.5 * (g - gt)
    ss = s @ s
    rr = r @ r
    tr = lambda a: np.trace(a, axis1=-2, axis2=-1)
    inv = np.stack([tr(ss), tr(rr), tr(ss @ s), tr(s @ rr), tr(ss @ rr)], axis=-1)
    return np.concatenate([g.reshape(g.shape[:-2] + (9,)), inv], axis=-1)


def targets_from_tau(tau6, rho_bar):
    """tau6: (..., 6) in order xx xy xz yy yz zz; returns tau / rho_bar."""
    return np.asarray(tau6, dtype=np.float64) / np.asarray(rho_bar, dtype=np.float64)[..., None]


def norm_stats(X):
    """Per-column mean and population standard deviation (two-pass, FP64)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    return mu, sd


# --------------------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------------------
def forward(params, x_std, bf16=True):
    """Forward pass with BF16 operand rounding (bf16=False: exact FP64). Returns (y, cache)."""
    q = bf16_round if bf16 else (lambda t: np.asarray(t, dtype=np.float64))
    layers = unpack(params)
    a = q(x_std)
    cache = {"a": [a], "z": []}
    for l, (W, b) in enumerate(layers):
        z = a @ q(W).T + b
        cache["z"].append(z)
        if l < 3:
            a = q(gelu(z))
            cache["a"].append(a)
        else:
            y = z
    return y, cache


def loss_and_grads(params, x_std, y_std, bf16=True):
    """MSE over the batch and 6 outputs, and its gradient with respect to every parameter."""
    q = bf16_round if bf16 else (lambda t: np.asarray(t, dtype=np.float64))
    layers = unpack(params)
    y, cache = forward(params, x_std, bf16)
    B = y.shape[0]
    diff = y - y_std
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / (B * SIZES[-1])
    grads = [None] * 4
    for l in range(3, -1, -1):
        W, _ = layers[l]
        dzb = q(dz)
        dW = dzb.T @ cache["a"][l]
        db = dz.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            da = dzb @ q(W)
            dz = da * gelu_grad(cache["z"][l - 1])
    return loss, pack(grads)


def adam(params, grads, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); step counts from 1. Returns new (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grads, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def infer(params, feats, rho_bar, tau_gm6, x_mu, x_sd, y_mu, y_sd, lo, hi):
    """Learned tau (..., 6) with the plain closure as fallback outside the envelope.

    The envelope is the per-feature [lo, hi] box of standardised training inputs; a point
    with any standardised input outside it, or non-finite, takes tau_gm instead.
    Returns (tau6, fallback_mask).
    """
    xs = (np.asarray(feats, dtype=np.float64) - x_mu) / x_sd
    out_flag = ~np.all(np.isfinite(xs) & (xs >= lo) & (xs <= hi), axis=-1)
    xs_safe = np.where(np.isfinite(xs), xs, 0.0)
    y, _ = forward(params, xs_safe.reshape(-1, 14))
    y = y.reshape(xs.shape[:-1] + (6,))
    tau = np.asarray(rho_bar, dtype=np.float64)[..., None] * (y_mu + y_sd * y)
    tau = np.where(out_flag[..., None], tau_gm6, tau)
    return tau, out_flag
