"""FP64 multilayer perceptron of the surrogate (test infrastructure).

The surrogate is not in the paper; this is the plain definition the MFMA kernels must match:
  Z1 = X W1 + b1, H1 = gelu(Z1), Z2 = H1 W2 + b2, H2 = gelu(Z2), Z3 = H2 W3 + b3,
  H3 = gelu(Z3), Y = H3 W4 + b4;  gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (exact erf);
  loss = mean over samples and outputs of (Y - T)^2;  Adam (Kingma & Ba 2015) on all weights.
``storage="bf16"`` rounds, as the device stores them, the inputs, the weights, the hidden
activations H and the back-propagated gradients dZ / dY to bfloat16 (round to nearest even),
while every sum is exact FP64 -- the device differs from it only by FP32 accumulation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = (96, 256, 256, 256, 3)


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _store(a, storage):
    return bf16(a) if storage == "bf16" else a


def forward(params, X, storage="fp64"):
    """params: [W1, b1, W2, b2, W3, b3, W4, b4]; returns (Y, cache)."""
    W = [_store(params[2 * l], storage) for l in range(4)]
    b = [params[2 * l + 1] for l in range(4)]
    H = _store(np.asarray(X, float), storage)
    cache = [H]
    for l in range(3):
        Z = H @ W[l] + b[l]
        H = _store(gelu(Z), storage)
        cache += [Z, H]
    Y = H @ W[3] + b[3]
    return Y, cache


def loss_and_grad(params, X, T, storage="fp64"):
    """MSE loss and its gradient with respect to every parameter."""
    Y, cache = forward(params, X, storage)
    B = len(X)
    diff = Y - T
    loss = float((diff * diff).mean())
    W = [_store(params[2 * l], storage) for l in range(4)]
    dY = _store(2.0 * diff / diff.size, storage)
    grads = [None] * 8
    H3 = cache[-1]
    grads[6] = H3.T @ dY
    grads[7] = dY.sum(axis=0)
    dH = dY @ W[3].T
    for l in (2, 1, 0):
        Z = cache[1 + 2 * l]
        Hin = cache[2 * l]
        dZ = _store(dH * gelu_grad(Z), storage)
        grads[2 * l] = Hin.T @ dZ
        grads[2 * l + 1] = dZ.sum(axis=0)
        if l:
            dH = dZ @ W[l].T
    return loss, grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); updates params, m, v in place."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** t)
        vhat = vv / (1.0 - beta2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
