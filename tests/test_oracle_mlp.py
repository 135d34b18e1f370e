"""Pins of the FP64 surrogate network oracle (CPU)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp as M


def test_gelu_values_and_derivative():
    # gelu(z) = z Phi(z): Phi(1) = 0.841344746068542948585...
    assert M.gelu(np.array(0.0)) == 0.0
    assert M.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array(-1.0)) == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert M.gelu_grad(np.array(0.0)) == pytest.approx(0.5, rel=1e-15)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), rtol=1e-8, atol=1e-9)


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e38, 1e-40])
    got = M.bf16(x)
    assert got[0] == 1.0 and got[1] == 1.0               # tie -> even (1.0)
    assert got[2] == 1 + 2 ** -6                         # tie -> even (mantissa ...10)
    assert got[3] == 1 + 2 ** -7
    assert got[4] == -2.5
    assert np.isfinite(got).all()
    # relative rounding error at most 2^-9 for normal numbers
    r = np.random.default_rng(0).normal(size=1000)
    assert np.abs(M.bf16(r) - r).max() <= 2 ** -9 * np.abs(r).max()


def _problem(batch=16, seed=3):
    params = W.mlp_init(4)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(batch, 96))
    T = rng.normal(size=(batch, 3))
    return params, X, T


def test_parameter_count_and_init_range():
    params = W.mlp_init(4)
    assert sum(p.size for p in params) == 157187
    for l in range(4):
        fi, fo = params[2 * l].shape
        assert np.abs(params[2 * l]).max() <= math.sqrt(6 / (fi + fo))


def test_gradients_match_central_differences():
    params, X, T = _problem()
    params = [p + 0.01 * np.random.default_rng(1).normal(size=p.shape) for p in params]
    loss, grads = M.loss_and_grad(params, X, T)
    rng = np.random.default_rng(2)
    h = 1e-6
    for li in range(8):
        p = params[li]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            old = p[idx]
            p[idx] = old + h
            lp = M.loss_and_grad(params, X, T)[0]
            p[idx] = old - h
            lm = M.loss_and_grad(params, X, T)[0]
            p[idx] = old
            fd = (lp - lm) / (2 * h)
            assert grads[li][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_adam_first_step_is_lr_times_sign():
    params, X, T = _problem()
    _, grads = M.loss_and_grad(params, X, T)
    before = [p.copy() for p in params]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    M.adam_step(params, grads, m, v, 1, lr=1e-3)
    for b, a, g in zip(before, params, grads):
        expect = -1e-3 * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(a - b, expect, rtol=1e-9, atol=1e-15)


def test_training_reduces_loss():
    params, X, T = _problem(batch=64)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    l0 = M.loss_and_grad(params, X, T)[0]
    for t in range(1, 101):
        loss, grads = M.loss_and_grad(params, X, T)
        M.adam_step(params, grads, m, v, t, lr=1e-3)
    assert loss < 0.2 * l0
