"""Pins for the float64 reference of the planner network: GELU against
closed forms and math.erf, gradients against finite differences, AdamW
against its definition on a scalar problem."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M


def rand_params(rng, scale=0.3):
    return {"W1": rng.normal(0, scale, (M.H, M.IN)), "b1": rng.normal(0, 0.1, M.H),
            "W2": rng.normal(0, scale, (M.H, M.H)), "b2": rng.normal(0, 0.1, M.H),
            "W3": rng.normal(0, scale, (M.OUT, M.H)), "b3": rng.normal(0, 0.1, M.OUT)}


def test_gelu_closed_forms():
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert M.gelu(np.array([10.0]))[0] == pytest.approx(10.0, rel=1e-15)
    x = np.linspace(-4, 4, 81)
    h = 1e-6
    num = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), num, rtol=1e-7, atol=1e-9)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265], dtype=np.float32)
    r = M.bf16_round(v)
    np.testing.assert_array_equal(r[:3], np.array([1.0, 1.0, 1.0 + 2 ** -6], dtype=np.float32))
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-7


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = rand_params(rng)
    B = 9
    X = rng.normal(0, 1, (B, M.IN))
    t = rng.normal(5, 2, (B, 2))
    pl = rng.integers(0, M.NPLAN, B)
    sl = rng.integers(-1, 3, B)
    y, cache = M.forward(p, X)
    g = M.backward(p, cache, M.loss_grad_y(y, t, pl, sl))
    # central differences: truncation error O(eps^2), rounding error about
    # 1e-16 * |loss| / eps; eps = 1e-5 keeps both below 1e-6 of a gradient
    eps = 1e-5
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = M.loss(M.forward(p, X)[0], t, pl, sl)
            flat[idx] = old - eps
            lm = M.loss(M.forward(p, X)[0], t, pl, sl)
            flat[idx] = old
            num = (lp - lm) / (2 * eps)
            assert g[name].reshape(-1)[idx] == pytest.approx(num, rel=1e-5, abs=1e-8), (name, idx)


def test_adamw_scalar():
    # minimise (w - 3)^2 with AdamW without decay: converges to 3
    w, m, v = np.array([0.0]), np.array([0.0]), np.array([0.0])
    for step in range(1, 3001):
        w, m, v = M.adamw(w, 2 * (w - 3), m, v, step, lr=0.01, wd=0.0)
    assert abs(w[0] - 3) < 1e-3
    # first step moves by lr * sign(g) exactly (bias-corrected)
    w1, _, _ = M.adamw(np.array([1.0]), np.array([5.0]), np.zeros(1), np.zeros(1), 1, lr=0.1, wd=0.0)
    assert w1[0] == pytest.approx(0.9, abs=1e-7)
