"""Float64 reference of the learned planner's network -- TEST INFRASTRUCTURE ONLY.

Network: x (IN) -> Linear(IN, H) -> GELU -> Linear(H, H) -> GELU -> Linear(H, OUT).
Weights are BF16 values (rounded from float32 master weights, round to
nearest even); activations and sums are carried in float64 here.  GELU is
the exact form x * Phi(x) with Phi the standard normal CDF.

Loss for a batch of B samples (the planner's heads):
  y[0], y[1]   : predicted log2(1 + |I|), log2(1 + |OUT|); squared error
                 against the targets, weight 1 each, averaged over B
  y[2:8]       : logits of the plan (three-way, cascade, star, star
                 cascade, oriented, S-largest); cross entropy, averaged
  y[8:11]      : logits of the share (1, 4, 16); cross entropy over the
                 samples whose share label is >= 0, divided by B
This module restates those definitions directly; it shares nothing with
the HIP kernels.  Parity of the reference itself is pinned by finite
differences and by the closed forms of GELU.
"""
from __future__ import annotations

import math

import numpy as np

IN, H, NPLAN = 100, 64, 6
PLAN0, SHARE0 = 2, 2 + NPLAN
OUT = SHARE0 + 3


def bf16_round(w32: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    b = np.ascontiguousarray(w32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32)


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(params, X):
    """params: dict W1 [H,IN], b1 [H], W2 [H,H], b2 [H], W3 [OUT,H], b3 [OUT]
    (values already BF16-rounded for the weights); X: [B, IN]."""
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], dtype=np.float64)
                              for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    z1 = X @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    y = a2 @ W3.T + b3
    return y, (X, z1, a1, z2, a2)


def _log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))


def loss(y, targets, plan_label, share_label):
    B = y.shape[0]
    t = np.asarray(targets, dtype=np.float64)
    l_reg = ((y[:, 0] - t[:, 0]) ** 2 + (y[:, 1] - t[:, 1]) ** 2).sum() / B
    lp = _log_softmax(y[:, PLAN0:SHARE0])
    l_plan = -lp[np.arange(B), plan_label].sum() / B
    m = share_label >= 0
    ls = _log_softmax(y[:, SHARE0:SHARE0 + 3])
    l_share = -ls[np.arange(B)[m], share_label[m]].sum() / B if m.any() else 0.0
    return l_reg + l_plan + l_share


def loss_grad_y(y, targets, plan_label, share_label):
    B = y.shape[0]
    g = np.zeros_like(y)
    t = np.asarray(targets, dtype=np.float64)
    g[:, 0] = 2.0 * (y[:, 0] - t[:, 0]) / B
    g[:, 1] = 2.0 * (y[:, 1] - t[:, 1]) / B
    p = np.exp(_log_softmax(y[:, PLAN0:SHARE0]))
    p[np.arange(B), plan_label] -= 1.0
    g[:, PLAN0:SHARE0] = p / B
    m = share_label >= 0
    q = np.exp(_log_softmax(y[:, SHARE0:SHARE0 + 3]))
    q[np.arange(B), np.maximum(share_label, 0)] -= 1.0
    g[:, SHARE0:SHARE0 + 3] = np.where(m[:, None], q / B, 0.0)
    return g


def backward(params, cache, gy):
    """Gradients of the loss with respect to every parameter."""
    X, z1, a1, z2, a2 = cache
    W2, W3 = (np.asarray(params[k], dtype=np.float64) for k in ("W2", "W3"))
    gW3 = gy.T @ a2
    gb3 = gy.sum(axis=0)
    dz2 = (gy @ W3) * gelu_grad(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def adamw(w, g, m, v, step, lr, wd, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW step (decoupled weight decay) on float64 copies."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
