"""Reference (float64, CPU) for the learned probe count: an extension of the
fixed probe count tau of Section 2 (Eq. 5 probes the tau nearest coarse
centroids) in which a small multilayer perceptron predicts tau per query.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the product path
never imports it.  Plain numpy in float64; every step follows the plain
definition of the network, the loss, the gradient and the Adam update.

Network (din inputs, h hidden units, one output):
    z1 = W1 x + b1,  h1 = relu(z1)
    z2 = W2 h1 + b2, h2 = relu(z2)
    yhat = w3 . h2 + b3
Loss over a batch of B rows: mean over rows of (yhat - y)^2.
Parameters are one flat vector in the order W1 (h x din, row-major), b1 (h),
W2 (h x h), b2 (h), w3 (h), b3 (1).
"""
from __future__ import annotations

import math

import numpy as np

N_DIST = 32  # coarse distances used as features


def n_params(din: int, h: int) -> int:
    return h * din + h + h * h + h + h + 1


def unpack(theta, din: int, h: int):
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (n_params(din, h),)
    o = 0
    W1 = theta[o:o + h * din].reshape(h, din); o += h * din
    b1 = theta[o:o + h]; o += h
    W2 = theta[o:o + h * h].reshape(h, h); o += h * h
    b2 = theta[o:o + h]; o += h
    w3 = theta[o:o + h]; o += h
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def forward(theta, X, din: int, h: int):
    """All intermediate values of the forward pass, float64."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, din, h)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    yhat = h2 @ w3 + b3[0]
    return z1, h1, z2, h2, yhat


def loss_and_grad(theta, X, y, din: int, h: int):
    """Mean squared error and its gradient (chain rule, float64)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, din, h)
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    B = X.shape[0]
    z1, h1, z2, h2, yhat = forward(theta, X, din, h)
    r = yhat - y
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B                    # d loss / d yhat
    g_w3 = h2.T @ dy
    g_b3 = np.array([dy.sum()])
    dz2 = np.outer(dy, w3) * (z2 > 0)   # relu passes the gradient where z > 0
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, g_b3])
    return loss, grad


def adam_step(theta, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction at step t >= 1."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(xq, coarse_dist):
    """[x ; the N_DIST smallest squared coarse distances, ascending]."""
    xq = np.asarray(xq, np.float64)
    cd = np.sort(np.asarray(coarse_dist, np.float64), axis=1)[:, :N_DIST]
    return np.concatenate([xq, cd], axis=1)


def standardization(F):
    """Column mean and standard deviation (population); zero spread -> 1."""
    F = np.asarray(F, np.float64)
    mean = F.mean(0)
    std = np.sqrt(((F - mean) ** 2).mean(0))
    std[std == 0] = 1.0
    return mean, std


def labels(nn_list, coarse_order, cap: int):
    """Probe count each query needs: the 1-based position of the list holding
    its true nearest neighbour in its coarse order (Eq. 5 sorted), at most cap
    (also when the list is not among the first cap)."""
    out = np.empty(len(nn_list), np.int64)
    for j, L in enumerate(nn_list):
        pos = np.nonzero(np.asarray(coarse_order[j])[:cap] == L)[0]
        out[j] = pos[0] + 1 if len(pos) else cap
    return out


def probe_count(yhat, delta: float, cap: int):
    """tau = clamp(ceil(2^(yhat + delta)), 1, cap) for a prediction of log2(tau)."""
    out = np.empty(len(yhat), np.int64)
    for j, v in enumerate(np.asarray(yhat, np.float64)):
        out[j] = min(max(math.ceil(2.0 ** (v + delta)), 1), cap)
    return out
