"""FP64 reference of the rank-selector MLP (test infrastructure only).

Network: x (F) -> h1 = relu(W1 x + b1) (H) -> h2 = relu(W2 h1 + b2) (H)
-> z = W3 h2 + b3 (R outputs).  The outputs regress the truncation errors
of an interaction at ranks 1..R (targets t); loss = mean over samples and
outputs of (z - t)^2.  Gradients written out by the chain rule (no
autograd); Adam with bias correction (Kingma & Ba, 2015).  Rank rule: the
smallest rank whose predicted error is at most a threshold, else the
maximum rank.

Weights are stored row-major as W[out][in]; a flat parameter vector is the
concatenation W1, b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import numpy as np


def shapes(F: int, H: int, R: int):
    return [(H, F), (H,), (H, H), (H,), (R, H), (R,)]


def unflatten(theta: np.ndarray, F: int, H: int, R: int):
    out, k = [], 0
    for s in shapes(F, H, R):
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    return out


def nparams(F: int, H: int, R: int) -> int:
    return sum(int(np.prod(s)) for s in shapes(F, H, R))


def forward(theta, X, F, H, R):
    W1, b1, W2, b2, W3, b3 = unflatten(np.asarray(theta, np.float64), F, H, R)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (a1, h1, a2, h2)


def loss_and_grad(theta, X, T, F, H, R):
    """Mean squared error over all samples and outputs, and its flat gradient."""
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    n = X.shape[0]
    W1, b1, W2, b2, W3, b3 = unflatten(np.asarray(theta, np.float64), F, H, R)
    z, (a1, h1, a2, h2) = forward(theta, X, F, H, R)
    d = z - T
    loss = float(np.mean(d * d))
    dz = 2.0 * d / (n * R)
    gW3 = dz.T @ h2
    gb3 = dz.sum(0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    gW1 = da1.T @ X
    gb1 = da1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new theta, m, v."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def rank_rule(z, thr: float, lmax: int):
    """rank = 1 + (first output index c with z[c] <= thr), capped at lmax; lmax
    when no output qualifies."""
    z = np.asarray(z, np.float64)
    ok = z <= thr
    r = np.where(ok.any(1), np.argmax(ok, axis=1) + 1, lmax)
    return np.minimum(r, lmax)
