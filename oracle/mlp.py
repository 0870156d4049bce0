"""Rank-proposal network and randomized residual check (oracle; test infrastructure).

Not part of the paper: the learned-proposal extension of the construction.
A two-hidden-layer perceptron maps features of one interpolative
decomposition (level, side, node and partner centres, kernel family
parameters) to a predicted rank; the proposal is then accepted or rejected by
a randomized residual test, and the plain ID of Section 2.1 is the fallback.

Everything here is plain NumPy in float64, written to be checked by eye:

* ``forward(params, X)``           -- y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3
* ``loss_and_grad(params, X, y)``  -- L = mean((f(x) - y)^2) / 2 and dL/dparams by
                                      the chain rule, layer by layer
* ``adam_step``                    -- one Adam update (Kingma & Ba, 2015)
* ``residual_ok``                  -- the acceptance test of a proposed ID
* ``splitmix64``                   -- Vigna's SplitMix64 output function, the
                                      counter-based generator both sides use for
                                      the check rows and the minibatch order

Parameter layout (one flat float vector, the same order as the GPU's):
W1 (n_in x H, row-major), b1 (H), W2 (H x H), b2 (H), W3 (H), b3 (1).
Pins: tests/test_oracle_mlp.py (central differences, closed forms, the Adam
recurrence written out for a scalar, SplitMix64 reference outputs).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def n_params(n_in: int, hidden: int) -> int:
    return n_in * hidden + hidden + hidden * hidden + hidden + hidden + 1


def unpack(params, n_in: int, hidden: int):
    p = np.asarray(params, dtype=np.float64)
    if p.size != n_params(n_in, hidden):
        raise ValueError("parameter vector has the wrong length")
    o = 0
    W1 = p[o:o + n_in * hidden].reshape(n_in, hidden); o += n_in * hidden
    b1 = p[o:o + hidden]; o += hidden
    W2 = p[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = p[o:o + hidden]; o += hidden
    W3 = p[o:o + hidden]; o += hidden
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def init_params(n_in: int, hidden: int, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float64; cast by the caller)."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (n_in, hidden)) * np.sqrt(6.0 / n_in), np.zeros(hidden),
             rng.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden), np.zeros(hidden),
             rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden), np.zeros(1)]
    return np.concatenate([x.ravel() for x in parts])


def forward(params, X, n_in: int, hidden: int) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, hidden)
    X = np.asarray(X, dtype=np.float64).reshape(-1, n_in)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def loss_and_grad(params, X, y, n_in: int, hidden: int):
    """Mean squared error / 2 over the rows of X and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, hidden)
    X = np.asarray(X, dtype=np.float64).reshape(-1, n_in)
    y = np.asarray(y, dtype=np.float64).ravel()
    n = X.shape[0]
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3
    r = out - y
    loss = 0.5 * np.mean(r * r)
    d_out = r / n                       # dL/d out
    gW3 = h2.T @ d_out
    gb3 = np.sum(d_out)
    d_h2 = np.outer(d_out, W3)
    d_z2 = d_h2 * (z2 > 0.0)
    gW2 = h1.T @ d_z2
    gb2 = d_z2.sum(axis=0)
    d_h1 = d_z2 @ W2.T
    d_z1 = d_h1 * (z1 > 0.0)
    gW1 = X.T @ d_z1
    gb1 = d_z1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def adam_step(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update; returns (params, m, v).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Vigna): the state is advanced by the
    golden-ratio increment, then mixed."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def check_positions(seed: int, level: int, side: int, q: int, n_allowed: int, r: int = 8) -> np.ndarray:
    """Positions (in the allowed set) of the r check rows of ID q: the high 32
    bits of splitmix64 of a counter built from (seed, level, side, q, i),
    scaled to [0, n_allowed)."""
    out = np.empty(r, dtype=np.int64)
    base = ((seed & 0xFFFFFFFF) << 32) ^ (level << 24) ^ (side << 23) ^ q
    for i in range(r):
        z = splitmix64((base * 16 + i) & MASK64)
        out[i] = ((z >> 32) * n_allowed) >> 32
    return out


def residual_ok(A_rows, skelpos, redpos, T, tol: float, factor: float = 1.0) -> bool:
    """Acceptance of a proposed ID on check rows A_rows (r x c):
    || A(:, red) - A(:, skel) T ||_F <= factor * tol * || A ||_F
    (factor 1 by default: the ID's own tolerance on the check rows)."""
    A_rows = np.asarray(A_rows)
    E = A_rows[:, redpos] - A_rows[:, skelpos] @ T
    return bool(np.linalg.norm(E) <= factor * tol * np.linalg.norm(A_rows))
