"""Pins of the rank-proposal network and residual check of the oracle
(oracle/mlp.py) against central differences, closed forms and published
reference values."""
import numpy as np
import pytest

from oracle import mlp

NI, H = 7, 16  # small hidden width keeps the finite-difference sweep fast


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(NI, H, seed=2) + 0.05 * rng.standard_normal(mlp.n_params(NI, H))
    X = rng.standard_normal((40, NI))
    y = rng.standard_normal(40)
    _, g = mlp.loss_and_grad(p, X, y, NI, H)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (mlp.loss_and_grad(p + e, X, y, NI, H)[0] - mlp.loss_and_grad(p - e, X, y, NI, H)[0]) / (2 * h)
    assert np.linalg.norm(num - g) <= 1e-6 * np.linalg.norm(g)


def test_forward_closed_forms():
    rng = np.random.default_rng(3)
    X = np.abs(rng.standard_normal((5, NI)))
    W1, W2, W3 = (np.abs(rng.standard_normal(s)) for s in ((NI, H), (H, H), (H,)))
    b1, b2, b3 = np.abs(rng.standard_normal(H)), np.abs(rng.standard_normal(H)), 0.7
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])
    # all pre-activations positive: the network is the affine map composed by hand
    expect = ((X @ W1 + b1) @ W2 + b2) @ W3 + b3
    assert np.allclose(mlp.forward(p, X, NI, H), expect, rtol=1e-14)
    # W2 = 0, b2 = 0: the output is the bias alone, whatever the input
    p0 = np.concatenate([W1.ravel(), b1, np.zeros(H * H), np.zeros(H), W3, [b3]])
    assert np.all(mlp.forward(p0, X, NI, H) == b3)


def test_adam_first_step_is_sign_step():
    # step 1: m = (1-b1) g, v = (1-b2) g^2, bias-corrected mhat = g, vhat = g^2
    g = np.array([0.3, -2.0, 1e-3])
    p = np.array([1.0, 1.0, 1.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), step=1, lr=0.01)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_splitmix64_reference_values():
    # first two outputs of SplitMix64 started from state 0 (Vigna's reference)
    assert mlp.splitmix64(0) == 0xE220A8397B1DCDAF
    assert mlp.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_check_positions_in_range_and_spread():
    pos = np.concatenate([mlp.check_positions(7, 2, 1, q, 50) for q in range(200)])
    assert pos.min() >= 0 and pos.max() < 50
    assert len(np.unique(pos)) == 50                 # every position is reachable
    assert np.array_equal(mlp.check_positions(7, 2, 1, 5, 50), mlp.check_positions(7, 2, 1, 5, 50))


def test_residual_check_accepts_exact_and_rejects_wrong_ids():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((12, 3)) + 1j * rng.standard_normal((12, 3))
    T = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    A = np.zeros((12, 7), complex)
    skel, red = np.array([0, 2, 5]), np.array([1, 3, 4, 6])
    A[:, skel] = S
    A[:, red] = S @ T
    assert mlp.residual_ok(A[:8], skel, red, T, 1e-12)
    assert not mlp.residual_ok(A[:8], skel, red, T + 1e-3, 1e-6)
