"""Pins of the oracle's kernel entries and dense matvec (closed forms, exact arithmetic)."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import inputs as I


@pytest.mark.parametrize("N", [8, 64, 256, 1024])
def test_dft_dense_matches_fft(N):
    X, O = I.uniform_grid(N)
    g = I.gaussian_vectors(N, None, seed=N)
    y = oracle.dense_matvec(I.dft_phase(), X, O, g)
    assert oracle.relative_error(y, oracle.dft_closed_form(g)) < 1e-13


@pytest.mark.parametrize("N,c0,cdiv", [(64, 2.0, 8.0), (512, 3.0, 16.0), (1024, 2.0, 8.0)])
def test_fio_constant_c_matches_ifft(N, c0, cdiv):
    X, O = I.uniform_grid(N)
    ph = I.fio_phase(a=0.0, freq=1.0, c0=c0, cdiv=cdiv)
    g = I.gaussian_vectors(N, 3, seed=7)
    y = oracle.dense_matvec(ph, X, O, g)
    assert oracle.relative_error(y, oracle.fio_const_closed_form(ph, g)) < 1e-13


def test_fio_continuity_in_a():
    # u(a) - u(0) = O(a): for small a the FIO matvec approaches the constant-c closed form
    N = 256
    X, O = I.uniform_grid(N)
    g = I.gaussian_vectors(N, None, seed=3)
    y0 = oracle.fio_const_closed_form(I.fio_phase(0.0, 1.0), g)
    errs = [oracle.relative_error(oracle.dense_matvec(I.fio_phase(a, 1.0), X, O, g), y0)
            for a in (1e-3, 1e-4, 1e-5)]
    assert errs[0] > errs[1] > errs[2]
    assert 5 < errs[0] / errs[1] < 20 and 5 < errs[1] / errs[2] < 20


def test_rows_agree_with_full_dense():
    N = 512
    X, O = I.uniform_grid(N)
    ph = I.fio_phase(0.8, 3.0)
    g = I.gaussian_vectors(N, 2, seed=11)
    full = oracle.dense_matvec(ph, X, O, g)
    rows = np.array([0, 3, 17, 255, 511])
    part = oracle.matvec_rows(ph, X, O, g, rows, chunk=1000)
    assert oracle.relative_error(part, full[rows]) < 1e-14


def _exact_turns(x, xi, phase):
    """Phi(x, xi) mod 1 in exact rational arithmetic from the float64 inputs
    (c(x) taken as its float64 value)."""
    fx, fxi = Fraction(float(x)), Fraction(float(xi))
    if phase.kind == I.PHASE_DFT:
        v = -fx * fxi
    else:
        c = Fraction(float(oracle.amplitude_shift(phase, np.array([x]))[0]))
        v = fx * fxi + c * abs(fxi)
    v -= math.floor(v + Fraction(1, 2))
    return v


@pytest.mark.parametrize("kind", ["dft", "fio"])
def test_phase_reduction_is_exact_at_large_N(kind):
    # At N = 2^20 the phase is ~1e5 turns.  x*xi is exact in extended precision;
    # c(x)|xi| has 73 significant bits and is rounded to 64 (<= 2^-64 * 0.375 * 2^19
    # ~ 1e-14 turns), so the reduced phase is exact to ~1e-14.
    N = 1 << 20
    X, O = I.uniform_grid(N)
    ph = I.dft_phase() if kind == "dft" else I.fio_phase(1.0, 1.0)
    rng = np.random.default_rng(5)
    rows = rng.integers(0, N, 40)
    cols = np.concatenate([rng.integers(0, N, 38), [0, N - 1]])
    th = oracle.phase_mod1(ph, X[rows], O[cols])
    assert np.all(np.abs(th) <= 0.5)
    worst = 0.0
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            ex = _exact_turns(X[i], O[j], ph)
            diff = abs(th[a, b] - float(ex))
            worst = max(worst, min(diff, 1 - diff))
    assert worst < (5e-15 if kind == "dft" else 2e-14)


def test_phase_reduction_on_nonuniform_points():
    # Example 3's points: w*x has up to 106 significant bits and is rounded to
    # 64 in extended precision (<= 2^-64 * N/2 ~ 3e-14 turns at N = 2^20)
    N = 1 << 20
    W, Xp = I.nufft_points(N, seed=4)
    rng = np.random.default_rng(6)
    rows = np.concatenate([rng.integers(0, N, 30), [0, N - 1]])
    cols = np.concatenate([rng.integers(0, N, 30), [0, N - 1]])
    th = oracle.phase_mod1(I.dft_phase(), W[rows], Xp[cols])
    worst = 0.0
    for a, i in enumerate(rows):
        for b, j in enumerate(cols):
            diff = abs(th[a, b] - float(_exact_turns(W[i], Xp[j], I.dft_phase())))
            worst = max(worst, min(diff, 1 - diff))
    assert worst < 4e-14
    K = oracle.entries(I.dft_phase(), W, Xp, rows, cols)
    ref = np.exp(-2j * np.pi * np.outer(W[rows], Xp[cols]))   # unreduced: loses ~N*eps turns
    assert np.max(np.abs(K - ref)) < 1e-9


def test_nufft_points_shape_and_order():
    W, Xp = I.nufft_points(4096, seed=2)
    assert W.shape == Xp.shape == (4096,)
    assert np.all(np.diff(W) > 0) and np.all(np.diff(Xp) > 0)
    assert -2048 <= W[0] and W[-1] < 2048 and 0 <= Xp[0] and Xp[-1] < 1
    W2, X2 = I.nufft_points(4096, seed=2)
    assert np.array_equal(W, W2) and np.array_equal(Xp, X2)


def test_entries_unimodular_and_dft_integer_form():
    N = 128
    X, O = I.uniform_grid(N)
    K = oracle.entries(I.dft_phase(), X, O, np.arange(N), np.arange(N))
    assert np.allclose(np.abs(K), 1.0, atol=1e-15)
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :] - N // 2
    ref = np.exp(-2j * np.pi * ((i * j) % N) / N)      # integer reduction of i*(j-N/2) mod N
    assert np.max(np.abs(K - ref)) < 1e-14
