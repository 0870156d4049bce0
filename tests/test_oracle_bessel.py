"""Pins of the oracle's J_0 (oracle/bessel.py) and of Example 2's Schloemilch
kernel: a 40-digit reference (mpmath) over the whole argument range, the
Cephes implementation in scipy where it is accurate, closed-form special
values, and the factorization of K(g, w) = J_0(g w)."""
import numpy as np
import pytest

import oracle
from oracle import bessel
from paper_1809_10573_amd import inputs as I

mpmath = pytest.importorskip("mpmath")


@pytest.mark.parametrize("lo,hi", [(0.0, 8.0), (8.0, 25.0), (25.0, 200.0), (200.0, 1e5), (1e5, 3.3e6)])
def test_j0_against_40_digit_reference(lo, hi):
    mpmath.mp.dps = 40
    z = np.random.default_rng(int(hi)).uniform(lo, hi, 60)
    ref = np.array([float(mpmath.besselj(0, mpmath.mpf(float(v)))) for v in z])
    got = bessel.j0(z)
    amp = np.minimum(1.0, np.sqrt(2.0 / (np.pi * np.maximum(z, 1e-300))))  # envelope of |J_0|
    assert np.max(np.abs(got - ref) / amp) < 3e-15


def test_j0_matches_cephes_below_25_and_special_values():
    from scipy import special
    z = np.linspace(0.0, 24.999, 2001)
    assert np.max(np.abs(bessel.j0(z) - special.j0(z))) < 1.5e-15
    assert bessel.j0(np.array([0.0]))[0] == 1.0
    assert np.array_equal(bessel.j0(-z), bessel.j0(z))              # even
    # the first two zeros j_{0,1}, j_{0,2} (A&S Table 9.5) and J_0(z) ~ 1 - z^2/4 near 0
    assert abs(bessel.j0(np.array([2.404825557695773]))[0]) < 1e-15
    assert abs(bessel.j0(np.array([5.520078110286311]))[0]) < 1e-15
    t = np.array([1e-4])
    assert abs(bessel.j0(t)[0] - (1 - t[0] ** 2 / 4)) <= 2.3e-16               # two ulps of 1


def test_methods_agree_across_the_switch():
    # around the switch both methods are accurate: they agree at the same arguments
    z = np.array([24.0, 24.9, 25.0, 25.1, 26.0])
    assert np.max(np.abs(bessel._miller(z) - bessel._hankel(z))) < 1e-15


def test_reduction_range_is_enforced():
    with pytest.raises(ValueError):
        bessel.j0(np.array([2.0 ** 24 * 1.6]))


def test_schlomilch_entries_and_points():
    N = 64
    g, w = I.schlomilch_points(N)
    assert g[0] == 0.0 and g[-1] == (N - 1) / N and w[0] == np.pi and w[-1] == N * np.pi
    K = oracle.entries(I.j0_kernel(), g, w, np.arange(N), np.arange(N))
    assert np.all(K.imag == 0) and np.all(K[0] == 1.0)                # J_0(0) = 1 on the first row
    from scipy import special
    z = np.outer(g, w)
    assert np.max(np.abs(K.real - special.j0(z))) < 2e-15          # z <= 64 pi: Cephes is accurate here


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_schlomilch_factorization_tracks_tolerance(tol):
    N, leaf = 512, 8
    g, w = I.schlomilch_points(N)
    ph = I.j0_kernel()
    F = oracle.build(ph, g, w, leaf, tol, oversample=2)
    x = I.gaussian_vectors(N, None, seed=1)
    assert oracle.relative_error(oracle.apply(F, x), oracle.dense_matvec(ph, g, w, x)) < 100 * tol
    y = I.gaussian_vectors(N, None, seed=2)
    K = oracle.entries(ph, g, w, np.arange(N), np.arange(N))
    assert oracle.relative_error(oracle.apply_adjoint(F, y), K.conj().T @ y) < 100 * tol


def test_schlomilch_full_sampling_reproduces_K():
    N, leaf = 128, 4
    g, w = I.schlomilch_points(N)
    ph = I.j0_kernel()
    F = oracle.build(ph, g, w, leaf, 1e-13, sample_all=True)
    K = oracle.entries(ph, g, w, np.arange(N), np.arange(N))
    assert np.linalg.norm(oracle.densify(F) - K, 2) / np.linalg.norm(K, 2) < 1e-11
