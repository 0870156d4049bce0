"""Kernel entries, dense matvec and closed forms (oracle; test infrastructure).

The matrix is K_ij = exp(2 pi i Phi(x_i, xi_j)) (Introduction: kernels of the
form a(x, xi) exp(2 pi i Phi(x, xi)) with a = 1; Example 1, eqs. 1D-FIO-kernal,
1D-FIO, 1D-xandxi).  Two phase functions are used:

* kind 0 (DFT):  Phi(x, xi) = -x * xi
* kind 1 (FIO):  Phi(x, xi) = x * xi + c(x) |xi|,  c(x) = (c0 + a sin(2 pi freq x)) / cdiv

and one kernel that is not of that form:

* kind 2 (J0):   K(g, w) = J_0(g w), the Schloemilch expansion of Example 2
                 (eq. S with nu = 0), real, evaluated at the float64 product
                 by ``bessel.j0``.

``phase`` arguments are any object with attributes kind, c0, a, freq, cdiv.

Phase evaluation.  At N = 2^20 the phase reaches ~10^5 turns, so a float64
phase would lose ~10 bits before the exponential.  The phase is therefore
formed in x87 extended precision (64-bit significand), each of the two terms
is reduced modulo 1 there, and only the reduced value theta in [-1/2, 1/2] is
rounded to float64 before exp(2 pi i theta).  On the uniform grids used here
x*xi is exact in extended precision and c(x)|xi| is within 2^-64 relative, so
the entries are correct to a few float64 ulps.  c(x) itself is the float64
value of its definition (numpy sin).
"""
from __future__ import annotations

import numpy as np

from . import bessel

PHASE_DFT = 0
PHASE_FIO = 1
PHASE_J0 = 2

_LD = np.longdouble


def amplitude_shift(phase, x) -> np.ndarray:
    """c(x) = (c0 + a sin(2 pi freq x)) / cdiv in float64 (Example 1, eq. 1D-FIO-kernal)."""
    x = np.asarray(x, dtype=np.float64)
    return (phase.c0 + phase.a * np.sin(2.0 * np.pi * phase.freq * x)) / phase.cdiv


def _frac(v):
    """v - round(v), in the dtype of v."""
    return v - np.rint(v)


def phase_mod1(phase, x, xi) -> np.ndarray:
    """Phi(x_i, xi_j) reduced to [-1/2, 1/2] (float64), outer over x and xi."""
    xl = np.asarray(x, dtype=np.float64).astype(_LD)[:, None]
    xil = np.asarray(xi, dtype=np.float64).astype(_LD)[None, :]
    if phase.kind == PHASE_DFT:
        th = -_frac(xl * xil)
    elif phase.kind == PHASE_FIO:
        c = amplitude_shift(phase, x).astype(_LD)[:, None]
        th = _frac(xl * xil) + _frac(c * np.abs(xil))
    else:
        raise ValueError(f"unknown phase kind {phase.kind}")
    return _frac(th).astype(np.float64)


def entries(phase, X, Omega, rows, cols) -> np.ndarray:
    """K(rows, cols) as a complex128 matrix: exp(2 pi i Phi(X[rows], Omega[cols])),
    or J_0(X[rows] Omega[cols]) for the Schloemilch kernel."""
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    if phase.kind == PHASE_J0:
        z = X[np.asarray(rows)][:, None] * Omega[np.asarray(cols)][None, :]
        return bessel.j0(z).astype(np.complex128)
    th = phase_mod1(phase, X[np.asarray(rows)], Omega[np.asarray(cols)])
    return np.exp(2j * np.pi * th)


def matvec_rows(phase, X, Omega, g, rows, chunk: int = 1 << 22) -> np.ndarray:
    """Exact rows of u = K g: u_i = sum_j K(x_i, xi_j) g_j for i in rows (Example 1, eq. 1D-FIO).

    g is (N,) or (N, nrhs).  Evaluated in row blocks of about ``chunk`` entries.
    """
    g = np.asarray(g, dtype=np.complex128)
    rows = np.asarray(rows, dtype=np.int64)
    N = len(Omega)
    cols = np.arange(N)
    out = np.zeros((len(rows),) + g.shape[1:], dtype=np.complex128)
    step = max(1, chunk // max(N, 1))
    for b in range(0, len(rows), step):
        r = rows[b:b + step]
        out[b:b + step] = entries(phase, X, Omega, r, cols) @ g
    return out


def dense_matvec(phase, X, Omega, g) -> np.ndarray:
    """u = K g with every row evaluated (O(N^2))."""
    return matvec_rows(phase, X, Omega, g, np.arange(len(X)))


def dft_closed_form(g) -> np.ndarray:
    """K g for the DFT kernel on the uniform grid x_i = i/N, xi_j = j - N/2.

    exp(-2 pi i (i/N)(j - N/2)) = (-1)^i exp(-2 pi i i j / N), so
    u = (-1)^i FFT(g)_i with numpy's forward FFT convention.
    """
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    sign = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    f = np.fft.fft(g, axis=0)
    return f * (sign if g.ndim == 1 else sign[:, None])


def fio_const_closed_form(phase, g) -> np.ndarray:
    """K g for the FIO kernel with a == 0 (constant c) on the uniform grid.

    K_ij = exp(2 pi i x_i xi_j) exp(2 pi i c |xi_j|) and
    exp(2 pi i (i/N)(j - N/2)) = (-1)^i exp(2 pi i i j / N), so
    u = (-1)^i N IFFT(g * exp(2 pi i c |xi|))_i.
    """
    if phase.kind != PHASE_FIO or phase.a != 0.0:
        raise ValueError("closed form needs the FIO kernel with a == 0")
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    c = phase.c0 / phase.cdiv
    xi = np.arange(N, dtype=np.float64) - N / 2
    # reduce c|xi| modulo 1 in extended precision, as in phase_mod1
    th = _frac(_frac(_LD(c) * np.abs(xi).astype(_LD))).astype(np.float64)
    h = np.exp(2j * np.pi * th)
    gh = g * (h if g.ndim == 1 else h[:, None])
    sign = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    f = N * np.fft.ifft(gh, axis=0)
    return f * (sign if g.ndim == 1 else sign[:, None])


def relative_error(approx, exact) -> float:
    """sqrt(sum |approx - exact|^2 / sum |exact|^2): the paper's epsilon^a over the given rows."""
    approx = np.asarray(approx)
    exact = np.asarray(exact)
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
