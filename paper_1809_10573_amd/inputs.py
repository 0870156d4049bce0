"""Seeded synthetic workloads for the IDBF hot path.

This module only generates inputs: point grids, phase-function parameter
sets and random right-hand sides.  It holds none of the factorization's
arithmetic.  Both the HIP path and the CPU reference consume what it returns,
so the two always see bit-identical inputs.

Workloads follow the 1D examples of the paper's numerical section
(Example 1: a Fourier integral operator on a uniform grid), with the
configurations this project measures:

* uniform grids ``x_i = i/N`` in [0, 1) and ``xi_j = j - N/2`` in
  [-N/2, N/2) (0-based form of the paper's discretisation of Example 1);
* sorted uniform random points for Example 3 (the non-uniform Fourier
  transform): frequencies in [-N/2, N/2) and points in [0, 1);
* Example 2's Schloemilch points g_k = (k-1)/N and w_n = n pi for the
  kernel J_0(g w);
* phase ``Phi(x, xi) = -x*xi`` (the DFT kernel) or
  ``Phi(x, xi) = x*xi + c(x)|xi|`` with ``c(x) = (c0 + a*sin(2*pi*m*x))/cdiv``
  (the FIO kernel; the paper's own member is c0=2, a=0.2, m=1, cdiv=16);
* right-hand sides with i.i.d. N(0,1) + i N(0,1) entries from
  ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PHASE_DFT = 0
PHASE_FIO = 1
PHASE_J0 = 2


@dataclass(frozen=True)
class Phase:
    """Parameters of the phase function Phi of K(x, xi) = exp(2*pi*i*Phi(x, xi)).

    kind == PHASE_DFT: Phi = -x*xi.
    kind == PHASE_FIO: Phi = x*xi + c(x)*|xi|, c(x) = (c0 + a*sin(2*pi*freq*x)) / cdiv.
    kind == PHASE_J0: not a phase: K(g, w) = J_0(g*w) (Example 2); no parameters.
    """

    kind: int
    c0: float = 0.0
    a: float = 0.0
    freq: float = 0.0
    cdiv: float = 1.0


def dft_phase() -> Phase:
    return Phase(PHASE_DFT, 0.0, 0.0, 0.0, 1.0)


def j0_kernel() -> Phase:
    """The Schloemilch kernel K(g, w) = J_0(g w) of Example 2."""
    return Phase(PHASE_J0, 0.0, 0.0, 0.0, 1.0)


def schlomilch_points(N: int) -> tuple[np.ndarray, np.ndarray]:
    """Example 2's points: g_k = (k-1)/N and w_n = n pi, k, n = 1..N (float64,
    ascending; w_n is the float64 product n * pi)."""
    i = np.arange(N, dtype=np.float64)
    return i / N, (i + 1.0) * np.pi


def fio_phase(a: float = 1.0, freq: float = 1.0, c0: float = 2.0, cdiv: float = 8.0) -> Phase:
    return Phase(PHASE_FIO, float(c0), float(a), float(freq), float(cdiv))


def paper_example1_phase() -> Phase:
    """c(x) = (2 + 0.2 sin(2 pi x)) / 16, the phase of the paper's Example 1."""
    return Phase(PHASE_FIO, 2.0, 0.2, 1.0, 16.0)


def uniform_grid(N: int) -> tuple[np.ndarray, np.ndarray]:
    """x_i = i/N and xi_j = j - N/2, i, j = 0..N-1, as float64 (ascending)."""
    i = np.arange(N, dtype=np.float64)
    return i / N, i - N / 2


def nufft_points(N: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Points of Example 3, the 1D non-uniform Fourier transform
    u_k = sum_n exp(-2 pi i x_n w_k) g_n: row frequencies w_k ~ U[-N/2, N/2)
    and column points x_n ~ U[0, 1), i.i.d. from ``default_rng(seed)``, each
    sorted ascending.  A value drawn twice is redrawn, so both arrays are
    strictly increasing.  With the DFT phase Phi(w, x) = -w x the matrix
    K(w_k, x_n) is the paper's, rows at the frequencies."""
    rng = np.random.default_rng(seed)

    def draw(lo: float, hi: float) -> np.ndarray:
        v = np.unique(lo + (hi - lo) * rng.random(N))
        while len(v) < N:
            v = np.unique(np.concatenate([v, lo + (hi - lo) * rng.random(N - len(v))]))
        return v

    w = draw(-N / 2, N / 2)
    x = draw(0.0, 1.0)
    return w, x


def gaussian_vectors(N: int, nrhs: int | None, seed: int) -> np.ndarray:
    """Complex128 array (N,) if nrhs is None else (N, nrhs): N(0,1) + i N(0,1)."""
    rng = np.random.default_rng(seed)
    shape = (N,) if nrhs is None else (N, nrhs)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def family_draws(count: int, seed: int) -> list[tuple[float, int]]:
    """(a, m) pairs with a ~ U[0, 1) and m ~ U{1..4} for the FIO family."""
    rng = np.random.default_rng(seed)
    a = rng.random(count)
    m = rng.integers(1, 5, size=count)
    return [(float(ai), int(mi)) for ai, mi in zip(a, m)]


def batched_workload(count: int = 64, seed: int = 3, emin: int = 12, emax: int = 18,
                     leaf: int = 16, tol: float = 1e-6) -> list[dict]:
    """Many independent IDBF instances of uneven size and rank: N = 2^e with
    e ~ U{emin..emax}; the first half DFT kernels, the second half members of
    the FIO family c(x) = (2 + a sin 2 pi m x)/8 with a ~ U[0, 1), m ~ U{1..4};
    nrhs ~ U{1, 16, 64} right-hand sides each."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        e = int(rng.integers(emin, emax + 1))
        a = float(rng.random())
        m = int(rng.integers(1, 5))
        nrhs = int(rng.choice([1, 16, 64]))
        phase = dft_phase() if i < count // 2 else fio_phase(a, float(m))
        out.append(dict(phase=phase, N=1 << e, leaf=leaf, tol=tol, nrhs=nrhs, a=a, m=m,
                        kind="dft" if i < count // 2 else "fio"))
    return out


# The measured configurations (sizes, tolerances, leaf sizes).
CONFIGS = {
    "dft_n1024": dict(phase=dft_phase(), N=1024, leaf=8, tol=1e-10, seed=1),
    "fio_n65536": dict(phase=fio_phase(1.0, 1.0), N=1 << 16, leaf=16, tol=1e-6, seed=2),
    "fio_n1048576": dict(phase=fio_phase(1.0, 1.0), N=1 << 20, leaf=16, tol=1e-6, seed=4),
}
