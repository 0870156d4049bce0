"""Mock-Chebyshev sample selection (oracle; test infrastructure).

Section 2.1 samples t*k rows (t = 1 in all experiments) of the matrix whose
ID is sought, choosing them "from the Mock-Chebyshev grids" of the index set;
the rule itself is only cited, not stated.  The reading used here is the
usual one for mock-Chebyshev points (the subset of a given ordered point set
closest to Chebyshev-Lobatto points):

* The allowed points have coordinates a_0 <= ... <= a_{n-1} (x for rows,
  xi for columns).  If s >= n every point is taken.
* Targets z_j = a_0 + (a_{n-1} - a_0) * f_j, j = 0..s-1, with
  f_j = (1 - cos(pi j / (s-1))) / 2 (the Chebyshev-Lobatto points mapped to
  [0, 1]); f = 1/2 when s = 1.  f_j is rational only for
  j/(s-1) in {0, 1/3, 1/2, 2/3, 1} (Niven's theorem); there it is set to its
  exact value 0, 1/4, 1/2, 3/4, 1 so that exact midpoint ties do not depend
  on the last bit of a cosine.
* For j = 0..s-1 in order, the unused allowed point nearest to z_j is taken
  (smaller position on a tie).
* The chosen positions are returned in ascending order.

Pins (the paper states no rule to check against): on an equispaced grid,
wherever the Chebyshev-Lobatto points' nearest grid points are distinct,
the picks are exactly those points (the published mock-Chebyshev subset,
computed in the test from 60-digit cosines); interpolation on the subsets
has a Lebesgue constant near Chebyshev-Lobatto's, far below an equispaced
subset's; picks are invariant under exact affine maps; hand-worked cases
fix the collision and tie rules.

``random_positions`` is the uniformly random alternative the paper compares
Mock-Chebyshev against (Section 3): s distinct positions of n by Floyd's
algorithm (for j = n-s .. n-1: draw t uniform in [0, j]; take t, or j when t
was taken already), each draw from SplitMix64 of a counter built from
(seed, level, side, ID, draw), returned ascending.
"""
from __future__ import annotations

import math

import numpy as np

from .mlp import MASK64, splitmix64

SAMPLER_SALT = 0xA0761D6478BD642F  # keeps the sampler's counters apart from other draws

_EXACT = {(0, 1): 0.0, (1, 3): 0.25, (1, 2): 0.5, (2, 3): 0.75, (1, 1): 1.0}


def chebyshev_fraction(j: int, s: int) -> float:
    """Position in [0, 1] of the j-th of s Chebyshev-Lobatto points (ascending)."""
    if s == 1:
        return 0.5
    g = math.gcd(j, s - 1)
    key = (j // g, (s - 1) // g)
    if key in _EXACT:
        return _EXACT[key]
    return 0.5 * (1.0 - math.cos(math.pi * j / (s - 1)))


def mock_chebyshev(coords, s: int) -> np.ndarray:
    """Ascending positions of s mock-Chebyshev points among sorted ``coords``."""
    coords = np.asarray(coords, dtype=np.float64)
    n = len(coords)
    if s >= n:
        return np.arange(n)
    lo, hi = coords[0], coords[-1]
    used = np.zeros(n, dtype=bool)
    picks = []
    for j in range(s):
        z = lo + (hi - lo) * chebyshev_fraction(j, s)
        d = np.abs(coords - z)
        d[used] = np.inf
        p = int(np.argmin(d))        # first minimum: the smaller position on ties
        used[p] = True
        picks.append(p)
    return np.sort(np.array(picks, dtype=np.int64))


def random_positions(seed: int, level: int, side: int, q: int, n: int, s: int) -> np.ndarray:
    """Ascending positions of s uniformly random distinct points among n
    (Floyd's algorithm, SplitMix64 draws)."""
    if s >= n:
        return np.arange(n)
    base = ((seed & 0xFFFFFFFF) << 32) ^ (level << 24) ^ (side << 23) ^ q
    chosen = []
    for i in range(s):
        j = n - s + i
        z = splitmix64((((base << 8) | i) ^ SAMPLER_SALT) & MASK64)
        t = ((z >> 32) * (j + 1)) >> 32          # uniform in [0, j]
        chosen.append(j if t in chosen else t)
    return np.sort(np.array(chosen, dtype=np.int64))
