"""The Mock-Chebyshev rule: hand-worked cases (collisions, ties), the
closed form of the published mock-Chebyshev subset on equispaced grids,
exact affine invariance and the stability of interpolation on its subsets;
and the uniformly random alternative."""
import numpy as np

import oracle


def test_fraction_exact_cases():
    assert oracle.chebyshev_fraction(0, 4) == 0.0
    assert oracle.chebyshev_fraction(1, 4) == 0.25      # j/(s-1) = 1/3
    assert oracle.chebyshev_fraction(2, 4) == 0.75      # 2/3
    assert oracle.chebyshev_fraction(3, 4) == 1.0
    assert oracle.chebyshev_fraction(2, 5) == 0.5       # 1/2
    assert oracle.chebyshev_fraction(0, 1) == 0.5
    f = [oracle.chebyshev_fraction(j, 9) for j in range(9)]
    assert all(a < b for a, b in zip(f, f[1:]))
    assert abs(f[1] - 0.5 * (1 - np.cos(np.pi / 8))) < 1e-16


def test_hand_worked_selections():
    c = np.arange(10.0)
    # targets 0, 2.25, 6.75, 9
    assert list(oracle.mock_chebyshev(c, 4)) == [0, 2, 7, 9]
    # targets 0, 1.5 (tie between 1 and 2 -> 1), 3
    assert list(oracle.mock_chebyshev(np.arange(4.0), 3)) == [0, 1, 3]
    # collision: targets 0, 5, 10 over {0, 1, 2, 10}; 5 is nearest to 2 among unused
    assert list(oracle.mock_chebyshev(np.array([0.0, 1.0, 2.0, 10.0]), 3)) == [0, 2, 3]
    # targets 0, 1.25, 3.75, 5: 0 -> 0, 1.25 -> 0.3, 3.75 -> 5.0; the last target's
    # nearest point (5.0) is taken, so the pick moves to the nearest unused one (0.2)
    assert list(oracle.mock_chebyshev(np.array([0.0, 0.1, 0.2, 0.3, 5.0]), 4)) == [0, 2, 3, 4]
    # s = 1 picks the point nearest the midpoint; s >= n takes everything
    assert list(oracle.mock_chebyshev(np.array([0.0, 0.4, 0.7, 1.0]), 1)) == [1]
    assert list(oracle.mock_chebyshev(np.array([3.0, 4.0]), 5)) == [0, 1]


def test_selection_is_distinct_sorted_and_endpoint_anchored():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(2, 200))
        coords = np.sort(rng.random(n))
        s = int(rng.integers(1, n + 1))
        p = oracle.mock_chebyshev(coords, s)
        assert len(p) == s and len(set(p.tolist())) == s
        assert np.all(np.diff(p) > 0)
        if 2 <= s < n:
            assert p[0] == 0 and p[-1] == n - 1


def test_random_positions_are_distinct_sorted_and_deterministic():
    from oracle.sampling import random_positions
    for (n, s) in [(10, 3), (128, 127), (1000, 128), (5, 5), (7, 9)]:
        p = random_positions(11, 2, 1, 17, n, s)
        assert len(p) == min(n, s) and len(np.unique(p)) == len(p)
        assert np.all(np.diff(p) > 0) and p.min() >= 0 and p.max() < n
        assert np.array_equal(p, random_positions(11, 2, 1, 17, n, s))
    assert not np.array_equal(random_positions(11, 2, 1, 17, 1000, 10), random_positions(11, 2, 1, 18, 1000, 10))


def test_random_positions_are_uniform_subsets():
    # Floyd's algorithm draws every s-subset with probability 1 / C(n, s): over
    # 20000 counters the 10 subsets of 2 out of 5 each appear 2000 +- a few %
    from oracle.sampling import random_positions
    from collections import Counter
    cnt = Counter(tuple(random_positions(3, 1, 0, q, 5, 2)) for q in range(20000))
    assert len(cnt) == 10
    assert all(abs(v - 2000) < 200 for v in cnt.values()), cnt


def _lebesgue_constant(nodes, fine):
    """max over `fine` of sum_j |l_j(x)| for polynomial interpolation at
    `nodes` (barycentric weights; nodes distinct)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    w = np.array([1.0 / np.prod(nodes[j] - np.delete(nodes, j)) for j in range(len(nodes))])
    lam = 0.0
    for x in fine:
        d = x - nodes
        if np.any(d == 0.0):
            lam = max(lam, 1.0)
            continue
        t = w / d
        lam = max(lam, np.sum(np.abs(t)) / abs(np.sum(t)))
    return lam


def test_equispaced_grids_give_the_rounded_chebyshev_lobatto_points():
    """Mock-Chebyshev subsets of an equispaced grid (Boyd and Xu's
    definition: the grid point nearest each Chebyshev-Lobatto point): where
    those nearest points are all distinct, the rule must return exactly them.
    The targets come from 60-digit cosines, the nearest index by rounding
    with ties to the lower index; no greedy pass is involved."""
    mp = __import__("pytest").importorskip("mpmath")
    mp.mp.dps = 60
    checked = 0
    for n, s in [(2001, 5), (2001, 17), (2001, 33), (513, 9), (100, 7), (4097, 65), (31, 4), (1001, 21)]:
        idx = []
        for j in range(s):
            z = (n - 1) * (1 - mp.cos(mp.pi * j / (s - 1))) / 2
            lo = int(mp.floor(z))
            idx.append(lo if z - lo <= mp.mpf(1) / 2 else lo + 1)  # a tie goes to the lower index
        if len(set(idx)) < s:
            continue  # two targets share a nearest point: the greedy rule decides, not this pin
        for a, h in [(0.0, 1.0), (-3.5, 0.25), (1e3, 2.0 ** -10)]:
            coords = a + h * np.arange(n, dtype=np.float64)
            assert list(oracle.mock_chebyshev(coords, s)) == idx, (n, s, a, h)
        checked += 1
    assert checked >= 6


def test_selection_is_invariant_under_exact_affine_maps():
    """The rule uses only the ordering of distances to targets placed
    proportionally over [min, max], so scaling by a power of two and
    shifting by an integer (both exact on integer-valued coordinates)
    leave the picks unchanged."""
    rng = np.random.default_rng(3)
    for _ in range(40):
        n = int(rng.integers(3, 300))
        coords = np.sort(rng.choice(10 ** 6, n, replace=False)).astype(np.float64)
        s = int(rng.integers(1, n + 1))
        base = oracle.mock_chebyshev(coords, s)
        for scale, shift in [(4.0, 1000.0), (0.5, -7.0), (2.0 ** 20, 3.0)]:
            assert np.array_equal(oracle.mock_chebyshev(scale * coords + shift, s), base)


def test_subsets_interpolate_stably():
    """The reason for mock-Chebyshev subsets: polynomial interpolation on
    them is as stable as on Chebyshev-Lobatto points (Lebesgue constant
    2/pi log(s) + 1 up to a small factor), where an equispaced subset of
    the same size grows like 2^s / (e s log s)."""
    n = 4001
    grid = np.linspace(-1.0, 1.0, n)
    fine = np.linspace(-1.0, 1.0, 20001)
    for s in (11, 21, 31):
        mock = grid[oracle.mock_chebyshev(grid, s)]
        lam = _lebesgue_constant(mock, fine)
        assert lam < 2.0 * (2.0 / np.pi * np.log(s) + 1.0), (s, lam)
        equi = grid[np.round(np.linspace(0, n - 1, s)).astype(int)]
        assert _lebesgue_constant(equi, fine) > 0.5 * 2.0 ** s / (np.e * s * np.log(s)), s
