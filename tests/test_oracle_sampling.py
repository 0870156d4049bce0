"""Hand-worked cases of the Mock-Chebyshev rule (the rule itself is parity unpinned)."""
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
