"""The seeded synthetic inputs against the workloads they stand in for:
Example 1's grid and phase, Example 2's Schloemilch points, Example 3's
non-uniform points, the complex Gaussian probes, the FIO family draws and
the many-instance batch (sizes log-uniform over powers of two, half DFT and
half FIO members, uneven right-hand-side counts)."""
import math
from collections import Counter

import numpy as np

from paper_1809_10573_amd import inputs as I


def test_uniform_grid_is_the_papers():
    N = 1024
    X, O = I.uniform_grid(N)
    assert X.dtype == np.float64 and O.dtype == np.float64
    assert np.array_equal(X, np.arange(N) / N)                        # x_i = (i - 1)/N, i = 1..N
    assert np.array_equal(O, np.arange(N) - N / 2)                    # xi_j = j - 1 - N/2
    assert X[0] == 0.0 and O[0] == -N / 2 and O[-1] == N / 2 - 1


def test_phases():
    ex1 = I.paper_example1_phase()                                     # c(x) = (2 + 0.2 sin 2 pi x)/16
    assert (ex1.kind, ex1.c0, ex1.a, ex1.freq, ex1.cdiv) == (I.PHASE_FIO, 2.0, 0.2, 1.0, 16.0)
    f = I.fio_phase(0.3, 3.0)                                          # c(x) = (2 + a sin 2 pi m x)/8
    assert (f.kind, f.c0, f.a, f.freq, f.cdiv) == (I.PHASE_FIO, 2.0, 0.3, 3.0, 8.0)
    assert I.dft_phase().kind == I.PHASE_DFT and I.j0_kernel().kind == I.PHASE_J0


def test_schlomilch_points():
    N = 256
    g, w = I.schlomilch_points(N)
    assert np.array_equal(g, np.arange(N) / N)                        # g_k = (k - 1)/N
    assert np.array_equal(w, np.arange(1, N + 1) * np.pi)             # w_n = n pi
    assert np.all(np.diff(g) > 0) and np.all(np.diff(w) > 0)


def test_nufft_points_are_strictly_increasing_in_range_and_seeded():
    N = 4096
    w, x = I.nufft_points(N, seed=5)
    assert len(w) == len(x) == N
    assert np.all(np.diff(w) > 0) and np.all(np.diff(x) > 0)
    assert w.min() >= -N / 2 and w.max() < N / 2 and x.min() >= 0.0 and x.max() < 1.0
    w2, x2 = I.nufft_points(N, seed=5)
    assert np.array_equal(w, w2) and np.array_equal(x, x2)
    assert not np.array_equal(w, I.nufft_points(N, seed=6)[0])
    # uniform: each tenth of the ranges holds about a tenth of the points
    assert np.all(np.abs(np.histogram(x, 10, (0, 1))[0] - N / 10) < 5 * math.sqrt(N / 10))


def test_gaussian_probes():
    v = I.gaussian_vectors(1 << 16, None, seed=1)
    m = I.gaussian_vectors(1000, 8, seed=1)
    assert v.dtype == np.complex128 and v.shape == (1 << 16,) and m.shape == (1000, 8)
    assert abs(np.mean(np.abs(v) ** 2) - 2.0) < 0.05                   # N(0,1) + i N(0,1)
    assert abs(np.mean(v.real)) < 0.02 and abs(np.mean(v.imag)) < 0.02
    assert np.array_equal(v, I.gaussian_vectors(1 << 16, None, seed=1))


def test_fio_family_draws():
    d = I.family_draws(4000, seed=2)
    a = np.array([x[0] for x in d])
    m = Counter(x[1] for x in d)
    assert a.min() >= 0.0 and a.max() < 1.0 and abs(a.mean() - 0.5) < 0.02
    assert set(m) == {1, 2, 3, 4} and all(abs(c - 1000) < 150 for c in m.values())


def test_batched_workload_matches_its_configuration():
    work = I.batched_workload()
    assert len(work) == 64
    kinds = [w["kind"] for w in work]
    assert kinds[:32] == ["dft"] * 32 and kinds[32:] == ["fio"] * 32
    e = [int(math.log2(w["N"])) for w in work]
    assert all(1 << k == w["N"] for k, w in zip(e, work))
    assert set(e) <= set(range(12, 19)) and len(set(e)) >= 6            # log-uniform over 2^12..2^18
    assert {w["nrhs"] for w in work} == {1, 16, 64}
    assert all(w["tol"] == 1e-6 and w["leaf"] == 16 for w in work)
    for w in work[32:]:
        p = w["phase"]
        assert (p.kind, p.c0, p.cdiv) == (I.PHASE_FIO, 2.0, 8.0)
        assert p.a == w["a"] and 0.0 <= p.a < 1.0 and p.freq == float(w["m"]) and w["m"] in (1, 2, 3, 4)
    assert all(w["phase"].kind == I.PHASE_DFT for w in work[:32])


def test_measured_configurations():
    c = I.CONFIGS
    assert (c["dft_n1024"]["N"], c["dft_n1024"]["leaf"], c["dft_n1024"]["tol"]) == (1024, 8, 1e-10)
    assert (c["fio_n65536"]["N"], c["fio_n65536"]["leaf"], c["fio_n65536"]["tol"]) == (1 << 16, 16, 1e-6)
    assert (c["fio_n1048576"]["N"], c["fio_n1048576"]["leaf"], c["fio_n1048576"]["tol"]) == (1 << 20, 16, 1e-6)
    for k in ("fio_n65536", "fio_n1048576"):
        p = c[k]["phase"]
        assert (p.c0, p.a, p.freq, p.cdiv) == (2.0, 1.0, 1.0, 8.0)     # c(x) = (2 + sin 2 pi x)/8
