"""Pins of the oracle's IDBF construction and apply (Sections 2.2-2.4)."""
import os
from functools import reduce

import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _K(ph, N, X=None, O=None):
    if X is None:
        X, O = I.uniform_grid(N)
    return oracle.entries(ph, X, O, np.arange(N), np.arange(N))


@pytest.mark.parametrize("N,leaf,kind", [(16, 8, "dft"), (32, 2, "fio"), (64, 4, "fio"),
                                         (128, 4, "fio"), (128, 2, "dft"), (256, 8, "fio"),
                                         (256, 2, "fio"), (256, 4, "nufft"), (128, 2, "nufft")])
def test_full_sampling_reproduces_K(N, leaf, kind):
    # With every allowed point sampled, each ID is accurate to its tolerance on its
    # whole block; at tol = 1e-13 the assembled factorization must equal K.
    ph = I.fio_phase(1.0, 2.0) if kind == "fio" else I.dft_phase()
    X, O = I.nufft_points(N, seed=N) if kind == "nufft" else I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, 1e-13, sample_all=True)
    K = _K(ph, N, X, O)
    err = np.linalg.norm(oracle.densify(F) - K, 2) / np.linalg.norm(K, 2)
    assert err < 1e-11


@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_approximation_tracks_tolerance(tol):
    N, leaf = 256, 4
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, tol, sample_all=True)
    K = _K(ph, N)
    err = np.linalg.norm(oracle.densify(F) - K, 2) / np.linalg.norm(K, 2)
    assert err < 100 * tol
    assert F.nnz() < K.size


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_nufft_tracks_tolerance_with_mock_chebyshev_samples(tol):
    # Example 3 (random points, unequal geometric block sizes at equal counts):
    # the sampled construction against the dense matrix
    N, leaf = 1024, 8
    W, Xp = I.nufft_points(N, seed=7)
    ph = I.dft_phase()
    F = oracle.build(ph, W, Xp, leaf, tol, oversample=2)
    g = I.gaussian_vectors(N, None, seed=3)
    err = oracle.relative_error(oracle.apply(F, g), oracle.dense_matvec(ph, W, Xp, g))
    assert err < 100 * tol
    assert F.nnz() < N * N


def test_ranks_bounded_by_block_svd():
    # every ID sees its whole block when sample_all is set, so its rank is bounded
    # below by the block's singular values (stopping rule bound of the cID)
    N, leaf, tol = 256, 8, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, tol, sample_all=True)
    L, H = F.L, F.H
    checked = 0
    for t in range(1, H + 1):
        for (r, p), rec in F.U[t].items():
            if t == 1:
                allowed = np.arange(p * N // 2, (p + 1) * N // 2)
            else:
                sh = L - 2 * t + 2
                allowed = np.concatenate([F.V[t - 1][(cc, r >> sh)].skel
                                          for cc in range(p << sh, (p + 1) << sh)])
            B = oracle.entries(ph, X, O, rec.cand, allowed).T
            sv = np.linalg.svd(B, compute_uv=False)
            assert len(rec.skel) >= np.count_nonzero(sv > np.sqrt(len(rec.cand)) * tol * sv[0])
            checked += 1
    assert checked == sum(len(F.U[t]) for t in F.U)


def test_dft_n1024_leaf8_matches_fft():
    # the DFT workload at N = 1024, leaf 8, tol 1e-10 against the FFT closed form
    N = 1024
    X, O = I.uniform_grid(N)
    F = oracle.build(I.dft_phase(), X, O, 8, 1e-10)
    assert (F.L, F.H) == (7, 3)
    g = I.gaussian_vectors(N, None, seed=1)
    err = oracle.relative_error(oracle.apply(F, g), oracle.dft_closed_form(g))
    assert err < 1e-8


def test_fio_leaf16_oversampling():
    # leaf 16 with t = 1 under-samples the leaf-level IDs of this phase; t = 2 does not
    N = 1024
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    g = I.gaussian_vectors(N, None, seed=2)
    y = oracle.dense_matvec(ph, X, O, g)
    F2 = oracle.build(ph, X, O, 16, 1e-6, oversample=2)
    assert oracle.relative_error(oracle.apply(F2, g), y) < 1e-5


def test_multiple_rhs_and_factor_product():
    N, leaf = 128, 4
    ph = I.fio_phase(0.5, 2.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, 1e-8)
    G = I.gaussian_vectors(N, 5, seed=4)
    Y = oracle.apply(F, G)
    for j in range(5):
        assert np.allclose(Y[:, j], oracle.apply(F, G[:, j]), rtol=0, atol=1e-13)
    P = reduce(np.matmul, oracle.factor_matrices(F))
    assert np.max(np.abs(P - oracle.densify(F))) < 1e-12


def _golden_patterns():
    pats = {}
    with open(os.path.join(GOLDEN, "tikz_factor_patterns_m16.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, x0, y0, x1, y1 = line.split()
            x0, y0, x1, y1 = map(int, (x0, y0, x1, y1))
            M = pats.setdefault(name, np.zeros((32, 32), dtype=bool))
            M[32 - max(y0, y1):32 - min(y0, y1), min(x0, x1):max(x0, x1)] = True
    return pats


def test_factor_patterns_match_paper_figures():
    # 16 leaves of 2 points, rank-1 IDs: Figures exlfac and exsfac.
    # Level 1 uses the figures' own order (q = partner * 16 + node).  At level 2 the
    # figures order IDs by (outer row half, outer column half, inner half, node)
    # while q orders them (outer, inner, other outer, node): bits 2 and 3 swap.
    pats = _golden_patterns()
    N, leaf = 32, 2
    X, O = I.uniform_grid(N)
    F = oracle.build(I.fio_phase(1.0, 1.0), X, O, leaf, 0.0, kmax=1)
    assert (F.L, F.H) == (4, 2)
    U1, U2, S, V2, V1 = oracle.factor_matrices(F)
    nz = lambda M: np.abs(M) > 0
    assert np.array_equal(nz(U1), pats["UL"])
    assert np.array_equal(nz(V1), pats["VL"])
    swap = np.array([(i & ~12) | ((i & 4) << 1) | ((i & 8) >> 1) for i in range(32)])
    SL = U2 @ S @ V2
    assert np.array_equal(nz(SL), pats["SL"])
    assert np.array_equal(nz(U2[:, swap]), pats["UL1"])
    assert np.array_equal(nz(S[swap][:, swap]), pats["SL1"])
    assert np.array_equal(nz(V2[swap]), pats["VL1"])


def test_bad_sizes_rejected():
    with pytest.raises(ValueError):
        oracle.tree_sizes(96, 8)
    with pytest.raises(ValueError):
        oracle.tree_sizes(64, 3)
    with pytest.raises(ValueError):
        oracle.tree_sizes(8, 16)


def test_mock_chebyshev_beats_random_sampling():
    """Section 3: Mock-Chebyshev samples give a far more accurate factorization
    than uniformly random ones at the same sample count."""
    N = 512
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    g = I.gaussian_vectors(N, None, 1)
    ex = oracle.dense_matvec(ph, X, O, g)
    err = {s: oracle.relative_error(oracle.apply(oracle.build(ph, X, O, 16, 1e-6, oversample=2, sampler=s,
                                                              seed=5), g), ex)
           for s in ("mockcheb", "random")}
    assert err["random"] > 10 * err["mockcheb"], err


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("N,leaf,kind,tol,os_", [(1024, 8, "dft", 1e-10, 1), (512, 16, "fio", 1e-6, 2),
                                                 (256, 2, "fio", 1e-8, 1), (512, 8, "nufft", 1e-8, 2),
                                                 (16, 8, "dft", 1e-10, 1)])
def test_adjoint_identity(N, leaf, kind, tol, os_):
    # <K~ x, y> = <x, K~^H y> for the same factors: pins the reversed,
    # conjugate-transposed stages against the (independently pinned) apply
    ph = I.fio_phase(1.0, 1.0) if kind == "fio" else I.dft_phase()
    X, O = I.nufft_points(N, seed=2) if kind == "nufft" else I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, tol, oversample=os_)
    x = I.gaussian_vectors(N, 3, seed=1)
    y = I.gaussian_vectors(N, 3, seed=2)
    lhs = np.einsum("ij,ij->j", y.conj(), oracle.apply(F, x))
    rhs = np.einsum("ij,ij->j", oracle.apply_adjoint(F, y).conj(), x)
    scale = np.linalg.norm(x, axis=0) * np.linalg.norm(y, axis=0) * np.linalg.norm(oracle.apply(F, x)) / \
        np.linalg.norm(x)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13


def test_adjoint_is_conjugate_transpose_of_densified_factors():
    N, leaf = 64, 4
    ph = I.fio_phase(1.0, 2.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, 1e-8, oversample=2)
    A = oracle.apply_adjoint(F, np.eye(N, dtype=np.complex128))
    assert np.max(np.abs(A - oracle.densify(F).conj().T)) < 1e-13
    # and the product of the explicit factors, conjugate transposed in reverse
    Fs = oracle.factor_matrices(F)
    P = reduce(lambda a, b: a @ b, [f.conj().T for f in Fs[::-1]])
    assert np.max(np.abs(A - P)) < 1e-12


def test_adjoint_with_full_sampling_reproduces_K_H():
    # tol 1e-13 with every allowed point sampled: K~^H equals K^H
    N, leaf = 256, 4
    W, Xp = I.nufft_points(N, seed=3)
    ph = I.dft_phase()
    F = oracle.build(ph, W, Xp, leaf, 1e-13, sample_all=True)
    K = oracle.entries(ph, W, Xp, np.arange(N), np.arange(N))
    g = I.gaussian_vectors(N, None, seed=4)
    assert oracle.relative_error(oracle.apply_adjoint(F, g), K.conj().T @ g) < 1e-11


def _full_blocks(F, ph, X, O):
    """Every ID's whole complementary block (candidates x the allowed set it
    sees), as the ID's matrix: K(allowed, cand) for V, K(cand, allowed)^T for U."""
    N, L, H = F.N, F.L, F.H
    for t in range(1, H + 1):
        for (r, p), rec in F.U[t].items():
            if t == 1:
                allowed = np.arange(p * N // 2, (p + 1) * N // 2)
            else:
                sh = L - 2 * t + 2
                allowed = np.concatenate([F.V[t - 1][(cc, r >> sh)].skel
                                          for cc in range(p << sh, (p + 1) << sh)])
            yield rec, oracle.entries(ph, X, O, rec.cand, allowed).T
        for (cn, p), rec in F.V[t].items():
            sh = L - 2 * t + 1
            allowed = np.concatenate([F.U[t][(rr, cn >> sh)].skel for rr in range(p << sh, (p + 1) << sh)])
            yield rec, oracle.entries(ph, X, O, allowed, rec.cand)


@pytest.mark.parametrize("kind,N,leaf,tol", [("fio", 256, 8, 1e-6), ("dft", 256, 8, 1e-10),
                                             ("fio", 256, 4, 1e-8), ("fio2", 256, 8, 1e-6),
                                             ("fio", 256, 16, 1e-6)])
def test_eps_rank_two_sided_against_block_svd(kind, N, leaf, tol):
    # With every allowed point sampled each ID sees its whole complementary
    # block B.  Its eps-rank (eq. acc) is compared with the SVD count
    # r_eps(B) = #{sigma_i > eps sigma_1} from both sides: |k - r| <= 2 on at
    # least 95% of the blocks of every level and side, and (empirically, with
    # |R_00| <= sigma_1 <= sqrt(c) |R_00| bracketing the thresholds) at least a
    # quarter of them agree exactly -- a rule that kept one column too many
    # would agree on none.
    ph = I.dft_phase() if kind == "dft" else I.fio_phase(1.0, 1.0 if kind == "fio" else 2.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, tol, sample_all=True)
    d = []
    for rec, B in _full_blocks(F, ph, X, O):
        sv = np.linalg.svd(B, compute_uv=False)
        d.append(len(rec.skel) - np.count_nonzero(sv > tol * sv[0]))
    d = np.array(d)
    assert len(d) == 2 * F.H * (2 * N // leaf)
    assert np.mean(np.abs(d) <= 2) >= 0.95
    assert np.mean(d == 0) >= 0.25
