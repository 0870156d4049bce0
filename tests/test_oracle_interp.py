"""Pins of the oracle's interpolative decomposition (Lemma 2.1; eqs. pivotedQR2, acc, R2)."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle


def _cgauss(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("s,c", [(24, 24), (40, 17), (12, 30), (64, 52)])
def test_pivots_and_rdiag_match_lapack_geqp3(s, c):
    rng = np.random.default_rng(s * 100 + c)
    B = _cgauss(rng, s, c)
    cid = oracle.column_id(B, tol=0.0)
    _, R, P = sl.qr(B, pivoting=True, mode="economic")
    k = min(s, c)
    assert cid.rank == k
    assert np.array_equal(cid.pivots, P[:k])
    assert np.allclose(cid.rdiag, np.abs(np.diag(R))[:k], rtol=1e-12)


@pytest.mark.parametrize("s,c,r", [(30, 20, 7), (20, 30, 11), (64, 64, 25)])
def test_exact_low_rank_is_recovered(s, c, r):
    rng = np.random.default_rng(r)
    B = _cgauss(rng, s, r) @ _cgauss(rng, r, c)
    cid = oracle.column_id(B, tol=1e-10)
    assert cid.rank == r
    err = np.linalg.norm(B[:, cid.red] - B[:, cid.skel] @ cid.T) / np.linalg.norm(B)
    assert err < 1e-12


def test_skeleton_columns_reproduced_exactly():
    # V = [I T] Lambda^*: the skeleton columns of A_{:,q} V are A_{:,q} itself, bit for bit
    rng = np.random.default_rng(1)
    B = _cgauss(rng, 20, 15) @ np.diag(np.logspace(0, -12, 15)) @ _cgauss(rng, 15, 15)
    cid = oracle.column_id(B, tol=1e-6)
    V = np.zeros((cid.rank, B.shape[1]), dtype=np.complex128)
    V[:, cid.skel] = np.eye(cid.rank)
    V[:, cid.red] = cid.T
    approx = B[:, cid.skel] @ V
    assert np.array_equal(approx[:, cid.skel], B[:, cid.skel])
    assert np.all(np.diff(cid.skel) > 0) and np.all(np.diff(cid.red) > 0)
    assert sorted(np.concatenate([cid.skel, cid.red]).tolist()) == list(range(15))


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
def test_stopping_rule_bounds(tol):
    # Stopping when every residual column norm is <= tol |R_00| gives
    #   ||B_red - B_skel T||_F = ||R_22||_F <= sqrt(c - k) tol |R_00|   and
    #   sigma_{k+1}(B) <= ||R_22||_2, |R_00| <= sigma_1  =>  k >= #{sigma_i > sqrt(c) tol sigma_1}.
    rng = np.random.default_rng(42)
    for trial in range(20):
        s, c = rng.integers(8, 60, 2)
        decay = np.logspace(0, rng.uniform(-14, -2), min(s, c))
        B = (_cgauss(rng, s, len(decay)) * decay) @ _cgauss(rng, len(decay), c)
        cid = oracle.column_id(B, tol=tol)
        k = cid.rank
        r00 = cid.rdiag[0]
        resid = np.linalg.norm(B[:, cid.red] - B[:, cid.skel] @ cid.T)
        assert resid <= np.sqrt(c - k) * tol * r00 * (1 + 1e-6) + 1e-13 * r00
        sv = np.linalg.svd(B, compute_uv=False)
        assert k >= np.count_nonzero(sv > np.sqrt(c) * tol * sv[0])
        assert np.all(cid.rdiag > tol * r00)


@pytest.mark.parametrize("perm", [[0, 1, 2, 3, 4], [3, 0, 4, 2, 1], [4, 3, 2, 1, 0]])
def test_eps_rank_count_on_known_diagonal(perm):
    # Columns with a single nonzero each: every Householder step is exact, the
    # pivots follow decreasing norm and |R_jj| are the norms themselves.  With
    # norms 1, 2^-10, 2^-20, 2^-30, 2^-40 and eps = 2^-20, eq. (acc)'s
    # stopping index is the first |R_jj| <= eps |R_00|, i.e. the third pivot
    # (2^-20, equal to the threshold).  The count kept is the entries strictly
    # above it: 2.  Keeping the stopping column as well (the literal index),
    # or comparing with >=, would give 3.
    d = 2.0 ** -np.array([0, 10, 20, 30, 40])
    B = np.zeros((7, 5), dtype=np.complex128)
    B[np.arange(5), np.arange(5)] = d * np.exp(1j * np.arange(5))
    B = B[:, perm]
    cid = oracle.column_id(B, tol=2.0 ** -20)
    assert cid.rank == 2
    assert list(cid.pivots) == [perm.index(0), perm.index(1)]
    assert np.array_equal(cid.rdiag, d[:2])
    # eps just above the third norm keeps two, just below it keeps three
    assert oracle.column_id(B, tol=2.0 ** -20 * (1 + 2.0 ** -40)).rank == 2
    assert oracle.column_id(B, tol=2.0 ** -20 * (1 - 2.0 ** -40)).rank == 3


def test_tie_rule_prefers_smallest_index():
    # every column has the same norm: the first pivot is the first column; a
    # column permutation moves the pivot with it only through the index order
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(_cgauss(rng, 6, 6))
    B = Q[:, :4] * 2.0                          # equal norms, orthogonal columns
    cid = oracle.column_id(B, tol=0.0)
    assert list(cid.pivots) == [0, 1, 2, 3]
    cid2 = oracle.column_id(B[:, [2, 0, 3, 1]], tol=0.0)
    assert list(cid2.pivots) == [0, 1, 2, 3]


def test_zero_block_and_rank_cap():
    z = oracle.column_id(np.zeros((5, 4)), tol=1e-6)
    assert z.rank == 1 and list(z.skel) == [0] and np.all(z.T == 0)
    rng = np.random.default_rng(9)
    B = _cgauss(rng, 20, 20)
    cap = oracle.column_id(B, tol=0.0, kmax=5)
    assert cap.rank == 5 and cap.T.shape == (5, 15)


def test_row_id_by_transpose():
    # rID of A (Section 2.1): A ~= Lambda [I T]^T A_{q,:}, from the cID of A^T
    rng = np.random.default_rng(8)
    A = _cgauss(rng, 16, 6) @ _cgauss(rng, 6, 40)
    cid = oracle.column_id(A.T, tol=1e-12)
    U = np.zeros((16, cid.rank), dtype=np.complex128)
    U[cid.skel] = np.eye(cid.rank)
    U[cid.red] = cid.T.T
    assert cid.rank == 6
    assert np.linalg.norm(A - U @ A[cid.skel]) / np.linalg.norm(A) < 1e-12


@pytest.mark.parametrize("s,c,r", [(200, 90, 30), (256, 128, 50), (150, 40, 12)])
def test_row_reduction_keeps_the_id(s, c, r):
    # Tall sample blocks may be reduced to their triangular factor R0 (B = Q0 R0)
    # before the pivoted QR: the pivots follow the norms of the columns'
    # components orthogonal to those already chosen, which depend on B only
    # through B^H B = R0^H R0, so the ID of R0 has B's skeleton and T.
    rng = np.random.default_rng(s + c)
    B = (_cgauss(rng, s, c) * np.logspace(0, -16 * c / r, c)) @ _cgauss(rng, c, c)
    R0 = sl.qr(B, mode="r")[0][:c]
    for tol in (1e-6, 1e-10):
        a, b = oracle.column_id(B, tol), oracle.column_id(R0, tol)
        assert 0 < a.rank < c
        assert np.array_equal(a.skel, b.skel)
        assert np.allclose(a.rdiag, b.rdiag, rtol=1e-10)
        kappa = a.rdiag[0] / a.rdiag[-1]
        assert np.max(np.abs(a.T - b.T)) <= 1e-12 * kappa * max(1.0, np.abs(a.T).max())


def test_restricted_id_without_restriction_is_the_plain_id():
    # among = every column, or exactly the plain ID's own pivots: the pivot
    # search finds the same column at every step, so the same arithmetic
    rng = np.random.default_rng(5)
    B = (_cgauss(rng, 40, 30) * np.logspace(0, -12, 30)) @ _cgauss(rng, 30, 30)
    a = oracle.column_id(B, 1e-8)
    for among in (np.arange(30), a.pivots, a.pivots[::-1]):
        b = oracle.column_id(B, 1e-8, among=among)
        assert np.array_equal(a.pivots, b.pivots) and np.array_equal(a.skel, b.skel)
        assert np.array_equal(a.T, b.T) and np.array_equal(a.rdiag, b.rdiag)


def test_restricted_id_first_pivot_and_threshold_by_brute_force():
    # first pivot: the largest column of the proposal; the eps rule is taken
    # against the largest column of all of B, not of the proposal
    rng = np.random.default_rng(7)
    B = _cgauss(rng, 12, 8) * np.array([1.0, 5.0, 0.5, 2.0, 3.0, 0.1, 4.0, 1e-4])
    among = [0, 2, 3, 7]
    cid = oracle.column_id(B, 1e-6, among=among)
    nrm = np.linalg.norm(B, axis=0)
    assert cid.pivots[0] == among[int(np.argmax(nrm[among]))]
    assert sorted(cid.pivots) == among and cid.rank == 4
    # |B_7| ~ 1e-4 stays below 1e-3 max|B_l| (max|B_l| is column 1's, outside
    # the proposal): column 7 is not kept, the other three are
    cid = oracle.column_id(B, 1e-3, among=among)
    assert sorted(cid.pivots) == [0, 2, 3]
    assert oracle.column_id(B, 1e-2, among=[7]) is None       # nothing kept: unusable


@pytest.mark.parametrize("s,c,r", [(30, 20, 7), (40, 33, 12), (16, 16, 5)])
def test_restricted_id_on_exact_low_rank(s, c, r):
    # B exactly of rank r: a proposal that spans it (r + 5 generic columns)
    # keeps exactly r of them, which interpolate the rest exactly with T the
    # least-squares solution B[:, skel]^+ B[:, red]
    rng = np.random.default_rng(s + c)
    B = _cgauss(rng, s, r) @ _cgauss(rng, r, c)
    among = rng.choice(c, min(c, r + 5), replace=False)
    cid = oracle.column_id(B, 1e-10, among=among)
    assert cid.rank == r and set(cid.skel) <= set(among)
    err = np.linalg.norm(B[:, cid.red] - B[:, cid.skel] @ cid.T) / np.linalg.norm(B)
    assert err < 1e-12
    ls = np.linalg.lstsq(B[:, cid.skel], B[:, cid.red], rcond=None)[0]
    assert np.allclose(cid.T, ls, atol=1e-10 * max(1.0, np.abs(ls).max()))
    # a proposal that misses a direction keeps what it spans and leaves a
    # large residual (what the acceptance test then sees)
    cid = oracle.column_id(B, 1e-10, among=among[:r - 2])
    assert cid.rank == r - 2
    assert np.linalg.norm(B[:, cid.red] - B[:, cid.skel] @ cid.T) / np.linalg.norm(B) > 1e-3


def test_restricted_id_keeps_the_rank_of_a_dependent_proposal():
    # three proposed columns spanning two dimensions: two are kept (the
    # largest first), and the third gets its exact coefficients in T
    rng = np.random.default_rng(6)
    B = _cgauss(rng, 20, 10)
    B[:, 3] = 2.0 * B[:, 1] - 1j * B[:, 7]
    cid = oracle.column_id(B, 1e-12, among=[1, 7, 3])
    assert cid.rank == 2 and cid.pivots[0] == 3
    (dep,) = [l for l in (1, 7) if l in cid.red]
    t = cid.T[:, list(cid.red).index(dep)]
    coef = np.linalg.lstsq(B[:, cid.skel], B[:, dep], rcond=None)[0]
    assert np.allclose(t, coef, rtol=0, atol=1e-12)
    assert np.linalg.norm(B[:, cid.skel] @ t - B[:, dep]) < 1e-12 * np.linalg.norm(B[:, dep])


def test_restricted_id_degenerate_cases():
    rng = np.random.default_rng(8)
    B = _cgauss(rng, 12, 6)
    B[:, 4] = 0.0
    assert oracle.column_id(B, 1e-12, among=[4]) is None                 # nothing kept: unusable
    Z = oracle.column_id(np.zeros((5, 4)), 1e-6, among=[2])              # zero block: the plain convention
    ref = oracle.column_id(np.zeros((5, 4)), 1e-6)
    assert np.array_equal(Z.skel, ref.skel) and np.array_equal(Z.T, ref.T)
    for bad in ([1, 1], [6], []):
        with pytest.raises(ValueError):
            oracle.column_id(B, 1e-6, among=bad)