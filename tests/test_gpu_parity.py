"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances are derived from the arithmetic:
* entries: the phase is reduced modulo 1 exactly on both sides except for c(x)
  itself (GPU sinpi vs host sin, a few ulps): |dK| <= 2 pi (|xi| * 8 ulp(1) * a/cdiv + 1e-15) + 1e-15;
* T = R11^{-1} R12: perturbations of the sampled block are amplified by the
  conditioning of R11, bounded by |R_00| / |R_kk|;
* apply: products of O(log N) factors in FP64 (c128) or FP32 (c64).
"""
import functools

import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_10573_amd import binding as B  # noqa: E402

DEV = "cuda:0"


def _entry_tol(phase, N, nonuniform=False):
    amp = 0.0 if phase.kind == I.PHASE_DFT else abs(phase.a) / abs(phase.cdiv)
    # on random reals the oracle's extended-precision product carries <= 2^-64 N/2 turns
    prod = 2.0 ** -64 * (N / 2) if nonuniform else 0.0
    return 2 * np.pi * ((N / 2) * 8 * 2.2e-16 * amp + prod + 1e-15) + 1e-15


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("kind,N", [("dft", 1024), ("fio", 1024), ("dft", 1 << 20), ("fio", 1 << 20),
                                    ("nufft", 1 << 20)])
def test_sampler_matches_oracle(kind, N):
    ph, X, O = _workload(kind, N)
    rng = np.random.default_rng(N + len(kind))
    rows = np.sort(rng.choice(N, 97, replace=False))
    cols = np.sort(np.concatenate([rng.choice(N, 60, replace=False), [0, N // 2, N - 1]]))
    cols = np.unique(cols)
    got = B.sample(ph, X, O, rows, cols, device=DEV).cpu().numpy()
    ref = oracle.entries(ph, X, O, rows, cols)
    assert np.max(np.abs(got - ref)) <= _entry_tol(ph, N, nonuniform=(kind == "nufft"))


@pytest.mark.parametrize("N", [1024, 1 << 20])
def test_j0_sampler_matches_oracle(N):
    """Example 2's J_0(g w) entries: both sides run Miller's recurrence below
    25 and Hankel's expansion above in the same operation order, so they
    agree to the rounding of sin, cos and sqrt (relative to the envelope
    sqrt(2 / (pi z)) of J_0); the first row is J_0(0) = 1 and rows near the
    top cross z = 25."""
    ph, g, w = _workload("j0", N)
    rng = np.random.default_rng(N)
    rows = np.unique(np.concatenate([rng.choice(N, 90, replace=False), [0, 1, 2, N - 1]]))
    cols = np.unique(np.concatenate([rng.choice(N, 60, replace=False), [0, 1, 7, N - 1]]))
    got = B.sample(ph, g, w, rows, cols, device=DEV).cpu().numpy()
    ref = oracle.entries(ph, g, w, rows, cols)
    z = np.outer(g[rows], w[cols])
    amp = np.minimum(1.0, np.sqrt(2.0 / (np.pi * np.maximum(z, 1e-300))))
    assert np.all(got.imag == 0)
    assert np.max(np.abs(got - ref) / amp) < 1e-14
    assert np.any(z < 25) and np.any(z >= 25)


def test_sampler_empty():
    X, O = I.uniform_grid(64)
    got = B.sample(I.dft_phase(), X, O, np.zeros(0, np.int32), np.arange(5), device=DEV)
    assert got.shape == (0, 5)


# ------------------------------------------------------------------ batched ID
def _id_problem(rng, N, c, wc, na, wa):
    """Candidates: c of a window of wc grid points; allowed: na of a window of wa
    points elsewhere.  wc * wa / N bounds the block's time-frequency product, as
    for the complementary blocks the construction meets."""
    c0 = int(rng.integers(0, N - wc))
    a0 = int(rng.integers(0, N - wa))
    cand = np.sort(c0 + rng.choice(wc, c, replace=False))
    allowed = np.sort(a0 + rng.choice(wa, na, replace=False))
    return cand, allowed


def _run_ids(ph, X, O, side, problems, tol, kmax, oversample):
    cands = [p[0] for p in problems]
    alloweds = [p[1] for p in problems]
    cb = np.cumsum([0] + [len(x) for x in cands[:-1]])
    ab = np.cumsum([0] + [len(x) for x in alloweds[:-1]])
    return B.id_batch(ph, X, O, side, np.concatenate(cands), cb, [len(x) for x in cands],
                      np.concatenate(alloweds), ab, [len(x) for x in alloweds], tol, kmax,
                      oversample, device=DEV)


NARROW_SHAPES = [(8, 8, 5, 5), (16, 16, 16, 16), (16, 16, 700, 2048), (24, 32, 30, 40),
                 (33, 40, 700, 800), (52, 64, 60, 64), (64, 128, 64, 100), (5, 5, 1, 1),
                 (40, 48, 128, 300), (17, 20, 1500, 1600), (1, 1, 50, 60), (12, 12, 12, 12),
                 (28, 28, 2000, 2048), (60, 64, 90, 90)]
# more than 64 candidates (two per lane, 8 rows per wavefront); a batch holding
# any of them runs every ID on that kernel variant
WIDE_SHAPES = [(96, 120, 150, 400), (70, 80, 60, 64), (128, 128, 200, 256), (65, 300, 90, 120),
               (100, 110, 1000, 1100), (16, 16, 700, 2048), (40, 48, 128, 300), (3, 3, 8, 8)]


# small IDs run several to a workgroup: up to 16 candidates and 32 samples
# four per workgroup, up to 32 and 64 two per workgroup; odd counts leave the
# last workgroup part empty, and the IDs differ in size and rank
PACKED4_SHAPES = [(16, 16, 700, 2048), (8, 8, 5, 5), (5, 5, 1, 1), (1, 1, 50, 60), (12, 12, 12, 12),
                  (3, 3, 8, 8), (16, 20, 30, 40)]
PACKED2_SHAPES = [(24, 32, 30, 40), (28, 28, 2000, 2048), (17, 20, 1500, 1600), (32, 32, 64, 70),
                  (20, 24, 40, 48)]
SHAPES = {"narrow": NARROW_SHAPES, "wide": WIDE_SHAPES, "packed4": PACKED4_SHAPES, "packed2": PACKED2_SHAPES}


@pytest.mark.parametrize("side", [B.SIDE_U, B.SIDE_V])
@pytest.mark.parametrize("oversample,kmax", [(1, 0), (2, 0), (2, 7)])
@pytest.mark.parametrize("shapes", ["narrow", "wide", "packed4", "packed2"])
def test_id_batch_matches_oracle(side, oversample, kmax, shapes):
    N = 4096
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    rng = np.random.default_rng(10 * side + oversample + kmax + 100 * list(SHAPES).index(shapes))
    problems = [_id_problem(rng, N, *sh) for sh in SHAPES[shapes]]
    tol = 1e-6
    _assert_ids_match_oracle(ph, X, O, side, problems, tol, kmax, oversample)


def _assert_ids_match_oracle(ph, X, O, side, problems, tol, kmax, oversample):
    """One batched launch over the problems against oracle.column_id on the
    same Mock-Chebyshev samples: ranks, skeletons and masks identical, T
    within the conditioning bound."""
    rank, mask, skel, T = _run_ids(ph, X, O, side, problems, tol, kmax, oversample)
    allow_coord = X if side == B.SIDE_V else O
    for q, (cand, allowed) in enumerate(problems):
        s = oracle.sample_count(len(cand), len(allowed), oversample)
        samp = allowed[oracle.mock_chebyshev(allow_coord[allowed], s)]
        Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
              else oracle.entries(ph, X, O, cand, samp).T)
        cid = oracle.column_id(Bm, tol, kmax)
        k = cid.rank
        assert rank[q] == k, (q, rank[q], k)
        assert np.array_equal(skel[q, :k], cand[cid.skel]), q
        bits = B.mask_bits(mask[q], len(cand))
        assert np.array_equal(np.nonzero(bits)[0], cid.skel)
        r = len(cand) - k
        flat = T[q, :k * r]
        Tg = flat.reshape(r, k).T if side == B.SIDE_V else flat.reshape(k, r)
        kappa = cid.rdiag[0] / cid.rdiag[-1]
        scale = max(1.0, np.abs(cid.T).max()) if r else 1.0
        assert np.max(np.abs(Tg - cid.T), initial=0.0) <= 1e-12 * kappa * scale, q


@pytest.mark.parametrize("side", [B.SIDE_U, B.SIDE_V])
@pytest.mark.parametrize("rows", [65, 80, 81, 96, 97, 112])
def test_id_batch_four_wave_shapes(side, rows):
    """65..80, 81..96 and 97..112 sampled rows of up to 64 candidates run as
    four wavefronts of 20, 24 and 28 rows.  A launch takes the batch's largest
    block, so the first and last IDs here sit exactly on a bucket edge (80, 96
    and 112 fill every row of the four wavefronts; 65, 81 and 97 leave all but
    one row of the last wavefront empty), and the others are ragged below."""
    N = 4096
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    rng = np.random.default_rng(rows + 1000 * side)
    # oversampling 2: s = min(2 c, |allowed|)
    shapes = [(56, 64, rows, rows + 20), (rows // 2, rows // 2 + 4, 400, 600), (33, 40, rows - 1, rows + 5),
              (9, 9, 300, 400), (64, 64, rows, 2 * rows)]
    problems = [_id_problem(rng, N, *sh) for sh in shapes]
    assert max(oracle.sample_count(len(c), len(a), 2) for c, a in problems) == rows
    _assert_ids_match_oracle(ph, X, O, side, problems, 1e-6, 0, 2)


# tall sample blocks (more than 128 sampled rows): the library first reduces
# them to their c x c triangular factor; oversampling 3 and 5 make them tall
# at small candidate counts too, mixed with IDs that are not
TALL_SHAPES = {3: [(60, 64, 300, 400), (50, 70, 151, 200), (64, 64, 256, 300), (20, 24, 30, 40),
                   (80, 100, 400, 500), (8, 8, 700, 800)],
               5: [(30, 32, 700, 800), (16, 16, 40, 48), (8, 8, 5, 5), (27, 30, 140, 200), (32, 32, 160, 160),
                   (51, 60, 500, 600)]}


@pytest.mark.parametrize("side", [B.SIDE_U, B.SIDE_V])
@pytest.mark.parametrize("oversample,packed", [(3, False), (5, False), (5, True)])
def test_id_batch_tall_blocks(side, oversample, packed):
    """s = t |cand| up to 256 rows (eq. pivotedQR2 without a cap): the reduced
    blocks give the oracle's skeletons and T.  `packed`: only the IDs of at
    most 32 candidates, so that the batch would otherwise run on the
    several-IDs-per-workgroup kernels."""
    N = 4096
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    shapes = [sh for sh in TALL_SHAPES[oversample] if not packed or sh[0] <= 32]
    rng = np.random.default_rng(7 + side + 10 * oversample + 100 * packed)
    problems = [_id_problem(rng, N, *sh) for sh in shapes]
    tol = 1e-6
    rank, mask, skel, T = _run_ids(ph, X, O, side, problems, tol, 0, oversample)
    allow_coord = X if side == B.SIDE_V else O
    tall = 0
    for q, (cand, allowed) in enumerate(problems):
        s = oracle.sample_count(len(cand), len(allowed), oversample)
        tall += s > 128
        samp = allowed[oracle.mock_chebyshev(allow_coord[allowed], s)]
        Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
              else oracle.entries(ph, X, O, cand, samp).T)
        cid = oracle.column_id(Bm, tol)
        k = cid.rank
        assert rank[q] == k, (q, rank[q], k)
        assert np.array_equal(skel[q, :k], cand[cid.skel]), q
        r = len(cand) - k
        flat = T[q, :k * r]
        Tg = flat.reshape(r, k).T if side == B.SIDE_V else flat.reshape(k, r)
        kappa = cid.rdiag[0] / cid.rdiag[-1]
        scale = max(1.0, np.abs(cid.T).max()) if r else 1.0
        assert np.max(np.abs(Tg - cid.T), initial=0.0) <= 1e-12 * kappa * scale, q
    assert tall >= 2


def test_id_batch_rejects_more_than_256_samples():
    # s = 3 * 128 = 384 sampled rows exceeds the supported 256: reported, not capped
    N = 4096
    X, O = I.uniform_grid(N)
    rng = np.random.default_rng(5)
    prob = _id_problem(rng, N, 128, 130, 500, 600)
    with pytest.raises(B.IdbfError) as e:
        _run_ids(I.fio_phase(1.0, 1.0), X, O, B.SIDE_V, [prob], 1e-6, 0, 3)
    assert e.value.status == B.EUNSUPPORTED


def test_id_batch_rank_overflow_is_reported():
    # 128 candidates spread over the whole grid against 128 spread allowed
    # points: full rank, above the 64 an ID may have -> IDBF_ERANK, not a wrong answer
    N = 4096
    X, O = I.uniform_grid(N)
    rng = np.random.default_rng(3)
    prob = (np.sort(rng.choice(N, 128, replace=False)), np.sort(rng.choice(N, 128, replace=False)))
    with pytest.raises(B.IdbfError) as e:
        _run_ids(I.dft_phase(), X, O, B.SIDE_V, [prob], 1e-6, 0, 1)
    assert e.value.status == B.ERANK
    rank, _, _, _ = _run_ids(I.dft_phase(), X, O, B.SIDE_V, [prob], 1e-6, 20, 1)
    assert rank[0] == 20


def test_id_batch_rejects_oversized():
    N = 1024
    X, O = I.uniform_grid(N)
    with pytest.raises(B.IdbfError) as e:
        B.id_batch(I.dft_phase(), X, O, B.SIDE_V, np.arange(129), [0], [129], np.arange(200), [0],
                   [200], 1e-6, device=DEV)
    assert e.value.status == B.EINVAL


# ------------------------------------------------------------------ construction
def _workload(kind, N):
    """Phase and points: the DFT or FIO kernel on the uniform grid, or Example
    3's non-uniform Fourier transform (DFT phase, rows at random frequencies,
    columns at random points)."""
    if kind == "nufft":
        W, Xp = I.nufft_points(N, seed=N + 1)
        return I.dft_phase(), W, Xp
    if kind == "j0":
        g, w = I.schlomilch_points(N)
        return I.j0_kernel(), g, w
    X, O = I.uniform_grid(N)
    if kind == "fio_m4":
        return I.fio_phase(1.0, 4.0), X, O
    return (I.dft_phase() if kind == "dft" else I.fio_phase(1.0, 1.0)), X, O


@functools.lru_cache(maxsize=8)
def _oracle_case(kind, N, leaf, tol, os_):
    """The workload and its oracle factors, built once per configuration:
    oracle.build is deterministic and oracle.apply only reads the factors,
    so the right-hand-side parametrizations share one build."""
    ph, X, O = _workload(kind, N)
    return ph, X, O, oracle.build(ph, X, O, leaf, tol, oversample=os_)


def _compare_construction(F, fac, ph, X, O, t_bound=1e-12):
    """Level-by-level comparison of GPU factors with the oracle's.

    Skeletons must agree exactly.  T = R11^{-1} R12 may differ by the sampled
    entries' perturbation amplified by R11's conditioning: the bound used is
    1e-12 * (|R_00| / |R_kk|) * max(1, max |T|)."""
    L, H = F.L, F.H
    mismatched = 0
    for t in range(1, H + 1):
        nn = 1 << (L - t + 1)
        for side, recs in ((B.SIDE_U, F.U[t]), (B.SIDE_V, F.V[t])):
            b = fac.batch(side, t)
            offs = np.concatenate([[0], np.cumsum(b.rank)])
            for q in range(len(b.rank)):
                rec = recs[(q % nn, q // nn)]
                k = len(rec.skel)
                assert b.cand_len[q] == len(rec.cand)
                gs = b.skel[offs[q]:offs[q + 1]]
                if b.rank[q] != k or not np.array_equal(gs, rec.skel):
                    mismatched += 1
                    continue
                r = len(rec.cand) - k
                flat = b.T[b.T_off[q]:b.T_off[q] + k * r]
                Tg = flat.reshape(r, k).T if side == B.SIDE_V else flat.reshape(k, r)
                scale = max(1.0, np.abs(rec.T).max(initial=0.0))
                kappa = rec.rdiag[0] / rec.rdiag[-1]
                if t_bound is not None:
                    assert np.max(np.abs(Tg - rec.T), initial=0.0) <= t_bound * kappa * scale
    return mismatched


@pytest.mark.parametrize("N,leaf,kind,tol,os_", [
    (1024, 8, "dft", 1e-10, 1),     # the DFT workload: L = 7 (odd), H = 3
    (16, 8, "dft", 1e-10, 1),       # L = 1: no levels, S = K
    (64, 16, "fio", 1e-6, 2),       # L = 2, H = 1
    (256, 2, "fio", 1e-8, 1),       # L = 7 with leaf 2
    (2048, 16, "fio", 1e-6, 2),     # the FIO workload's shape at a small N
    (1024, 4, "fio", 1e-4, 1),
    (2048, 16, "nufft", 1e-6, 2),   # Example 3: random points, the workload's leaf and t
    (1024, 8, "nufft", 1e-10, 1),
    (1024, 8, "j0", 1e-10, 2),      # Example 2: the Schloemilch kernel J_0(g w)
    (2048, 16, "j0", 1e-6, 2),
    (1024, 32, "dft", 1e-10, 5),    # every ID samples more than 128 rows (up to 248)
    (1024, 64, "dft", 1e-6, 4),     # tall IDs of up to 90 candidates and 256 rows
])
def test_construct_and_apply_match_oracle(N, leaf, kind, tol, os_):
    ph, X, O = _workload(kind, N)
    F = oracle.build(ph, X, O, leaf, tol, oversample=os_)
    fac = B.construct(ph, X, O, tol, leaf, oversample=os_, device=DEV)
    info = fac.info()
    assert (info["L"], info["H"]) == (F.L, F.H)
    assert _compare_construction(F, fac, ph, X, O) == 0
    assert info["nnz_T"] + info["nnz_S"] >= F.nnz()
    g = I.gaussian_vectors(N, None, seed=N)
    y_or = oracle.apply(F, g)
    x = torch.as_tensor(g, device=DEV)
    y128 = fac.apply(x).cpu().numpy()
    assert oracle.relative_error(y128, y_or) < 1e-12
    y64 = fac.apply(x.to(torch.complex64)).cpu().numpy()
    assert oracle.relative_error(y64, y_or) < 2e-6
    # against the exact matvec
    y_ex = (oracle.dft_closed_form(g) if kind == "dft" else oracle.dense_matvec(ph, X, O, g))
    assert oracle.relative_error(y128, y_ex) < max(100 * tol, 1e-12)


def test_apply_many_rhs_and_repeat():
    N, leaf, tol = 2048, 16, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    F = oracle.build(ph, X, O, leaf, tol, oversample=2)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    G = I.gaussian_vectors(N, 67, seed=5)          # a ragged right-hand-side count
    Y_or = oracle.apply(F, G)
    Gd = torch.as_tensor(G, device=DEV)
    Y = fac.apply(Gd).cpu().numpy()
    assert oracle.relative_error(Y, Y_or) < 1e-12
    Y2 = fac.apply(Gd).cpu().numpy()
    assert np.array_equal(Y, Y2)                    # deterministic: no atomics
    Y64 = fac.apply(Gd.to(torch.complex64)).cpu().numpy()
    assert oracle.relative_error(Y64, Y_or) < 2e-6
    one = fac.apply(Gd[:, 3].contiguous()).cpu().numpy()
    assert oracle.relative_error(one, Y_or[:, 3]) < 1e-12
    empty = torch.zeros((N, 0), dtype=torch.complex128, device=DEV)
    assert fac.apply(empty).shape == (N, 0)


@pytest.mark.parametrize("N,leaf,kind,tol,os_", [
    (1024, 8, "dft", 1e-10, 1),     # odd L: the middle stage has 4 blocks per output
    (16, 8, "dft", 1e-10, 1),       # H = 0: dense
    (2048, 16, "fio", 1e-6, 2),
    (256, 2, "fio", 1e-8, 1),
    (2048, 16, "nufft", 1e-6, 2),
])
@pytest.mark.parametrize("nrhs", [2, 65, 300, 1024, 1100])
def test_many_rhs_matrix_core_paths(N, leaf, kind, tol, os_, nrhs):
    """complex64 apply on the matrix cores (FP32 MFMA, and BF16 hi/lo split
    products with FP32 accumulation) against the oracle's FP64 apply of its
    own factors (identical skeletons, so the factors agree to 1e-12); ragged
    right-hand-side counts cover the tails of the 64-column blocks."""
    ph, X, O, F = _oracle_case(kind, N, leaf, tol, os_)
    fac = B.construct(ph, X, O, tol, leaf, oversample=os_, device=DEV)
    G = I.gaussian_vectors(N, nrhs, seed=nrhs)
    Y_or = oracle.apply(F, G)
    x = torch.as_tensor(G, device=DEV).to(torch.complex64)
    for dtype, bound in ((B.C64, 2e-6), (B.C64_BF16X3, 2e-4)):
        Y = fac.apply(x, dtype=dtype).cpu().numpy()
        assert oracle.relative_error(Y, Y_or) < bound
        col = np.linalg.norm(Y - Y_or, axis=0) / np.linalg.norm(Y_or, axis=0)
        assert col.max() < 10 * bound       # every column, tails included


def _expected_fused_launches(levels, H):
    """Stage pairs the apply fuses, from the documented rule: greedy from
    V_1 up and from U_H down, a pair where both levels' ranks are <= 32, the
    second stage's output rows <= 64 and the four staged blocks fit 152 KiB
    of LDS (FP32 complex, 16-row tiles, rows padded to 16 plus 2)."""
    lda = lambda K: ((K + 15) & ~15) + 2
    def ok(r1, r2, kmax1, mmax2):
        r = max(r1, r2)
        tk = 1 if r <= 16 else 2 if r <= 32 else 0
        lds = 8 * (2 * 32 * tk * lda(kmax1) + 2 * ((mmax2 + 15) & ~15) * lda(32 * tk))
        return tk > 0 and kmax1 <= 256 and mmax2 <= 64 and lds <= 152 * 1024
    n, t = 0, 1
    while t <= H:
        a, b = levels[t - 1]["V"], levels[t]["V"] if t < H else None
        if b is not None and ok(a["rank_max"], b["rank_max"], a["cand_max"], 2 * b["rank_max"]):
            n, t = n + 1, t + 2
        else:
            t += 1
    t = H
    while t >= 1:
        a, b = levels[t - 1]["U"], levels[t - 2]["U"] if t > 1 else None
        if b is not None and ok(a["rank_max"], b["rank_max"], 2 * a["rank_max"], b["cand_max"]):
            n, t = n + 1, t - 2
        else:
            t -= 1
    return n


@pytest.mark.parametrize("N,leaf,kind,tol,os_,fusable", [
    (2048, 16, "fio", 1e-6, 2, True),     # H = 3: one V pair, one U pair, one stage each left over
    (4096, 16, "fio", 1e-6, 2, True),     # H = 4: every stage in a pair
    (1024, 8, "dft", 1e-10, 1, True),     # ranks <= 16: one register tile per part
    (256, 2, "fio", 1e-8, 1, True),
    (4096, 16, "fio_m4", 1e-6, 2, False),  # ranks above 32: one launch per stage
])
@pytest.mark.parametrize("nrhs", [2, 65, 1100])
def test_fused_stage_groups(N, leaf, kind, tol, os_, fusable, nrhs):
    """The fused two-stage groups of the complex64 many-RHS apply against the
    oracle's FP64 apply and against the per-stage kernels on the same
    factors; the right-hand-side blocking changes no bit of the result."""
    ph, X, O, F = _oracle_case(kind, N, leaf, tol, os_)
    fac = B.construct(ph, X, O, tol, leaf, oversample=os_, device=DEV, profile=True)
    assert fac.apply_config() == {"fuse": 0, "rhs_iter": 0}
    fac.set_apply_config(fuse=1)
    G = I.gaussian_vectors(N, nrhs, seed=3 + nrhs)
    Y_or = oracle.apply(F, G)
    x = torch.as_tensor(G, device=DEV).to(torch.complex64)
    fac.profile(reset=True)
    Yf = fac.apply(x)
    prof = fac.profile(reset=True)
    fused = prof.get("applyn_vv", {}).get("launches", 0) + prof.get("applyn_uu", {}).get("launches", 0)
    H = fac.info()["H"]
    expect = _expected_fused_launches(fac.stats()["per_level"], H)
    assert fused == expect
    assert (expect == 2 * (H // 2)) if fusable else (0 < expect < 2 * (H // 2)), expect
    yf = Yf.cpu().numpy()
    assert oracle.relative_error(yf, Y_or) < 2e-6
    col = np.linalg.norm(yf - Y_or, axis=0) / np.linalg.norm(Y_or, axis=0)
    assert col.max() < 2e-5
    # BF16 hi/lo split products: the same groups on the 16x16x16 BF16 matrix cores
    Yb = fac.apply(x, dtype=B.C64_BF16X3)
    prof = fac.profile(reset=True)
    fused_b = prof.get("applyb_vv", {}).get("launches", 0) + prof.get("applyb_uu", {}).get("launches", 0)
    assert fused_b == expect
    yb = Yb.cpu().numpy()
    assert oracle.relative_error(yb, Y_or) < 2e-4
    fac.set_apply_config(fuse=0)
    Ys = fac.apply(x)
    assert fac.profile(reset=True).get("applyn_vv") is None
    assert oracle.relative_error(yf, Ys.cpu().numpy()) < 1e-6
    Ysb = fac.apply(x, dtype=B.C64_BF16X3).cpu().numpy()
    assert oracle.relative_error(yb, Ysb) < 1e-4
    fac.set_apply_config(fuse=1)
    for r in (1, 2, 16):
        fac.set_apply_config(rhs_iter=r)
        assert torch.equal(fac.apply(x), Yf), r
        assert torch.equal(fac.apply(x, dtype=B.C64_BF16X3), Yb), r
    with pytest.raises(B.IdbfError):
        fac.set_apply_config(rhs_iter=3)
    assert fac.apply_config() == {"fuse": 1, "rhs_iter": 16}


def test_wide_ranks_construct_and_every_apply_path():
    """c(x) = (2 + sin 8 pi x)/8 at N = 4096 (leaf 16, tol 1e-6, t = 2): ranks
    reach the 40s and candidate sets exceed 64, so the two-candidates-per-lane
    QR variant, the chunked back-substitution and the 128-bit skeleton masks
    all run; every apply path is checked against the oracle."""
    N, leaf, tol = 4096, 16, 1e-6
    ph, X, O, F = _oracle_case("fio_m4", N, leaf, tol, 2)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    info = fac.info()
    assert info["cand_max"] > 64 and info["rank_max"] > 32
    assert _compare_construction(F, fac, ph, X, O) == 0
    G = I.gaussian_vectors(N, 65, seed=11)
    Y_or = oracle.apply(F, G)
    x = torch.as_tensor(G, device=DEV)
    assert oracle.relative_error(fac.apply(x[:, 0].contiguous()).cpu().numpy(), Y_or[:, 0]) < 1e-12
    assert oracle.relative_error(fac.apply(x).cpu().numpy(), Y_or) < 1e-12
    x64 = x.to(torch.complex64)
    assert oracle.relative_error(fac.apply(x64[:, 0].contiguous()).cpu().numpy(), Y_or[:, 0]) < 2e-6
    assert oracle.relative_error(fac.apply(x64).cpu().numpy(), Y_or) < 2e-6
    assert oracle.relative_error(fac.apply(x64, dtype=B.C64_BF16X3).cpu().numpy(), Y_or) < 2e-4
    y_ex = oracle.dense_matvec(ph, X, O, G[:, 0])
    assert oracle.relative_error(fac.apply(x[:, 0].contiguous()).cpu().numpy(), y_ex) < 100 * tol


@pytest.mark.parametrize("N,leaf,kind,t,seed", [(1024, 16, "fio", 2, 5), (1024, 8, "dft", 1, 9),
                                                  (2048, 16, "fio", 1, 3)])
def test_random_sampler_matches_oracle(N, leaf, kind, t, seed):
    """The uniformly random sampler (Section 3's comparison): the same SplitMix64
    draws on both sides give identical sample sets.  At t = 2 the skeletons
    are then identical.  At t = 1 (as many random rows as candidates) R11 is
    so ill-conditioned that the eps-rank decision of a few IDs sits within
    rounding of the threshold and may differ (with its knock-on effects one
    level up), so up to 1% of the IDs may differ and both factorizations are
    held to the exact product instead.  T is held to the apply's agreement,
    not to the Mock-Chebyshev entry bound, for the same conditioning reason."""
    ph = I.dft_phase() if kind == "dft" else I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    tol = 1e-6
    F = oracle.build(ph, X, O, leaf, tol, oversample=t, sampler="random", seed=seed)
    fac = B.construct(ph, X, O, tol, leaf, oversample=t, device=DEV, sampler=B.SAMPLER_RANDOM, seed=seed)
    mismatched = _compare_construction(F, fac, ph, X, O, t_bound=None)
    n_ids = fac.info()["n_ids"]
    g = I.gaussian_vectors(N, None, seed=2)
    y = fac.apply(torch.as_tensor(g, device=DEV)).cpu().numpy()
    y_or = oracle.apply(F, g)
    if t == 2:
        assert mismatched == 0
        assert oracle.relative_error(y, y_or) < 1e-6
    else:
        assert mismatched <= max(1, n_ids // 100), (mismatched, n_ids)
        y_ex = oracle.dft_closed_form(g) if kind == "dft" else oracle.dense_matvec(ph, X, O, g)
        assert oracle.relative_error(y, y_ex) <= 2 * oracle.relative_error(y_or, y_ex) + 1e-12


def test_construct_errors():
    X, O = I.uniform_grid(64)
    with pytest.raises(B.IdbfError) as e:
        B.construct(I.dft_phase(), X, O, 1e-6, 3, device=DEV)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.IdbfError) as e:
        B.construct(I.dft_phase(), X[::-1].copy(), O, 1e-6, 4, device=DEV)
    assert e.value.status == B.EINVAL
    Xn = X.copy()
    Xn[5] = np.nan
    with pytest.raises(B.IdbfError) as e:
        B.construct(I.dft_phase(), Xn, O, 1e-6, 4, device=DEV)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.IdbfError) as e:
        B.construct(I.fio_phase(1.0, 1.0), *I.uniform_grid(4096), 1e-6, 16, mem_cap_bytes=1 << 16,
                    device=DEV)
    assert e.value.status == B.ENOMEM
    g, w = I.schlomilch_points(64)
    with pytest.raises(B.IdbfError) as e:     # J_0 arguments beyond the exact reduction's range
        B.construct(I.j0_kernel(), g, w * 1e6, 1e-6, 4, device=DEV)
    assert e.value.status == B.EINVAL and "J0" in str(e.value)


# ------------------------------------------------------------------ full size
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_fio_sampled_rows(dtype):
    """N = 2^20, leaf 16, tol 1e-6, t = 2 (the measured workload): 48 exact rows."""
    N, leaf, tol = 1 << 20, 16, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    info = fac.info()
    assert info["H"] == 8 and info["rank_max"] <= 32
    g = I.gaussian_vectors(N, None, seed=4)
    x = torch.as_tensor(g, device=DEV)
    if dtype == "c64":
        x = x.to(torch.complex64)
    y = fac.apply(x).cpu().numpy()
    rows = np.sort(np.random.default_rng(4).choice(N, 48, replace=False))
    ex = oracle.matvec_rows(ph, X, O, g, rows)
    assert oracle.relative_error(y[rows], ex) < 1e-4


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_nufft_sampled_rows(dtype):
    """Example 3 at N = 2^20 (leaf 16, tol 1e-6, t = 2): 48 exact rows."""
    N, leaf, tol = 1 << 20, 16, 1e-6
    ph, W, Xp = _workload("nufft", N)
    fac = B.construct(ph, W, Xp, tol, leaf, oversample=2, device=DEV)
    info = fac.info()
    assert info["H"] == 8 and info["rank_max"] <= 64
    g = I.gaussian_vectors(N, None, seed=6)
    x = torch.as_tensor(g, device=DEV)
    if dtype == "c64":
        x = x.to(torch.complex64)
    y = fac.apply(x).cpu().numpy()
    rows = np.sort(np.random.default_rng(6).choice(N, 48, replace=False))
    ex = oracle.matvec_rows(ph, W, Xp, g, rows)
    assert oracle.relative_error(y[rows], ex) < 1e-4


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_j0_sampled_rows(dtype):
    """Example 2 at N = 2^20 (leaf 16, tol 1e-6, t = 2): 48 exact rows."""
    N, leaf, tol = 1 << 20, 16, 1e-6
    ph, g, w = _workload("j0", N)
    fac = B.construct(ph, g, w, tol, leaf, oversample=2, device=DEV)
    info = fac.info()
    assert info["H"] == 8 and info["rank_max"] <= 64
    x = I.gaussian_vectors(N, None, seed=7)
    xd = torch.as_tensor(x, device=DEV)
    if dtype == "c64":
        xd = xd.to(torch.complex64)
    y = fac.apply(xd).cpu().numpy()
    rows = np.sort(np.random.default_rng(7).choice(N, 48, replace=False))
    ex = oracle.matvec_rows(ph, g, w, x, rows)
    assert oracle.relative_error(y[rows], ex) < 1e-4


def test_full_size_many_rhs_precisions():
    """N = 2^20 workload, 8 probe vectors: complex64 FP32-MFMA apply within
    1e-6 and BF16-split apply within 1e-3 of the FP64 apply of the same factors."""
    N, leaf, tol = 1 << 20, 16, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    P = torch.as_tensor(I.gaussian_vectors(N, 8, seed=5), device=DEV)
    y128 = fac.apply(P)
    p64 = P.to(torch.complex64)
    for dtype, bound in ((B.C64, 1e-6), (B.C64_BF16X3, 1e-3)):
        y = fac.apply(p64, dtype=dtype).to(torch.complex128)
        rel = float(torch.linalg.norm(y - y128) / torch.linalg.norm(y128))
        assert rel < bound, (dtype, rel)


def test_stats_describe_the_levels():
    """idbf_stats against the exported levels: rank histograms sum to the ID
    counts and match the ranks, per-level T entries and skeleton counts match,
    tall IDs are the ones that sampled more than 128 points."""
    ph, X, O = _workload("dft", 1024)
    fac = B.construct(ph, X, O, 1e-6, 64, oversample=4, device=DEV)
    st = fac.stats()
    info = fac.info()
    assert st["levels"] == info["H"] == st["H"]
    total_T, records = 0, 0
    for t, row in enumerate(st["per_level"], start=1):
        for side, name in ((B.SIDE_U, "U"), (B.SIDE_V, "V")):
            L, b = row[name], fac.batch(side, t)
            assert L["n_ids"] == len(b.rank) == L["rank_hist"].sum()
            assert np.array_equal(L["rank_hist"], np.bincount(b.rank, minlength=B.STATS_RANKS))
            assert (L["rank_min"], L["rank_max"]) == (b.rank.min(), b.rank.max())
            assert L["n_skel"] == b.rank.sum()
            assert L["nnz_T"] == int(np.sum(b.rank.astype(np.int64) * (b.cand_len - b.rank)))
            _, used, _ = fac.proposal(side, t)
            assert L["tall"] == int(np.sum(used > 128))
            assert L["proposed"] == L["accepted"] == L["rejected"] == 0
            total_T += L["nnz_T"]
            records += L["n_ids"]
    assert sum(row[s]["tall"] for row in st["per_level"] for s in "UV") > 0
    assert st["nnz_S"] == info["nnz_S"]
    assert st["apply_bytes_c64"] == 8 * (total_T + st["nnz_S"]) + 40 * records
    assert st["apply_bytes_c128"] == 16 * (total_T + st["nnz_S"]) + 40 * records


def test_allow_truncate_keeps_rank_64():
    """An eps-rank above the supported 64 (FIO, leaf 64, tol 1e-10) fails with
    IDBF_ERANK; with IDBF_FLAG_ALLOW_TRUNCATE those IDs keep 64 skeletons,
    which is the oracle's ID with rank parameter k = 64 (Section 2.1's
    (eps, k)-ID)."""
    N, leaf, tol = 2048, 64, 1e-10
    ph, X, O = _workload("fio", N)
    with pytest.raises(B.IdbfError) as e:
        B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    assert e.value.status == B.ERANK
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV, allow_truncate=True)
    assert fac.info()["rank_max"] == 64
    F = oracle.build(ph, X, O, leaf, tol, oversample=2, kmax=64)
    assert _compare_construction(F, fac, ph, X, O) == 0
    g = I.gaussian_vectors(N, None, seed=3)
    y = fac.apply(torch.as_tensor(g, device=DEV)).cpu().numpy()
    assert oracle.relative_error(y, oracle.apply(F, g)) < 1e-12


def test_profile_records_tile_one_apply():
    """With IDBF_FLAG_PROFILE one apply records each stage once. Consecutive
    stages share their boundary event (one kernel launch per record, back to
    back on the stream), so the records tile the apply: their sum is at most
    the time between two events around the call, and the events go back to
    the profiler's pool once each (three rounds reuse them)."""
    N, leaf, tol = 4096, 16, 1e-6
    ph, X, O = _workload("fio", N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV, profile=True)
    H = fac.info()["H"]
    stream = torch.cuda.Stream()
    for dtype, ct, pre in ((B.C64, torch.complex64, "apply1"), (B.C128, torch.complex128, "apply1d")):
        x = torch.randn(N, dtype=ct, device=DEV)
        y = torch.empty_like(x)
        for _ in range(3):
            fac.profile(reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fac.apply(x, y, dtype=dtype, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            prof = fac.profile(reset=True)
            assert {k: v["launches"] for k, v in prof.items()} == {f"{pre}_v": H, f"{pre}_s": 1, f"{pre}_u": H}
            assert all(v["ms"] > 0.0 for v in prof.values())
            assert sum(v["ms"] for v in prof.values()) <= e0.elapsed_time(e1) + 1e-3
        # switched off, the apply records nothing; records taken before stay readable
        fac.apply(x, y, dtype=dtype, stream=stream)
        fac.set_profile(False)
        fac.apply(x, y, dtype=dtype, stream=stream)
        torch.cuda.synchronize()
        assert {k: v["launches"] for k, v in fac.profile(reset=True).items()} == {f"{pre}_v": H, f"{pre}_s": 1,
                                                                                  f"{pre}_u": H}
        with pytest.raises(B.IdbfError):
            fac.profile(reset=True)  # off and nothing held
        fac.set_profile(True)
    fac.close()
