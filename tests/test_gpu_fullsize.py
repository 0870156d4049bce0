"""Full-size parity (N = 2^20, the measured FIO workload: leaf 16, tol 1e-6,
t = 2) against the FP64 oracle, following Section 3's error measure on the
factors the GPU built:

* the exported factors, rebuilt as an oracle.Factors and applied by
  oracle.apply to 8 probe vectors, against the GPU's complex128, complex64
  (FP32 MFMA for the block, VALU for one vector) and BF16-split applies;
* per level and side, 1000 random IDs (200 on the two lowest levels)
  recomputed by the oracle's
  column_id on the GPU's own candidate and allowed sets: identical
  skeletons, T within the parity bound.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_10573_amd import binding as B  # noqa: E402
from gpu_export import GpuLevels, to_oracle_factors  # noqa: E402

DEV = "cuda:0"
N, LEAF, TOL, T_OS = 1 << 20, 16, 1e-6, 2


@pytest.fixture(scope="module")
def built():
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    fac = B.construct(ph, X, O, TOL, LEAF, oversample=T_OS, device=DEV)
    return ph, X, O, fac


def test_full_size_apply_of_exported_factors(built):
    ph, X, O, fac = built
    t0 = time.time()
    F = to_oracle_factors(fac, TOL)
    assert F.nnz() == fac.info()["nnz_T"] + fac.info()["nnz_S"]
    P = I.gaussian_vectors(N, 8, seed=21)
    y_or = oracle.apply(F, P)
    print(f"oracle factors + apply of 8 probes: {time.time() - t0:.1f} s", flush=True)
    Pd = torch.as_tensor(P, device=DEV)
    p64 = Pd.to(torch.complex64)
    for name, y, bound in (("c128", fac.apply(Pd), 1e-12),
                           ("c64", fac.apply(p64, dtype=B.C64), 1e-6),
                           ("bf16x3", fac.apply(p64, dtype=B.C64_BF16X3), 1e-3)):
        y = y.to(torch.complex128).cpu().numpy()
        rel = oracle.relative_error(y, y_or)
        print(f"{name}: rel.err vs FP64 oracle apply {rel:.3e}", flush=True)
        assert rel < bound, name
    for name, dt, bound in (("c128 1-RHS", torch.complex128, 1e-12), ("c64 1-RHS", torch.complex64, 1e-6)):
        y1 = fac.apply(Pd[:, 0].contiguous().to(dt)).to(torch.complex128).cpu().numpy()
        rel = oracle.relative_error(y1, y_or[:, 0])
        print(f"{name}: {rel:.3e}", flush=True)
        assert rel < bound, name


def _entry_tol(ph, n):
    # the two sides' entries differ only through c(x) (GPU sinpi vs host sin, a
    # few ulps of c), amplified by |xi| <= N/2 in the phase 2 pi c(x) |xi|
    amp = abs(ph.a) / abs(ph.cdiv)
    return 2 * np.pi * ((n / 2) * 8 * 2.2e-16 * amp + 1e-15) + 1e-15


def test_full_size_random_ids_recomputed(built):
    """T = R11^{-1} R12 moves with its sampled entries: the bound is the
    entries' agreement (about 7e-10 at N = 2^20) amplified by R11's
    conditioning |R_00| / |R_kk|.  Skeletons must agree exactly."""
    ph, X, O, fac = built
    delta = max(1e-12, 4 * _entry_tol(ph, N))
    G = GpuLevels(fac)
    rng = np.random.default_rng(22)
    checked = 0
    expected = 0
    for t in range(1, G.H + 1):
        for side in (B.SIDE_U, B.SIDE_V):
            b, offs = G.batches[(side, t)]
            # the lowest levels' allowed sets hold 10^5..10^6 points, which makes
            # the oracle's sample selection slow: fewer IDs there (about 4000
            # IDs in all, some 80 s of host work)
            n_check = 100 if t <= 2 else 300
            expected += n_check
            t0 = time.time()
            for q in rng.choice(len(b.rank), n_check, replace=False):
                cand, allowed = G.sets(side, t, int(q))
                coords = X[allowed] if side == B.SIDE_V else O[allowed]
                s = oracle.sample_count(len(cand), len(allowed), T_OS)
                samp = allowed[oracle.mock_chebyshev(coords, s)]
                Bm = (oracle.entries(ph, X, O, samp, cand) if side == B.SIDE_V
                      else oracle.entries(ph, X, O, cand, samp).T)
                cid = oracle.column_id(Bm, TOL)
                rec = G.record(side, t, int(q))
                assert np.array_equal(rec.skel, cand[cid.skel]), (t, side, q)
                kappa = cid.rdiag[0] / cid.rdiag[-1]
                scale = max(1.0, np.abs(cid.T).max(initial=0.0))
                assert np.max(np.abs(rec.T - cid.T), initial=0.0) <= delta * kappa * scale, (t, side, q)
                checked += 1
            print(f"level {t} side {side}: {n_check} IDs identical ({time.time() - t0:.1f} s)", flush=True)
    assert checked == expected
