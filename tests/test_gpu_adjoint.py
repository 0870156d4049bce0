"""Adjoint apply y = K~^H x (idbf_apply_adjoint) against the oracle's adjoint
of its own factors (identical skeletons), in every precision and path, and
the adjoint identity <K~ x, y> = <x, K~^H y> at the full workload size."""
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


def _workload(kind, N):
    if kind == "nufft":
        W, Xp = I.nufft_points(N, seed=N + 1)
        return I.dft_phase(), W, Xp
    if kind == "j0":
        g, w = I.schlomilch_points(N)
        return I.j0_kernel(), g, w
    X, O = I.uniform_grid(N)
    return (I.dft_phase() if kind == "dft" else I.fio_phase(1.0, 1.0)), X, O


@pytest.mark.parametrize("N,leaf,kind,tol,os_", [
    (1024, 8, "dft", 1e-10, 1),     # odd L: four middle blocks per V_H ID
    (16, 8, "dft", 1e-10, 1),       # H = 0: the dense block, conjugate transposed
    (64, 16, "fio", 1e-6, 2),       # H = 1
    (256, 2, "fio", 1e-8, 1),       # leaf 2, L = 7
    (2048, 16, "fio", 1e-6, 2),     # the workload's shape at a small N
    (2048, 16, "nufft", 1e-6, 2),
    (1024, 8, "j0", 1e-10, 2),      # real kernel: K^H = K^T
])
def test_adjoint_matches_oracle_every_path(N, leaf, kind, tol, os_):
    ph, X, O = _workload(kind, N)
    F = oracle.build(ph, X, O, leaf, tol, oversample=os_)
    fac = B.construct(ph, X, O, tol, leaf, oversample=os_, device=DEV)
    # 1 RHS (wavefront per ID) and 67 RHS (VALU complex128 / matrix-core complex64)
    for nrhs in (None, 67):
        g = I.gaussian_vectors(N, nrhs, seed=N + (nrhs or 1))
        ref = oracle.apply_adjoint(F, g)
        x = torch.as_tensor(g, device=DEV)
        y128 = fac.apply_adjoint(x).cpu().numpy()
        assert oracle.relative_error(y128, ref) < 1e-12, (nrhs, "c128")
        x64 = x.to(torch.complex64)
        y64 = fac.apply_adjoint(x64).cpu().numpy()
        assert oracle.relative_error(y64, ref) < 2e-6, (nrhs, "c64")
        ybf = fac.apply_adjoint(x64, dtype=B.C64_BF16X3).cpu().numpy()
        assert oracle.relative_error(ybf, ref) < 2e-4, (nrhs, "bf16")
        if nrhs:
            col = np.linalg.norm(y64 - ref, axis=0) / np.linalg.norm(ref, axis=0)
            assert col.max() < 2e-5            # every column, the ragged tail included
    # against the exact K^H
    g = I.gaussian_vectors(N, None, seed=3)
    K = oracle.entries(ph, X, O, np.arange(N), np.arange(N))
    y = fac.apply_adjoint(torch.as_tensor(g, device=DEV)).cpu().numpy()
    assert oracle.relative_error(y, K.conj().T @ g) < max(100 * tol, 1e-12)


def test_adjoint_deterministic_and_errors():
    N, leaf, tol = 2048, 16, 1e-6
    ph, X, O = _workload("fio", N)
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    x = torch.as_tensor(I.gaussian_vectors(N, 5, seed=1), device=DEV)
    a = fac.apply_adjoint(x)
    assert torch.equal(a, fac.apply_adjoint(x))
    with pytest.raises(ValueError):
        fac.apply_adjoint(x, y=x)                 # in place is refused by the binding ...
    lib = B.load()                                # ... and by the C ABI
    assert lib.idbf_apply_adjoint(fac._h, x.data_ptr(), x.data_ptr(), 5, B.C128, None) == B.EINVAL
    with pytest.raises(ValueError):
        fac.apply_adjoint(x[:N - 1])              # short input: refused before any launch
    empty = torch.zeros((N, 0), dtype=torch.complex128, device=DEV)
    assert fac.apply_adjoint(empty).shape == (N, 0)


@pytest.mark.parametrize("kind", ["fio", "nufft"])
def test_full_size_adjoint_identity(kind):
    """N = 2^20 (leaf 16, tol 1e-6, t = 2): <K~ x, y> = <x, K~^H y> for the
    same factors, complex128, and complex64 within its rounding."""
    N = 1 << 20
    ph, X, O = _workload(kind, N)
    fac = B.construct(ph, X, O, 1e-6, 16, oversample=2, device=DEV)
    x = torch.as_tensor(I.gaussian_vectors(N, None, seed=8), device=DEV)
    y = torch.as_tensor(I.gaussian_vectors(N, None, seed=9), device=DEV)
    kx = fac.apply(x)
    khy = fac.apply_adjoint(y)
    lhs, rhs = torch.vdot(y, kx), torch.vdot(khy, x)
    scale = float(torch.linalg.norm(y) * torch.linalg.norm(kx))
    assert abs(complex(lhs - rhs)) / scale < 1e-12
    khy64 = fac.apply_adjoint(y.to(torch.complex64)).to(torch.complex128)
    assert float(torch.linalg.norm(khy64 - khy) / torch.linalg.norm(khy)) < 1e-6
