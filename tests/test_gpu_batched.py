"""Batched construction and apply (idbf_construct_batched / idbf_apply_batched)
against the same instances built and applied one by one: the lockstep sweep
runs the same kernels on the same inputs, so factors and outputs must agree
bit for bit; the small instances are also checked against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_10573_amd import binding as B  # noqa: E402
from gpu_export import same_factors  # noqa: E402

DEV = "cuda:0"

# uneven N (odd and even L, H = 0), both kernels, different tolerances and leaves
CASES = [
    (I.dft_phase(), 1024, 8, 1e-10),
    (I.fio_phase(0.3, 2.0), 2048, 16, 1e-6),
    (I.fio_phase(1.0, 1.0), 4096, 16, 1e-6),
    (I.dft_phase(), 256, 16, 1e-6),
    (I.fio_phase(0.0, 1.0), 512, 8, 1e-8),
    (I.dft_phase(), 16, 8, 1e-10),
    (I.fio_phase(0.7, 1.0), 8192, 16, 1e-6),
]


def test_construct_batched_equals_one_by_one():
    grids = [I.uniform_grid(N) for _, N, _, _ in CASES]
    facs = B.construct_batched([c[0] for c in CASES], [g[0] for g in grids], [g[1] for g in grids],
                               [c[3] for c in CASES], [c[2] for c in CASES], oversample=2, device=DEV)
    for (ph, N, leaf, tol), (X, O), fb in zip(CASES, grids, facs):
        f1 = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
        same_factors(fb, f1)
    # the smallest ones against the oracle's apply of its own factors
    for (ph, N, leaf, tol), (X, O), fb in list(zip(CASES, grids, facs))[3:6]:
        F = oracle.build(ph, X, O, leaf, tol, oversample=2)
        g = I.gaussian_vectors(N, None, seed=N)
        y = fb.apply(torch.as_tensor(g, device=DEV)).cpu().numpy()
        assert oracle.relative_error(y, oracle.apply(F, g)) < 1e-12


@pytest.mark.parametrize("dtype", [B.C128, B.C64, B.C64_BF16X3])
def test_apply_batched_equals_one_by_one(dtype):
    grids = [I.uniform_grid(N) for _, N, _, _ in CASES]
    facs = B.construct_batched([c[0] for c in CASES], [g[0] for g in grids], [g[1] for g in grids],
                               [c[3] for c in CASES], [c[2] for c in CASES], oversample=2, device=DEV)
    tdt = torch.complex128 if dtype == B.C128 else torch.complex64
    nrhs = [1, 16, 64, 1, 16, 64, 3]
    xs = [torch.as_tensor(I.gaussian_vectors(N, r if r > 1 else None, seed=7 + i), device=DEV).to(tdt)
          for i, ((_, N, _, _), r) in enumerate(zip(CASES, nrhs))]
    ys = B.apply_batched(facs, xs, dtype=dtype)
    torch.cuda.synchronize()
    for f, x, y in zip(facs, xs, ys):
        y1 = f.apply(x, dtype=dtype)
        assert torch.equal(y, y1)


def test_batched_errors_name_the_instance():
    X, O = I.uniform_grid(256)
    with pytest.raises(B.IdbfError) as e:
        B.construct_batched([I.dft_phase(), I.dft_phase()], [X, X], [O, O], [1e-6, 1e-6], [16, 3],
                            device=DEV)
    assert e.value.status == B.EINVAL and "instance 1" in str(e.value)
    f = B.construct(I.dft_phase(), X, O, 1e-6, 16, device=DEV)
    x = torch.zeros(256, dtype=torch.complex128, device=DEV)
    with pytest.raises(B.IdbfError):
        B.apply_batched([f, f], [x, x])        # handles must be distinct


def test_uneven_family_batch():
    """The many-instance workload at reduced sizes (12 instances, N = 2^12..2^14,
    DFT and FIO members c(x) = (2 + a sin 2 pi m x)/8 with uneven ranks): the
    batched construction equals one-by-one construction, the batched apply
    equals one-by-one applies, and every instance approximates its kernel
    (exact rows) to the method's tolerance."""
    work = I.batched_workload(count=12, seed=5, emin=12, emax=14)
    grids = [I.uniform_grid(w["N"]) for w in work]
    facs = B.construct_batched([w["phase"] for w in work], [g[0] for g in grids], [g[1] for g in grids],
                               [w["tol"] for w in work], [w["leaf"] for w in work], oversample=2, device=DEV)
    ranks = [f.info()["rank_max"] for f in facs]
    assert max(ranks) > min(ranks)                       # uneven ranks across instances
    for w, (X, O), fb in zip(work, grids, facs):
        same_factors(fb, B.construct(w["phase"], X, O, w["tol"], w["leaf"], oversample=2, device=DEV))
    xs = [torch.as_tensor(I.gaussian_vectors(w["N"], w["nrhs"] if w["nrhs"] > 1 else None, seed=i),
                          device=DEV) for i, w in enumerate(work)]
    ys = B.apply_batched(facs, xs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for w, (X, O), f, x, y in zip(work, grids, facs, xs, ys):
        assert torch.equal(y, f.apply(x))
        rows = np.sort(rng.choice(w["N"], 32, replace=False))
        g = x.cpu().numpy()
        g0 = g if g.ndim == 1 else g[:, 0]
        y0 = y.cpu().numpy()
        y0 = y0 if y0.ndim == 1 else y0[:, 0]
        ex = oracle.matvec_rows(w["phase"], X, O, g0, rows)
        assert oracle.relative_error(y0[rows], ex) < 100 * w["tol"], (w["kind"], w["N"], w["a"], w["m"])


@pytest.mark.parametrize("dtype", [B.C64, B.C64_BF16X3, B.C128])
def test_captured_plan_replays_match_eager(dtype):
    """A batched apply captured into a HIP graph, replayed three times with the
    program's own eager work and synchronizations in between: every replay
    equals the eager batched apply bit for bit."""
    stream = torch.cuda.Stream()
    grids = [I.uniform_grid(N) for _, N, _, _ in CASES]
    with torch.cuda.stream(stream):
        facs = B.construct_batched([c[0] for c in CASES], [g[0] for g in grids], [g[1] for g in grids],
                                   [c[3] for c in CASES], [c[2] for c in CASES], oversample=2, device=DEV)
        tdt = torch.complex128 if dtype == B.C128 else torch.complex64
        nrhs = [1, 16, 64, 1, 16, 64, 3]
        xs = [torch.as_tensor(I.gaussian_vectors(N, r if r > 1 else None, seed=20 + i), device=DEV).to(tdt)
              for i, ((_, N, _, _), r) in enumerate(zip(CASES, nrhs))]
        ref = B.apply_batched(facs, xs, dtype=dtype)
        ys = [torch.zeros_like(x) for x in xs]
        plan = B.ApplyPlan(facs, xs, ys, dtype=dtype, stream=stream)
        for rep in range(3):
            for y in ys:
                y.zero_()
            scratch = torch.randn(1 << 20, device=DEV).sum()   # unrelated eager work
            plan.launch(stream)
            stream.synchronize()
            assert float(scratch) == float(scratch)
            for y, r in zip(ys, ref):
                assert torch.equal(y, r), rep
        plan.close()


def test_live_plan_pins_the_workspace():
    """A captured plan writes its handles' apply workspaces: while it lives, an
    apply that would need a larger workspace is refused (IDBF_EINVAL) instead
    of moving it, the handle cannot be destroyed, and replays still give the
    eager result; once the plan is gone both work again."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        facs = [B.construct(ph, *I.uniform_grid(N), tol, leaf, oversample=2, device=DEV)
                for ph, N, leaf, tol in CASES[:3]]
        xs = [torch.as_tensor(I.gaussian_vectors(f.X.numel(), None, seed=30 + i), device=DEV)
              for i, f in enumerate(facs)]
        ref = B.apply_batched(facs, xs)
        ys = [torch.zeros_like(x) for x in xs]
        plan = B.ApplyPlan(facs, xs, ys, stream=stream)
        big = torch.as_tensor(I.gaussian_vectors(facs[1].X.numel(), 65, seed=3), device=DEV)
        with pytest.raises(B.IdbfError) as e:
            facs[1].apply(big, stream=stream)
        assert e.value.status == B.EINVAL and "plan" in str(e.value)
        with pytest.raises(B.IdbfError) as e:
            facs[1].reserve(65, B.C128)
        assert e.value.status == B.EINVAL
        lib = B.load()
        assert lib.idbf_destroy(facs[0]._h) == B.EINVAL        # still held by the plan
        small = facs[1].apply(xs[1], stream=stream)             # fits the workspace: allowed
        plan.launch(stream)
        stream.synchronize()
        for y, r in zip(ys, ref):
            assert torch.equal(y, r)
        assert torch.equal(small, ref[1])
        plan.close()
        Y = facs[1].apply(big, stream=stream)                   # grows now
        stream.synchronize()
        assert Y.shape == big.shape
        for f in facs:
            f.close()
