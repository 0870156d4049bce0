"""The apply autotuner: it sets the fastest configuration it timed on the
handle, records it in its cache file, and a later handle of the same problem
takes it from there without timing; the tuned apply still matches the
oracle."""
import numpy as np
import pytest

import oracle
from paper_1809_10573_amd import binding as B, inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_tune_apply_and_cache(tmp_path):
    N, leaf, tol = 2048, 16, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    cache = str(tmp_path / "idbf_tune.txt")
    fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    got = fac.tune_apply(300, B.C64, cache)
    assert not got["from_cache"] and got["ms"] > 0
    assert got["fuse"] in (0, 1) and got["rhs_iter"] in (1, 2, 4, 8, 16)
    assert fac.apply_config() == {"fuse": got["fuse"], "rhs_iter": got["rhs_iter"]}
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[0].startswith(("gfx", "unknown"))
    again = B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV)
    hit = again.tune_apply(300, B.C64, cache)
    assert hit["from_cache"] and (hit["fuse"], hit["rhs_iter"]) == (got["fuse"], got["rhs_iter"])
    assert len(open(cache).read().splitlines()) == 1
    other = again.tune_apply(17, B.C128, cache)          # a different problem: timed, appended
    assert not other["from_cache"] and other["fuse"] == got["fuse"]   # complex128 keeps the fusion setting
    assert len(open(cache).read().splitlines()) == 2
    nocache = again.tune_apply(64, B.C64_BF16X3)          # no file; fusion is timed for the BF16 split too
    assert not nocache["from_cache"] and nocache["fuse"] in (0, 1)
    F = oracle.build(ph, X, O, leaf, tol, oversample=2)
    G = I.gaussian_vectors(N, 300, seed=4)
    fac.set_apply_config(fuse=got["fuse"], rhs_iter=got["rhs_iter"])
    y = fac.apply(torch.as_tensor(G, device=DEV).to(torch.complex64)).cpu().numpy()
    assert oracle.relative_error(y, oracle.apply(F, G)) < 2e-6


def test_tune_construct_shapes_and_cache(tmp_path):
    """The QR-shape tuner (idbf_tune_construct) sets the mask it timed fastest
    and records it; a later call takes it from the cache file.  Both shape
    families give the same factors: identical ranks, masks and skeletons,
    and complex128 applies that agree to rounding."""
    N, leaf, tol = 1 << 14, 16, 1e-6
    ph = I.fio_phase(1.0, 1.0)
    X, O = I.uniform_grid(N)
    keep = B.qr_shapes()
    try:
        cache = str(tmp_path / "idbf_qr_tune.txt")
        got = B.tune_construct(ph, X, O, tol, leaf, oversample=2, cache_path=cache, device=DEV)
        assert 0 <= got["mask"] <= 7 and not got["from_cache"] and got["ms"] > 0
        assert B.qr_shapes() == got["mask"]
        lines = open(cache).read().splitlines()
        assert len(lines) == 1 and " qr N=16384 " in lines[0].split("\t")[0]
        B.set_qr_shapes(7 - got["mask"])
        hit = B.tune_construct(ph, X, O, tol, leaf, oversample=2, cache_path=cache, device=DEV)
        assert hit["from_cache"] and hit["mask"] == got["mask"] and B.qr_shapes() == got["mask"]
        with pytest.raises(B.IdbfError):
            B.set_qr_shapes(8)
        facs = []
        for mask in (0, 7):  # every range on the tall, then on the short wavefronts
            B.set_qr_shapes(mask)
            facs.append(B.construct(ph, X, O, tol, leaf, oversample=2, device=DEV))
        a, b = facs
        s = 0
        for side in (B.SIDE_U, B.SIDE_V):
            for t in range(1, a.info()["H"] + 1):
                x, y = a.batch(side, t), b.batch(side, t)
                for f in ("rank", "cand_len", "mask", "skel"):
                    assert np.array_equal(getattr(x, f), getattr(y, f)), (side, t, f)
                s = max(s, int(oracle.sample_count(int(x.cand_len.max()), N, 2)))
        assert s > 64  # some IDs ran on the shapes the mask chooses
        Sa, oa = a.middle()
        Sb, ob = b.middle()
        assert np.array_equal(oa, ob)
        ends = np.append(oa[1:], len(Sa))
        for o, e in zip(oa, ends):  # a block's reservation is rounded up to even: its last slot may be padding
            assert np.array_equal(Sa[o:e - 1], Sb[o:e - 1])
        v = torch.as_tensor(I.gaussian_vectors(N, 1, 3)[:, 0], device=DEV)
        ya, yb = a.apply(v).cpu().numpy(), b.apply(v).cpu().numpy()
        assert np.linalg.norm(ya - yb) <= 1e-12 * np.linalg.norm(ya)
    finally:
        B.set_qr_shapes(keep)
