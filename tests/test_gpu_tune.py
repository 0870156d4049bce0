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
