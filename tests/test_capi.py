"""The C-ABI library loads and exports every declared symbol; host-side
argument checks answer without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1809_10573_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="library not built")


def _declared():
    src = open(os.path.join(ROOT, "include", "idbf.h")).read()
    return sorted(set(re.findall(r"\b(idbf_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = B.load()
    names = _declared()
    assert set(names) == set(B.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_defaults_and_error_string():
    lib = B.load()
    o = B.Opts_t()
    o.kmax, o.oversample = 7, 9
    lib.idbf_opts_default(C.byref(o))
    assert (o.kmax, o.oversample, o.mem_cap_bytes) == (0, 1, 0)
    lib.idbf_opts_default(None)          # NULL-safe
    assert isinstance(lib.idbf_last_error(), bytes)
    assert lib.idbf_destroy(None) == B.OK


def test_argument_errors_without_gpu():
    lib = B.load()
    ph = B.Phase_t(B.PHASE_DFT, 0, 0.0, 0.0, 0.0, 1.0)
    h = C.c_void_p()
    fake = C.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1e-6, 8, None, None) == B.EINVAL
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1000, 1e-6, 8, None, C.byref(h)) == B.EINVAL
    assert b"power of two" in lib.idbf_last_error()
    assert h.value is None
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1e-6, 3, None, C.byref(h)) == B.EINVAL
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1e-6, 256, None, C.byref(h)) == B.EINVAL
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1.5, 8, None, C.byref(h)) == B.EINVAL
    assert lib.idbf_construct(C.byref(ph), None, fake, 1024, 1e-6, 8, None, C.byref(h)) == B.EINVAL
    bad = B.Phase_t(7, 0, 0.0, 0.0, 0.0, 1.0)
    assert lib.idbf_construct(C.byref(bad), fake, fake, 1024, 1e-6, 8, None, C.byref(h)) == B.EINVAL
    fio0 = B.Phase_t(B.PHASE_FIO, 0, 2.0, 1.0, 1.0, 0.0)
    assert lib.idbf_construct(C.byref(fio0), fake, fake, 1024, 1e-6, 8, None, C.byref(h)) == B.EINVAL
    o = B.Opts_t()
    lib.idbf_opts_default(C.byref(o))
    o.oversample = 0
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1e-6, 8, C.byref(o), C.byref(h)) == B.EINVAL
    assert lib.idbf_apply(None, fake, fake, 1, B.C128, None) == B.EINVAL
    assert lib.idbf_profile_enable(None, 1) == B.EINVAL
    # the QR shape mask is host state: set, read back, reject bits above the three
    m = C.c_uint32()
    assert lib.idbf_get_qr_shapes(C.byref(m)) == B.OK
    keep = m.value
    assert lib.idbf_set_qr_shapes(5) == B.OK
    assert lib.idbf_get_qr_shapes(C.byref(m)) == B.OK and m.value == 5
    assert lib.idbf_set_qr_shapes(8) == B.EINVAL
    assert lib.idbf_get_qr_shapes(C.byref(m)) == B.OK and m.value == 5
    assert lib.idbf_get_qr_shapes(None) == B.EINVAL
    assert lib.idbf_set_qr_shapes(keep) == B.OK
    assert lib.idbf_tune_construct(C.byref(bad), fake, fake, 1024, 1e-6, 8, None, None, None, None,
                                   None) == B.EINVAL
    assert lib.idbf_tune_construct(C.byref(ph), None, fake, 1024, 1e-6, 8, None, None, None, None,
                                   None) == B.EINVAL
    assert lib.idbf_apply_adjoint(None, fake, fake, 1, B.C128, None) == B.EINVAL
    assert b"handle is NULL" in lib.idbf_last_error()
    assert lib.idbf_get_info(None, None) == B.EINVAL
    assert lib.idbf_batch_sizes(None, 0, 1, None, None, None) == B.EINVAL
    assert lib.idbf_sample(C.byref(ph), fake, fake, fake, -1, fake, 3, fake, None) == B.EINVAL
    assert lib.idbf_sample(C.byref(ph), fake, fake, fake, 0, fake, 3, fake, None) == B.OK
    assert lib.idbf_id_batch(C.byref(ph), fake, fake, 5, 1, fake, fake, fake, fake, fake, fake, 1e-6, 0, 1,
                             fake, fake, fake, fake, None) == B.EINVAL
    assert lib.idbf_construct_batched(0, None, None, None, None, None, None, None, None) == B.EINVAL
    assert lib.idbf_apply_batched(0, None, None, None, None, B.C64, None) == B.EINVAL
    cfg = B.ApplyConfig_t()
    assert lib.idbf_get_apply_config(None, C.byref(cfg)) == B.EINVAL
    assert lib.idbf_set_apply_config(None, C.byref(cfg)) == B.EINVAL
    assert lib.idbf_tune_apply(None, 16, B.C64, None, None, C.byref(cfg)) == B.EINVAL
    assert C.sizeof(B.ApplyConfig_t) == 32
    assert C.sizeof(B.Opts_t) == 88
    o = B.Opts_t()
    lib.idbf_opts_default(C.byref(o))
    assert (o.dev_alloc, o.dev_free, o.alloc_user) == (None, None, None)
    o.dev_alloc = C.cast(B.DEV_ALLOC_FN(lambda n, u: None), C.c_void_p).value  # no dev_free: refused
    assert lib.idbf_construct(C.byref(ph), fake, fake, 1024, 1e-6, 8, C.byref(o), C.byref(h)) == B.EINVAL
    assert b"dev_alloc and dev_free" in lib.idbf_last_error()


def test_binding_rejects_bad_operands_before_any_launch():
    # the C ABI takes no lengths, so the binding checks every vector block:
    # shape (N,) or (N, nrhs), dtype, contiguity, device, and y against x
    torch = pytest.importorskip("torch")
    cpu = torch.device("cpu")
    good = torch.zeros((8, 3), dtype=torch.complex128)
    B._check_operand("x", good, 8, torch.complex128, cpu)
    for bad in (torch.zeros((7, 3), dtype=torch.complex128),           # wrong N
                torch.zeros((8, 3, 1), dtype=torch.complex128),        # 3-D
                torch.zeros((8, 3), dtype=torch.complex64),            # dtype
                torch.zeros((3, 8), dtype=torch.complex128).t(),       # not contiguous
                np.zeros((8, 3), dtype=np.complex128)):                # not a tensor
        with pytest.raises(ValueError):
            B._check_operand("x", bad, 8, torch.complex128, cpu)
    with pytest.raises(ValueError):
        B._check_operand("x", good, 8, torch.complex128, torch.device("meta"))
    B._check_output(good, torch.zeros_like(good))
    for bad in (torch.zeros((8, 2), dtype=torch.complex128), torch.zeros((8, 3), dtype=torch.complex64),
                torch.zeros((3, 8), dtype=torch.complex128).t(), good, good[1:]):
        with pytest.raises(ValueError):
            B._check_output(good, bad)
