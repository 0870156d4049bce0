"""ctypes binding of libidbf.so (the C ABI declared in include/idbf.h).

Argument marshalling only: every step of construction and apply runs in the
HIP kernels of the library.  Device buffers are torch tensors on a ROCm
device; torch is used for memory and streams, nothing else.  The library is
loaded on first use; if it is missing or fails to load, calls raise -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libidbf.so")

OK, EINVAL, ENOMEM, EHIP, ERANK, EUNSUPPORTED = range(6)
PHASE_DFT, PHASE_FIO, PHASE_J0 = 0, 1, 2
C128, C64, C64_BF16X3 = 0, 1, 2
SIDE_U, SIDE_V = 0, 1
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ERANK", 5: "EUNSUPPORTED"}

# every symbol include/idbf.h declares
EXPORTED = [
    "idbf_opts_default", "idbf_construct", "idbf_apply", "idbf_destroy", "idbf_last_error",
    "idbf_get_info", "idbf_batch_sizes", "idbf_batch_export", "idbf_middle_sizes",
    "idbf_middle_export", "idbf_sample", "idbf_id_batch", "idbf_profile_read", "idbf_profile_enable",
    "idbf_reserve",
    "idbf_construct_batched", "idbf_apply_batched", "idbf_mlp_param_count", "idbf_mlp_create",
    "idbf_mlp_destroy", "idbf_mlp_params", "idbf_mlp_forward", "idbf_mlp_loss_grad", "idbf_mlp_train",
    "idbf_rank_samples", "idbf_apply_batched_plan", "idbf_plan_launch", "idbf_plan_destroy",
    "idbf_apply_adjoint", "idbf_release_cached_memory", "idbf_stats", "idbf_batch_proposal",
    "idbf_apply_noalloc", "idbf_skeleton_samples", "idbf_batch_skeleton_proposal",
    "idbf_get_apply_config", "idbf_set_apply_config", "idbf_tune_apply", "idbf_set_qr_shapes",
    "idbf_get_qr_shapes", "idbf_tune_construct",
]
MLP_INPUTS = 8
FLAG_PROFILE, FLAG_PROPOSER_FORCE_REJECT, FLAG_ALLOW_TRUNCATE = 1, 2, 4
STATS_LEVELS, STATS_RANKS = 16, 65
SAMPLER_MOCKCHEB, SAMPLER_RANDOM = 0, 1
MAX_CAND, MAX_RANK, MAX_SAMPLES, SLOT = 128, 64, 256, 4096  # limits of include/idbf.h


def mask_bits(mask_row, c: int) -> np.ndarray:
    """Skeleton flags of candidates 0..c-1 from a (lo, hi) 128-bit mask pair."""
    lo, hi = int(mask_row[0]), int(mask_row[1])
    word = lo | (hi << 64)
    return np.array([(word >> l) & 1 for l in range(c)], bool)


class IdbfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Phase_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("c0", C.c_double),
                ("a", C.c_double), ("freq", C.c_double), ("cdiv", C.c_double)]


class Opts_t(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("oversample", C.c_int32), ("flags", C.c_int32),
                ("sampler", C.c_int32), ("mem_cap_bytes", C.c_uint64), ("stream", C.c_void_p),
                ("proposer", C.c_void_p), ("proposal_margin", C.c_int32), ("proposal_accept", C.c_float),
                ("seed", C.c_uint64), ("skeleton_proposer", C.c_void_p), ("dev_alloc", C.c_void_p),
                ("dev_free", C.c_void_p), ("alloc_user", C.c_void_p)]


DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class TorchAllocator:
    """A handle's device memory from torch's caching allocator
    (opts.dev_alloc / dev_free): blocks are taken on the device's current
    stream and given back to torch when the library frees them."""

    def __init__(self, device="cuda"):
        import torch
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.live: dict = {}
        self.calls = 0

        def _alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device)
            except RuntimeError:
                return None
            self.live[int(p)] = int(nbytes)
            self.calls += 1
            return p

        def _free(ptr, nbytes, user):
            self.live.pop(int(ptr), None)
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = DEV_ALLOC_FN(_alloc)  # kept alive as long as any handle that uses them
        self._free = DEV_FREE_FN(_free)

    def set(self, opts) -> None:
        opts.dev_alloc = C.cast(self._alloc, C.c_void_p).value
        opts.dev_free = C.cast(self._free, C.c_void_p).value


class Info_t(C.Structure):
    _fields_ = [("N", C.c_int64), ("leaf", C.c_int32), ("L", C.c_int32), ("H", C.c_int32),
                ("oversample", C.c_int32), ("tol", C.c_double), ("n_ids", C.c_int64),
                ("nnz_T", C.c_int64), ("nnz_S", C.c_int64), ("n_skel", C.c_int64),
                ("rank_min", C.c_int32), ("rank_max", C.c_int32), ("cand_max", C.c_int32),
                ("samples_max", C.c_int32), ("device_bytes", C.c_int64), ("construct_ms", C.c_double),
                ("id_flops", C.c_double), ("sampled_entries", C.c_int64), ("proposed", C.c_int64),
                ("rejected", C.c_int64)]


class LevelStats_t(C.Structure):
    _fields_ = [("n_ids", C.c_int64), ("rank_hist", C.c_int64 * STATS_RANKS), ("rank_min", C.c_int32),
                ("rank_max", C.c_int32), ("cand_max", C.c_int32), ("samples_max", C.c_int32),
                ("n_skel", C.c_int64), ("nnz_T", C.c_int64), ("sampled_entries", C.c_int64), ("tall", C.c_int64),
                ("proposed", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("id_flops", C.c_double), ("wall_ms", C.c_double)]


class Stats_t(C.Structure):
    _fields_ = [("L", C.c_int32), ("H", C.c_int32), ("levels", C.c_int32), ("reserved", C.c_int32),
                ("level", (LevelStats_t * 2) * STATS_LEVELS), ("nnz_S", C.c_int64), ("n_blocks_S", C.c_int64),
                ("apply_bytes_c64", C.c_int64), ("apply_bytes_c128", C.c_int64), ("device_bytes", C.c_int64),
                ("construct_ms", C.c_double)]


class ApplyConfig_t(C.Structure):
    _fields_ = [("fuse", C.c_int32), ("rhs_iter", C.c_int32), ("from_cache", C.c_int32), ("ms", C.c_float),
                ("reserved", C.c_int32 * 4)]


class KernelStat_t(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int32), ("reserved", C.c_int32),
                ("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libidbf.so once; raises if it is absent (build it with paper_1809_10573_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"IDBF HIP library not built: {path} is missing "
                           "(run `python -m paper_1809_10573_amd.build`)")
    lib = C.CDLL(path)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    lib.idbf_opts_default.argtypes = [P(Opts_t)]
    lib.idbf_opts_default.restype = None
    lib.idbf_last_error.argtypes = []
    lib.idbf_last_error.restype = C.c_char_p
    lib.idbf_construct.argtypes = [P(Phase_t), VP, VP, I64, D, I32, P(Opts_t), P(VP)]
    lib.idbf_apply.argtypes = [VP, VP, VP, I64, I32, VP]
    lib.idbf_apply_adjoint.argtypes = [VP, VP, VP, I64, I32, VP]
    lib.idbf_apply_noalloc.argtypes = [VP, VP, VP, I64, I32, VP]
    lib.idbf_destroy.argtypes = [VP]
    lib.idbf_get_info.argtypes = [VP, P(Info_t)]
    lib.idbf_stats.argtypes = [VP, P(Stats_t)]
    lib.idbf_batch_proposal.argtypes = [VP, I32, I32, VP, VP, VP]
    lib.idbf_batch_sizes.argtypes = [VP, I32, I32, P(I64), P(I64), P(I64)]
    lib.idbf_batch_export.argtypes = [VP, I32, I32, VP, VP, VP, VP, VP, VP]
    lib.idbf_middle_sizes.argtypes = [VP, P(I64), P(I64)]
    lib.idbf_middle_export.argtypes = [VP, VP, VP]
    lib.idbf_sample.argtypes = [P(Phase_t), VP, VP, VP, I64, VP, I64, VP, VP]
    lib.idbf_id_batch.argtypes = [P(Phase_t), VP, VP, I32, I64, VP, VP, VP, VP, VP, VP, D, I32, I32,
                                  VP, VP, VP, VP, VP]
    lib.idbf_profile_read.argtypes = [VP, P(KernelStat_t), I32, P(I32), I32]
    lib.idbf_profile_enable.argtypes = [VP, I32]
    lib.idbf_reserve.argtypes = [VP, I64, I32]
    lib.idbf_construct_batched.argtypes = [I32, P(Phase_t), P(VP), P(VP), P(I64), P(D), P(I32), P(Opts_t),
                                           P(VP)]
    lib.idbf_apply_batched.argtypes = [I32, P(VP), P(VP), P(VP), P(I64), I32, VP]
    F32 = C.c_float
    lib.idbf_mlp_param_count.argtypes = [I32]
    lib.idbf_mlp_create.argtypes = [I32, VP, P(VP)]
    lib.idbf_mlp_destroy.argtypes = [VP]
    lib.idbf_mlp_params.argtypes = [VP, VP]
    lib.idbf_mlp_forward.argtypes = [VP, VP, I64, VP, VP]
    lib.idbf_mlp_loss_grad.argtypes = [VP, VP, VP, I64, VP, P(F32), VP]
    lib.idbf_mlp_train.argtypes = [VP, VP, VP, I64, I32, I32, F32, C.c_uint64, VP, VP]
    lib.idbf_rank_samples.argtypes = [VP, I32, I32, VP, VP]
    lib.idbf_skeleton_samples.argtypes = [VP, I32, I32, P(I32), VP, VP]
    lib.idbf_batch_skeleton_proposal.argtypes = [VP, I32, I32, VP, VP]
    lib.idbf_get_apply_config.argtypes = [VP, P(ApplyConfig_t)]
    lib.idbf_set_apply_config.argtypes = [VP, P(ApplyConfig_t)]
    lib.idbf_tune_apply.argtypes = [VP, I64, I32, C.c_char_p, VP, P(ApplyConfig_t)]
    lib.idbf_set_qr_shapes.argtypes = [C.c_uint32]
    lib.idbf_get_qr_shapes.argtypes = [P(C.c_uint32)]
    lib.idbf_tune_construct.argtypes = [P(Phase_t), VP, VP, I64, D, I32, P(Opts_t), C.c_char_p, P(C.c_uint32),
                                        P(C.c_float), P(I32)]
    lib.idbf_apply_batched_plan.argtypes = [I32, P(VP), P(VP), P(VP), P(I64), I32, VP, P(VP)]
    lib.idbf_plan_launch.argtypes = [VP, VP]
    lib.idbf_plan_destroy.argtypes = [VP]
    for name in EXPORTED:
        if name not in ("idbf_opts_default", "idbf_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != OK:
        raise IdbfError(status, load().idbf_last_error().decode())


def _phase(phase) -> Phase_t:
    return Phase_t(int(phase.kind), 0, float(phase.c0), float(phase.a), float(phase.freq),
                   float(phase.cdiv))


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dev_f64(a, device):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def _dev_i32(a, device):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32), device=device)


def _check_operand(name, x, N, want, device) -> None:
    """The C ABI takes no lengths: a vector block must be exactly (N,) or
    (N, nrhs), contiguous, of the apply's dtype and on the factorization's
    device, or the stage kernels would read past its end."""
    import torch
    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if x.dtype != want or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {want} tensor")
    if x.dim() not in (1, 2) or x.shape[0] != N:
        raise ValueError(f"{name} must have shape ({N},) or ({N}, nrhs), got {tuple(x.shape)}")
    if x.device != device:
        raise ValueError(f"{name} is on {x.device}, the factorization on {device}")


def _check_output(x, y) -> None:
    """y must match x in dtype, shape and device, be contiguous and not overlap x."""
    import torch
    if not isinstance(y, torch.Tensor) or y.dtype != x.dtype or y.shape != x.shape or not y.is_contiguous():
        raise ValueError("y must be a contiguous tensor of x's dtype and shape")
    if y.device != x.device:
        raise ValueError("y must be on x's device")
    nb = x.numel() * x.element_size()
    if nb and y.data_ptr() < x.data_ptr() + nb and x.data_ptr() < y.data_ptr() + nb:
        raise ValueError("y must not overlap x")


@dataclass
class Batch:
    rank: np.ndarray
    cand_len: np.ndarray
    mask: np.ndarray
    skel: np.ndarray
    T: np.ndarray
    T_off: np.ndarray


class Factorization:
    """A constructed IDBF living on the GPU (owns the C handle)."""

    def __init__(self, handle: int, X, Omega, allocator=None):
        self._h = C.c_void_p(handle)
        self.X, self.Omega = X, Omega
        self._allocator = allocator  # its callbacks must outlive the handle

    def close(self) -> None:
        if self._h:
            _check(load().idbf_destroy(self._h))
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = Info_t()
        _check(load().idbf_get_info(self._h, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in Info_t._fields_}

    def stats(self) -> dict:
        """idbf_stats: per level and side ("U"/"V") the rank histogram and what
        the level stores and cost, plus whole-factorization totals."""
        st = Stats_t()
        _check(load().idbf_stats(self._h, C.byref(st)))
        levels = []
        for t in range(st.levels):
            row = {}
            for side, name in ((SIDE_U, "U"), (SIDE_V, "V")):
                L = st.level[t][side]
                d = {f: getattr(L, f) for f, _ in LevelStats_t._fields_ if f != "rank_hist"}
                d["rank_hist"] = np.array(L.rank_hist[:], dtype=np.int64)
                row[name] = d
            levels.append(row)
        out = {f: getattr(st, f) for f, _ in Stats_t._fields_ if f not in ("level", "reserved")}
        out["per_level"] = levels
        return out

    def apply(self, x, y=None, dtype: int | None = None, stream=None):
        """y = K~ x for a (N,) or (N, nrhs) complex128/complex64 device tensor."""
        return self._apply(load().idbf_apply, x, y, dtype, stream)

    def apply_noalloc(self, x, y, dtype: int | None = None, stream=None):
        """idbf_apply_noalloc: y = K~ x with the library's fixed scratch array
        (no device allocation in the library; y must be given)."""
        if y is None:
            raise ValueError("apply_noalloc needs the output tensor y")
        return self._apply(load().idbf_apply_noalloc, x, y, dtype, stream)

    def apply_adjoint(self, x, y=None, dtype: int | None = None, stream=None):
        """y = K~^H x (idbf_apply_adjoint), same argument rules as apply."""
        return self._apply(load().idbf_apply_adjoint, x, y, dtype, stream)

    def _apply(self, fn, x, y, dtype, stream):
        import torch
        if dtype is None:
            dtype = C128 if x.dtype == torch.complex128 else C64
        want = torch.complex128 if dtype == C128 else torch.complex64
        _check_operand("x", x, self.X.numel(), want, self.X.device)
        if y is None:
            y = torch.empty_like(x)
        else:
            _check_output(x, y)
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        _check(fn(self._h, _ptr(x), _ptr(y), nrhs, dtype, _stream(stream)))
        return y

    def reserve(self, nrhs: int, dtype: int = C64) -> None:
        """Pre-allocate the apply workspace for up to nrhs right-hand sides."""
        _check(load().idbf_reserve(self._h, int(nrhs), int(dtype)))

    def batch(self, side: int, level: int) -> Batch:
        lib = load()
        n, ns, nt = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.idbf_batch_sizes(self._h, side, level, C.byref(n), C.byref(ns), C.byref(nt)))
        rank = np.zeros(n.value, np.int32)
        cand = np.zeros(n.value, np.int32)
        mask = np.zeros((n.value, 2), np.uint64)
        skel = np.zeros(max(ns.value, 1), np.int32)
        T = np.zeros(max(nt.value, 1), np.complex128)
        toff = np.zeros(n.value, np.int64)
        _check(lib.idbf_batch_export(self._h, side, level, rank.ctypes.data, cand.ctypes.data,
                                     mask.ctypes.data, skel.ctypes.data, T.ctypes.data,
                                     toff.ctypes.data))
        return Batch(rank, cand, mask, skel[:ns.value], T[:nt.value], toff)

    def proposal(self, side: int, level: int):
        """(proposed, used, rejected) sample counts of one level's IDs (idbf_batch_proposal)."""
        lib = load()
        n = C.c_int64()
        _check(lib.idbf_batch_sizes(self._h, side, level, C.byref(n), None, None))
        out = [np.zeros(n.value, np.int32) for _ in range(3)]
        _check(lib.idbf_batch_proposal(self._h, side, level, *[a.ctypes.data for a in out]))
        return tuple(out)

    def skeleton_proposal(self, side: int, level: int):
        """(n_prop, order (n, 64) uint8): the proposed skeleton sets of one level (idbf_batch_skeleton_proposal)."""
        lib = load()
        n = C.c_int64()
        _check(lib.idbf_batch_sizes(self._h, side, level, C.byref(n), None, None))
        k = np.zeros(n.value, np.int32)
        order = np.zeros((n.value, MAX_RANK), np.uint8)
        _check(lib.idbf_batch_skeleton_proposal(self._h, side, level, k.ctypes.data, order.ctypes.data))
        return k, order

    def apply_config(self) -> dict:
        """{'fuse', 'rhs_iter'} of the many-RHS apply (idbf_get_apply_config)."""
        cfg = ApplyConfig_t()
        _check(load().idbf_get_apply_config(self._h, C.byref(cfg)))
        return {"fuse": cfg.fuse, "rhs_iter": cfg.rhs_iter}

    def set_apply_config(self, fuse: int = None, rhs_iter: int = None) -> None:
        """Change the many-RHS apply configuration (idbf_set_apply_config); None keeps a value."""
        cur = self.apply_config()
        cfg = ApplyConfig_t()
        cfg.fuse = cur["fuse"] if fuse is None else int(fuse)
        cfg.rhs_iter = cur["rhs_iter"] if rhs_iter is None else int(rhs_iter)
        _check(load().idbf_set_apply_config(self._h, C.byref(cfg)))

    def tune_apply(self, nrhs: int, dtype: int = C64, cache_path: str | None = None, stream=None) -> dict:
        """idbf_tune_apply: time the apply configurations for (nrhs, dtype), keep the fastest."""
        cfg = ApplyConfig_t()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load().idbf_tune_apply(self._h, int(nrhs), int(dtype), path, _stream(stream), C.byref(cfg)))
        return {"fuse": cfg.fuse, "rhs_iter": cfg.rhs_iter, "from_cache": bool(cfg.from_cache), "ms": cfg.ms}

    def set_profile(self, on: bool) -> None:
        """Record (or stop recording) per-launch events for later calls (idbf_profile_enable)."""
        _check(load().idbf_profile_enable(self._h, int(bool(on))))

    def profile(self, reset: bool = True) -> dict:
        """{kernel name: {launches, ms, bytes, flops}} since the last reset (IDBF_FLAG_PROFILE)."""
        arr = (KernelStat_t * 64)()
        n = C.c_int32()
        _check(load().idbf_profile_read(self._h, arr, 64, C.byref(n), int(reset)))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms,
                                       "bytes": arr[i].bytes, "flops": arr[i].flops}
                for i in range(n.value)}

    def middle(self) -> tuple[np.ndarray, np.ndarray]:
        lib = load()
        nb, ne = C.c_int64(), C.c_int64()
        _check(lib.idbf_middle_sizes(self._h, C.byref(nb), C.byref(ne)))
        S = np.zeros(max(ne.value, 1), np.complex128)
        off = np.zeros(nb.value, np.int64)
        _check(lib.idbf_middle_export(self._h, S.ctypes.data, off.ctypes.data))
        return S[:ne.value], off


def _flags(profile: bool, force_reject: bool, allow_truncate: bool) -> int:
    return ((FLAG_PROFILE if profile else 0) | (FLAG_PROPOSER_FORCE_REJECT if force_reject else 0)
            | (FLAG_ALLOW_TRUNCATE if allow_truncate else 0))


def construct(phase, X, Omega, tol: float, leaf: int, kmax: int = 0, oversample: int = 1,
              mem_cap_bytes: int = 0, profile: bool = False, device="cuda",
              stream=None, proposer=None, proposal_margin: int = 4, seed: int = 0,
              sampler: int = SAMPLER_MOCKCHEB, force_reject: bool = False,
              allow_truncate: bool = False, skeleton_proposer=None,
              proposal_accept: float = 0.0, allocator: TorchAllocator | None = None) -> Factorization:
    """idbf_construct on device copies of X and Omega (float64, ascending)."""
    lib = load()
    Xd, Od = _dev_f64(X, device), _dev_f64(Omega, device)
    if Xd.numel() != Od.numel():
        raise ValueError("X and Omega must have the same length")
    opts = Opts_t()
    lib.idbf_opts_default(C.byref(opts))
    opts.kmax, opts.oversample, opts.mem_cap_bytes = kmax, oversample, mem_cap_bytes
    opts.flags = _flags(profile, force_reject, allow_truncate)
    opts.stream = _stream(stream)
    opts.sampler, opts.seed = int(sampler), int(seed)
    if proposer is not None:
        opts.proposer, opts.proposal_margin = proposer._h.value, int(proposal_margin)
        opts.proposal_accept = float(proposal_accept)
    if skeleton_proposer is not None:
        opts.skeleton_proposer = skeleton_proposer._h.value
    if allocator is not None:
        allocator.set(opts)
    ph = _phase(phase)
    h = C.c_void_p()
    _check(lib.idbf_construct(C.byref(ph), _ptr(Xd), _ptr(Od), Xd.numel(), float(tol), int(leaf),
                              C.byref(opts), C.byref(h)))
    return Factorization(h.value, Xd, Od, allocator)


def construct_batched(phases, Xs, Omegas, tols, leafs, kmax: int = 0, oversample: int = 1,
                      mem_cap_bytes: int = 0, profile: bool = False, device="cuda",
                      stream=None, proposer=None, proposal_margin: int = 4, seed: int = 0,
                      sampler: int = SAMPLER_MOCKCHEB, force_reject: bool = False,
                      allow_truncate: bool = False, skeleton_proposer=None,
              proposal_accept: float = 0.0, allocator: TorchAllocator | None = None) -> list:
    """idbf_construct_batched: one lockstep construction of len(phases) instances."""
    lib = load()
    n = len(phases)
    if not (len(Xs) == len(Omegas) == len(tols) == len(leafs) == n):
        raise ValueError("per-instance argument lists must have equal lengths")
    Xd = [_dev_f64(x, device) for x in Xs]
    Od = [_dev_f64(o, device) for o in Omegas]
    for x, o in zip(Xd, Od):
        if x.numel() != o.numel():
            raise ValueError("X and Omega must have the same length")
    opts = Opts_t()
    lib.idbf_opts_default(C.byref(opts))
    opts.kmax, opts.oversample, opts.mem_cap_bytes = kmax, oversample, mem_cap_bytes
    opts.flags = _flags(profile, force_reject, allow_truncate)
    opts.stream = _stream(stream)
    opts.sampler, opts.seed = int(sampler), int(seed)
    if proposer is not None:
        opts.proposer, opts.proposal_margin = proposer._h.value, int(proposal_margin)
        opts.proposal_accept = float(proposal_accept)
    if skeleton_proposer is not None:
        opts.skeleton_proposer = skeleton_proposer._h.value
    if allocator is not None:
        allocator.set(opts)
    ph = (Phase_t * n)(*[_phase(p) for p in phases])
    xp = (C.c_void_p * n)(*[_ptr(x) for x in Xd])
    op = (C.c_void_p * n)(*[_ptr(o) for o in Od])
    Ns = (C.c_int64 * n)(*[x.numel() for x in Xd])
    ts = (C.c_double * n)(*[float(t) for t in tols])
    ls = (C.c_int32 * n)(*[int(v) for v in leafs])
    out = (C.c_void_p * n)()
    _check(lib.idbf_construct_batched(n, ph, xp, op, Ns, ts, ls, C.byref(opts), out))
    return [Factorization(out[i], Xd[i], Od[i], allocator) for i in range(n)]


def release_cached_memory() -> None:
    """Free the device and pinned memory kept from destroyed factorizations
    (idbf_release_cached_memory)."""
    _check(load().idbf_release_cached_memory())


def apply_batched(facs, xs, ys=None, dtype: int | None = None, stream=None) -> list:
    """idbf_apply_batched over distinct factorizations; returns the outputs."""
    import torch
    n = len(facs)
    if len(xs) != n:
        raise ValueError("one input per factorization")
    if dtype is None:
        dtype = C128 if xs[0].dtype == torch.complex128 else C64
    want = torch.complex128 if dtype == C128 else torch.complex64
    for i, (f, x) in enumerate(zip(facs, xs)):
        _check_operand(f"xs[{i}]", x, f.X.numel(), want, f.X.device)
    if ys is None:
        ys = [torch.empty_like(x) for x in xs]
    elif len(ys) != n:
        raise ValueError("one output per factorization")
    else:
        for x, y in zip(xs, ys):
            _check_output(x, y)
    hs = (C.c_void_p * n)(*[f._h.value for f in facs])
    xp = (C.c_void_p * n)(*[_ptr(x) for x in xs])
    yp = (C.c_void_p * n)(*[_ptr(y) for y in ys])
    nr = (C.c_int64 * n)(*[1 if x.dim() == 1 else x.shape[1] for x in xs])
    _check(load().idbf_apply_batched(n, hs, xp, yp, nr, int(dtype), _stream(stream)))
    return ys


class ApplyPlan:
    """A batched apply captured once into a HIP graph (idbf_apply_batched_plan);
    launch() replays it.  The factorizations and tensors must outlive the plan."""

    def __init__(self, facs, xs, ys, dtype: int | None = None, stream=None):
        import torch
        n = len(facs)
        if len(xs) != n or len(ys) != n:
            raise ValueError("one input and one output per factorization")
        if dtype is None:
            dtype = C128 if xs[0].dtype == torch.complex128 else C64
        want = torch.complex128 if dtype == C128 else torch.complex64
        for i, (f, x, y) in enumerate(zip(facs, xs, ys)):
            _check_operand(f"xs[{i}]", x, f.X.numel(), want, f.X.device)
            _check_output(x, y)
        self._keep = (list(facs), list(xs), list(ys))
        hs = (C.c_void_p * n)(*[f._h.value for f in facs])
        xp = (C.c_void_p * n)(*[_ptr(x) for x in xs])
        yp = (C.c_void_p * n)(*[_ptr(y) for y in ys])
        nr = (C.c_int64 * n)(*[1 if x.dim() == 1 else x.shape[1] for x in xs])
        self._h = C.c_void_p()
        _check(load().idbf_apply_batched_plan(n, hs, xp, yp, nr, int(dtype), _stream(stream), C.byref(self._h)))

    def launch(self, stream=None) -> None:
        _check(load().idbf_plan_launch(self._h, _stream(stream)))

    def close(self) -> None:
        if self._h:
            _check(load().idbf_plan_destroy(self._h))
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_init(hidden: int, seed: int) -> np.ndarray:
    """He-uniform weights and zero biases in the flat parameter layout (float32)."""
    rng = np.random.default_rng(seed)
    n_in = MLP_INPUTS
    parts = [rng.uniform(-1, 1, (n_in, hidden)) * np.sqrt(6.0 / n_in), np.zeros(hidden),
             rng.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden), np.zeros(hidden),
             rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden), np.zeros(1)]
    return np.concatenate([x.ravel() for x in parts]).astype(np.float32)


class RankProposer:
    """The rank-proposal network (idbf_mlp): forward, gradient, Adam training."""

    def __init__(self, hidden: int = 128, params=None, seed: int = 0):
        lib = load()
        self.hidden = hidden
        self.n_params = lib.idbf_mlp_param_count(hidden)
        p = mlp_init(hidden, seed) if params is None else np.ascontiguousarray(params, np.float32)
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self._h = C.c_void_p()
        _check(lib.idbf_mlp_create(hidden, p.ctypes.data, C.byref(self._h)))

    def close(self) -> None:
        if self._h:
            _check(load().idbf_mlp_destroy(self._h))
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(load().idbf_mlp_params(self._h, out.ctypes.data))
        return out

    def forward(self, X, stream=None):
        import torch
        X = X.to(torch.float32).contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(load().idbf_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(y), _stream(stream)))
        return y

    def loss_grad(self, X, y, stream=None):
        import torch
        X, y = X.to(torch.float32).contiguous(), y.to(torch.float32).contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        loss = C.c_float()
        _check(load().idbf_mlp_loss_grad(self._h, _ptr(X), _ptr(y), X.shape[0], _ptr(g), C.byref(loss),
                                         _stream(stream)))
        return float(loss.value), g

    def train(self, X, y, epochs: int, batch: int = 512, lr: float = 1e-3, seed: int = 0, stream=None):
        import torch
        X, y = X.to(torch.float32).contiguous(), y.to(torch.float32).contiguous()
        losses = np.zeros(max(epochs, 1), np.float32)
        _check(load().idbf_mlp_train(self._h, _ptr(X), _ptr(y), X.shape[0], int(epochs), int(batch),
                                     float(lr), int(seed), losses.ctypes.data, _stream(stream)))
        return losses[:epochs]


def rank_samples(fac: Factorization, side: int, level: int, device="cuda"):
    """(features (n, 8), targets (n,)) float32 device tensors of one level's IDs."""
    import torch
    n = C.c_int64()
    ns, nt = C.c_int64(), C.c_int64()
    _check(load().idbf_batch_sizes(fac._h, side, level, C.byref(n), C.byref(ns), C.byref(nt)))
    F = torch.empty((n.value, MLP_INPUTS), dtype=torch.float32, device=device)
    t = torch.empty(n.value, dtype=torch.float32, device=device)
    _check(load().idbf_rank_samples(fac._h, side, level, _ptr(F), _ptr(t)))
    return F, t


def skeleton_samples(fac: Factorization, side: int, level: int, device="cuda"):
    """(features (rows, 8), targets (rows,)) float32 device tensors: one row per
    (ID, candidate) of one level, target 1 for a skeleton of the plain
    construction and 0 otherwise (idbf_skeleton_samples, padding removed)."""
    import torch
    lib = load()
    n = C.c_int64()
    _check(lib.idbf_batch_sizes(fac._h, side, level, C.byref(n), None, None))
    cmax = C.c_int32()
    _check(lib.idbf_skeleton_samples(fac._h, side, level, C.byref(cmax), None, None))
    F = torch.empty((n.value * cmax.value, MLP_INPUTS), dtype=torch.float32, device=device)
    t = torch.empty(n.value * cmax.value, dtype=torch.float32, device=device)
    _check(lib.idbf_skeleton_samples(fac._h, side, level, C.byref(cmax), _ptr(F), _ptr(t)))
    keep = t >= 0
    return F[keep], t[keep]


def sample(phase, X, Omega, rows, cols, device="cuda", stream=None):
    """K(X[rows], Omega[cols]) as a complex128 device tensor (idbf_sample)."""
    import torch
    Xd, Od = _dev_f64(X, device), _dev_f64(Omega, device)
    r, c = _dev_i32(rows, device), _dev_i32(cols, device)
    out = torch.empty((r.numel(), c.numel()), dtype=torch.complex128, device=device)
    ph = _phase(phase)
    _check(load().idbf_sample(C.byref(ph), _ptr(Xd), _ptr(Od), _ptr(r), r.numel(), _ptr(c),
                              c.numel(), _ptr(out), _stream(stream)))
    return out


def set_qr_shapes(mask: int) -> None:
    """Process-wide wave shapes of the QR kernels for 65..112 sampled rows
    (idbf_set_qr_shapes; bit b set: short wavefronts for the b-th range)."""
    _check(load().idbf_set_qr_shapes(int(mask)))


def qr_shapes() -> int:
    """The current QR shape mask (idbf_get_qr_shapes)."""
    m = C.c_uint32()
    _check(load().idbf_get_qr_shapes(C.byref(m)))
    return int(m.value)


def tune_construct(phase, X, Omega, tol: float, leaf: int, kmax: int = 0, oversample: int = 1,
                   cache_path: str | None = None, device="cuda", stream=None) -> dict:
    """idbf_tune_construct: times the ID kernels of this construction per QR
    shape mask, sets the fastest process-wide and returns
    {"mask", "ms", "from_cache"}."""
    lib = load()
    Xd, Od = _dev_f64(X, device), _dev_f64(Omega, device)
    if Xd.numel() != Od.numel():
        raise ValueError("X and Omega must have the same length")
    opts = Opts_t()
    lib.idbf_opts_default(C.byref(opts))
    opts.kmax, opts.oversample = kmax, oversample
    opts.stream = _stream(stream)
    ph = _phase(phase)
    m, ms, cached = C.c_uint32(), C.c_float(), C.c_int32()
    _check(lib.idbf_tune_construct(C.byref(ph), _ptr(Xd), _ptr(Od), Xd.numel(), float(tol), int(leaf),
                                   C.byref(opts), cache_path.encode() if cache_path else None, C.byref(m),
                                   C.byref(ms), C.byref(cached)))
    return {"mask": int(m.value), "ms": float(ms.value), "from_cache": bool(cached.value)}


def id_batch(phase, X, Omega, side: int, cand_idx, cand_beg, cand_len, allow_idx, allow_beg,
             allow_len, tol: float, kmax: int = 0, oversample: int = 1, device="cuda", stream=None):
    """idbf_id_batch; returns host arrays (rank, mask (n, 2), skel (n, 128), T (n, 4096))."""
    import torch
    Xd, Od = _dev_f64(X, device), _dev_f64(Omega, device)
    ci, cb, cl = (_dev_i32(a, device) for a in (cand_idx, cand_beg, cand_len))
    ai, abg, al = (_dev_i32(a, device) for a in (allow_idx, allow_beg, allow_len))
    n = cb.numel()
    rank = torch.zeros(n, dtype=torch.int32, device=device)
    mask = torch.zeros((n, 2), dtype=torch.int64, device=device)
    skel = torch.full((n, MAX_CAND), -1, dtype=torch.int32, device=device)
    T = torch.zeros((n, SLOT), dtype=torch.complex128, device=device)
    ph = _phase(phase)
    _check(load().idbf_id_batch(C.byref(ph), _ptr(Xd), _ptr(Od), side, n, _ptr(ci), _ptr(cb),
                                _ptr(cl), _ptr(ai), _ptr(abg), _ptr(al), float(tol), int(kmax),
                                int(oversample), _ptr(rank), _ptr(mask), _ptr(skel), _ptr(T),
                                _stream(stream)))
    torch.cuda.synchronize()
    return (rank.cpu().numpy(), mask.cpu().numpy().view(np.uint64), skel.cpu().numpy(),
            T.cpu().numpy())
