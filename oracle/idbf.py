"""IDBF construction and apply (oracle; test infrastructure).

Sections 2.2 (LRCS), 2.3 (MSCS) and 2.4 (recursive MSCS), eq. finishIDBF:

    K ~= U^L U^{L-1} ... U^h S^h V^h ... V^{L-1} V^L.

Trees.  N = 2^L n0; the row tree T_X and column tree T_Omega are dyadic over
index ranges: a node at depth d (root depth 0) with index r covers
[r N/2^d, (r+1) N/2^d).  Leaves sit at depth L and hold n0 points.

Notation for level t = 1..H, H = floor(L/2) (level t builds the t-th factor
pair from the outside in: t = 1 is U^L / V^L of the paper):

* U_t holds one row ID (rID) per pair (R at depth L-t+1, C at depth t):
    candidate rows   t = 1: the n0 rows of leaf R;
                     t > 1: skel_r(2R, C/2) ++ skel_r(2R+1, C/2) from U_{t-1}
                     (the merged children of Figure rc: rbar_i = rhat_{2i-1} U rhat_{2i});
    allowed columns  t = 1: all columns of C;
                     t > 1: ++ over C'' at depth L-t+2 below C of
                     skel_c(C'', ancestor of R at depth t-1) from V_{t-1}.
* V_t holds one column ID (cID) per pair (C at depth L-t+1, R at depth t):
    candidate cols   t = 1: the n0 columns of leaf C;
                     t > 1: skel_c(2C, R/2) ++ skel_c(2C+1, R/2) from V_{t-1};
    allowed rows     ++ over R'' at depth L-t+1 below R of
                     skel_r(R'', ancestor of C at depth t) from U_t
                     (the cIDs of LRCS act on the row-skeletonized matrix).
* S: with d = L-H+1, for every R, C' at depth d the block
    K(skel_r(R, ancestor of C' at depth H), skel_c(C', ancestor of R at depth H)).

Each ID samples s = min(t |cand|, |allowed|) points of its allowed set by the
Mock-Chebyshev rule (the t k rows of eq. pivotedQR2 with k = |cand|, i.e.
k = min{m, n} of the ID's matrix; the paper's experiments use t = 1,
Section 3), or all of them with ``sample_all`` (used to pin the assembly: then every ID is exact to
its tolerance on the whole block).  An rID of A(cand, allowed) is the cID of
the transpose A(cand, s)^T (plain transpose; U = Lambda [I T]^T).

Readings: H = floor(L/2) for odd L too (the paper assumes L even); for odd L
the middle factor pairs nodes at depth L-H+1 and has 8m blocks instead of 4m.
The factor count is H U-factors, H V-factors and one S (the stopping count of
Section 2.4 and Figure exsfac; the Introduction's range U^L..U^{L/2} is one
too many).  The block orders of U^{L-1} and V^{L-1} in eq. expressUSV_L-1 are
read as blockdiag(U11, U21, U12, U22) and blockdiag(V11, V12, V21, V22), as in
eq. expressUSV.  For L <= 1 (H = 0) the factorization is K itself.

Apply (eq. finishIDBF read right to left):
    V stage t:  z_t(C, R) = u[skel] + T u[red],  u = x[C] (t = 1) or
                z_{t-1}(2C, R/2) ++ z_{t-1}(2C+1, R/2);
    S stage:    w_H(R, C_H) = sum over C' at depth d below C_H of S(R, C') z_H(C', anc_H(R));
    U stage t:  v = U_{R,C} w_t(R, C) (v[skel] = w, v[red] = T^T w) is added
                into y[R] (t = 1) or into w_{t-1}(2R, C/2) ++ w_{t-1}(2R+1, C/2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .interp import column_id
from .kernel import entries
from .sampling import mock_chebyshev, random_positions

@dataclass
class IDRecord:
    cand: np.ndarray      # global indices of the candidates (ascending)
    skel: np.ndarray      # global indices of the skeleton (ascending)
    skelpos: np.ndarray   # positions of skel within cand
    redpos: np.ndarray    # positions of the redundant candidates within cand
    T: np.ndarray         # (k, c-k): redundant ~= skeleton interpolation
    nsamples: int
    rdiag: np.ndarray     # |R_jj| of the pivoted QR, j < k


@dataclass
class Factors:
    N: int
    leaf: int
    L: int
    H: int
    tol: float
    U: dict = field(default_factory=dict)    # U[t][(node, partner)] -> IDRecord
    V: dict = field(default_factory=dict)    # V[t][(node, partner)] -> IDRecord
    S: dict = field(default_factory=dict)    # S[(r, c)] -> complex block
    dense: np.ndarray | None = None          # H == 0: K itself

    @property
    def d(self) -> int:
        return self.L - self.H + 1

    def nnz(self) -> int:
        """Stored complex entries: every T block plus every S block (or K when H = 0)."""
        if self.dense is not None:
            return int(self.dense.size)
        n = sum(r.T.size for t in self.U for r in self.U[t].values())
        n += sum(r.T.size for t in self.V for r in self.V[t].values())
        n += sum(b.size for b in self.S.values())
        return int(n)


def tree_sizes(N: int, leaf: int) -> tuple[int, int]:
    """(L, H) for N = 2^L leaf; both N and leaf must be powers of two."""
    if N <= 0 or leaf <= 0 or N % leaf or (N & (N - 1)) or (leaf & (leaf - 1)):
        raise ValueError("N and leaf must be powers of two with leaf <= N")
    L = (N // leaf).bit_length() - 1
    return L, L // 2


def _interp(B, tol, kmax, cand):
    cid = column_id(B, tol, kmax)
    return IDRecord(cand=cand, skel=cand[cid.skel], skelpos=cid.skel, redpos=cid.red,
                    T=cid.T, nsamples=B.shape[0], rdiag=cid.rdiag)


def sample_count(c: int, n_allowed: int, oversample: int, smax: int = 0) -> int:
    """s = min(t |cand|, |allowed|): the t k rows of eq. pivotedQR2 (Section
    2.1) with k = |cand|.  smax > 0 adds a cap the paper does not have (an
    explicit option for experiments only; no parity test uses it)."""
    s = min(oversample * c, n_allowed)
    return s if smax <= 0 else min(s, smax)


def _samples(coords_of_allowed, allowed, c, oversample, sample_all, smax, sampler="mockcheb", key=None):
    s = len(allowed) if sample_all else sample_count(c, len(allowed), oversample, smax)
    if sampler == "random":
        seed, level, side, q = key
        return allowed[random_positions(seed, level, side, q, len(allowed), s)]
    return allowed[mock_chebyshev(coords_of_allowed, s)]


@dataclass
class _Context:
    """What every ID of one construction shares (held per worker process)."""
    phase: object
    X: np.ndarray
    Omega: np.ndarray
    tol: float
    kmax: int
    oversample: int
    sample_all: bool
    smax: int
    sampler: str


_CTX: _Context | None = None


def _set_context(ctx: _Context) -> None:
    global _CTX
    _CTX = ctx


def _one_id(job) -> IDRecord:
    """One ID of a level (Section 2.1): samples of the allowed set, the sampled
    block of the candidates, its column ID.  side 0: a row ID of
    A(cand, allowed) as the column ID of K(cand, samples)^T; side 1: a column
    ID of K(samples, cand)."""
    side, cand, allowed, key = job
    c = _CTX
    coords = c.Omega[allowed] if side == 0 else c.X[allowed]
    samp = _samples(coords, allowed, len(cand), c.oversample, c.sample_all, c.smax, c.sampler, key)
    if side == 0:
        B = entries(c.phase, c.X, c.Omega, cand, samp).T            # s x c
    else:
        B = entries(c.phase, c.X, c.Omega, samp, cand)              # s x c
    return _interp(B, c.tol, c.kmax, cand)


def build(phase, X, Omega, leaf: int, tol: float, kmax: int = 0, oversample: int = 1,
          sample_all: bool = False, smax: int = 0, sampler: str = "mockcheb",
          seed: int = 0, workers: int = 0) -> Factors:
    """Construct the IDBF of K(X, Omega) level by level (Sections 2.2-2.4).

    oversample is the parameter t of Section 2.1: s = min(t |cand|, |allowed|)
    samples per ID (eq. pivotedQR2); smax > 0 caps s, a departure from the
    paper kept only as an explicit option.  sampler "mockcheb" (default)
    or "random" (uniform, sampling.random_positions with this seed; the ID of
    node n and partner p at level t is q = p 2^(L-t+1) + n, side 0 = U, 1 = V).
    workers > 1 computes the independent IDs of each level in that many
    processes (the same IDs, in any order; used to time the oracle on all
    host cores).
    """
    if sampler not in ("mockcheb", "random"):
        raise ValueError("sampler must be 'mockcheb' or 'random'")
    if oversample < 1:
        raise ValueError("oversample must be >= 1")
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    N = len(X)
    if len(Omega) != N:
        raise ValueError("X and Omega must have the same length")
    L, H = tree_sizes(N, leaf)
    F = Factors(N=N, leaf=leaf, L=L, H=H, tol=tol)
    if H == 0:
        idx = np.arange(N)
        F.dense = entries(phase, X, Omega, idx, idx)
        return F
    ctx = _Context(phase, X, Omega, tol, kmax, oversample, sample_all, smax, sampler)
    pool = None
    if workers > 1:
        import multiprocessing
        pool = multiprocessing.get_context("fork").Pool(workers, initializer=_set_context, initargs=(ctx,))
    else:
        _set_context(ctx)

    def run(jobs):
        if pool is None:
            return [_one_id(j) for j in jobs]
        return pool.map(_one_id, jobs, chunksize=max(1, len(jobs) // (8 * workers)))

    try:
        for t in range(1, H + 1):
            nn, npart = 1 << (L - t + 1), 1 << t
            # U_t: row IDs of (R at depth L-t+1, C at depth t)
            keys, jobs = [], []
            for r in range(nn):
                for p in range(npart):
                    if t == 1:
                        cand = np.arange(r * leaf, (r + 1) * leaf)
                        allowed = np.arange(p * (N // 2), (p + 1) * (N // 2))
                    else:
                        Up = F.U[t - 1]
                        cand = np.concatenate([Up[(2 * r, p >> 1)].skel, Up[(2 * r + 1, p >> 1)].skel])
                        sh = L - 2 * t + 2
                        Vp = F.V[t - 1]
                        allowed = np.concatenate([Vp[(cc, r >> sh)].skel
                                                  for cc in range(p << sh, (p + 1) << sh)])
                    keys.append((r, p))
                    jobs.append((0, cand, allowed, (seed, t, 0, p * nn + r)))
            U = dict(zip(keys, run(jobs)))
            F.U[t] = U
            # V_t: column IDs of (C at depth L-t+1, R at depth t)
            keys, jobs = [], []
            for cnode in range(nn):
                for p in range(npart):
                    if t == 1:
                        cand = np.arange(cnode * leaf, (cnode + 1) * leaf)
                    else:
                        Vp = F.V[t - 1]
                        cand = np.concatenate([Vp[(2 * cnode, p >> 1)].skel,
                                               Vp[(2 * cnode + 1, p >> 1)].skel])
                    sh = L - 2 * t + 1
                    allowed = np.concatenate([U[(rr, cnode >> sh)].skel
                                              for rr in range(p << sh, (p + 1) << sh)])
                    keys.append((cnode, p))
                    jobs.append((1, cand, allowed, (seed, t, 1, p * nn + cnode)))
            F.V[t] = dict(zip(keys, run(jobs)))
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    d = F.d
    sh = d - H
    for r in range(1 << d):
        for cc in range(1 << d):
            rows = F.U[H][(r, cc >> sh)].skel
            cols = F.V[H][(cc, r >> sh)].skel
            F.S[(r, cc)] = entries(phase, X, Omega, rows, cols)
    return F


def apply(F: Factors, x) -> np.ndarray:
    """y = U^L ... U^h S^h V^h ... V^L x (eq. finishIDBF), x of shape (N,) or (N, nrhs)."""
    x = np.asarray(x, dtype=np.complex128)
    if x.shape[0] != F.N:
        raise ValueError("x has the wrong number of rows")
    if F.dense is not None:
        return F.dense @ x
    L, H, leaf, d = F.L, F.H, F.leaf, F.d
    tail = x.shape[1:]
    z = None
    for t in range(1, H + 1):
        zt = {}
        for (cnode, p), rec in F.V[t].items():
            if t == 1:
                u = x[cnode * leaf:(cnode + 1) * leaf]
            else:
                u = np.concatenate([z[(2 * cnode, p >> 1)], z[(2 * cnode + 1, p >> 1)]])
            zt[(cnode, p)] = u[rec.skelpos] + rec.T @ u[rec.redpos]
        z = zt
    sh = d - H
    w = {}
    for r in range(1 << d):
        for q in range(1 << H):
            acc = np.zeros((len(F.U[H][(r, q)].skel),) + tail, dtype=np.complex128)
            for cc in range(q << sh, (q + 1) << sh):
                acc += F.S[(r, cc)] @ z[(cc, r >> sh)]
            w[(r, q)] = acc
    y = np.zeros_like(x)
    for t in range(H, 0, -1):
        wn = {}
        for (r, p), rec in F.U[t].items():
            v = np.zeros((len(rec.cand),) + tail, dtype=np.complex128)
            v[rec.skelpos] = w[(r, p)]
            v[rec.redpos] = rec.T.T @ w[(r, p)]
            if t == 1:
                y[r * leaf:(r + 1) * leaf] += v
            else:
                k1 = len(F.U[t - 1][(2 * r, p >> 1)].skel)
                for child, part in ((2 * r, v[:k1]), (2 * r + 1, v[k1:])):
                    key = (child, p >> 1)
                    wn[key] = wn[key] + part if key in wn else part.copy()
        w = wn
    return y


def apply_adjoint(F: Factors, x) -> np.ndarray:
    """y = K~^H x, the conjugate transpose of apply: the factors of
    eq. (finishIDBF) in reverse order, each conjugate transposed.  x is indexed
    by the rows of K (X), y by its columns (Omega); (N,) or (N, nrhs).

    U_t^H: each ID (r, p) reads the candidate segment its forward stage writes
    and returns v[skel] + conj(T) v[red].  S^H: the V_H ID (C', p) collects
    S(R, C')^H w(R, C' >> sh) over R >> sh == p.  V_t^H: the IDs (C, 2P) and
    (C, 2P + 1) both write their shared candidate segment, e[skel] = z and
    e[red] = T^H z, summed.
    """
    x = np.asarray(x, dtype=np.complex128)
    if x.shape[0] != F.N:
        raise ValueError("x has the wrong number of rows")
    if F.dense is not None:
        return F.dense.conj().T @ x
    L, H, leaf, d = F.L, F.H, F.leaf, F.d
    tail = x.shape[1:]
    w = None
    for t in range(1, H + 1):
        wt = {}
        for (r, p), rec in F.U[t].items():
            if t == 1:
                v = x[r * leaf:(r + 1) * leaf]
            else:
                v = np.concatenate([w[(2 * r, p >> 1)], w[(2 * r + 1, p >> 1)]])
            wt[(r, p)] = v[rec.skelpos] + rec.T.conj() @ v[rec.redpos]
        w = wt
    sh = d - H
    z = {}
    for cc in range(1 << d):
        for p in range(1 << H):
            acc = np.zeros((len(F.V[H][(cc, p)].skel),) + tail, dtype=np.complex128)
            for r in range(p << sh, (p + 1) << sh):
                acc += F.S[(r, cc)].conj().T @ w[(r, cc >> sh)]
            z[(cc, p)] = acc
    y = np.zeros_like(x)
    for t in range(H, 0, -1):
        zn = {}
        for (cnode, p), rec in F.V[t].items():
            e = np.zeros((len(rec.cand),) + tail, dtype=np.complex128)
            e[rec.skelpos] = z[(cnode, p)]
            e[rec.redpos] = rec.T.conj().T @ z[(cnode, p)]
            if t == 1:
                y[cnode * leaf:(cnode + 1) * leaf] += e
            else:
                k1 = len(F.V[t - 1][(2 * cnode, p >> 1)].skel)
                for child, part in ((2 * cnode, e[:k1]), (2 * cnode + 1, e[k1:])):
                    key = (child, p >> 1)
                    zn[key] = zn[key] + part if key in zn else part.copy()
        z = zn
    return y


def densify(F: Factors) -> np.ndarray:
    """The N x N matrix the factorization represents (apply to the identity)."""
    return apply(F, np.eye(F.N, dtype=np.complex128))


def _offsets(recs: dict, nn: int, npart: int) -> dict:
    """Start of each ID's skeleton segment when IDs are laid out in the order
    q = partner * nn + node (the order of Figures exlfac and rlfac at level 1)."""
    off, pos = {}, 0
    for p in range(npart):
        for n in range(nn):
            off[(n, p)] = pos
            pos += len(recs[(n, p)].skel)
    off["total"] = pos
    return off


def factor_matrices(F: Factors) -> list:
    """Explicit factors [U_1, ..., U_H, S, V_H, ..., V_1] whose product is densify(F).

    Rows/columns of the level-t factors follow the ID order q = partner * 2^(L-t+1)
    + node; V_t maps level t-1 coefficients to level t ones, U_t the reverse.
    """
    if F.dense is not None:
        return [F.dense.copy()]
    L, H, leaf, N = F.L, F.H, F.leaf, F.N
    offV, offU = {}, {}
    for t in range(1, H + 1):
        nn, npart = 1 << (L - t + 1), 1 << t
        offV[t] = _offsets(F.V[t], nn, npart)
        offU[t] = _offsets(F.U[t], nn, npart)
    Vs, Us = [], []
    for t in range(1, H + 1):
        nn = 1 << (L - t + 1)
        ncol = N if t == 1 else offV[t - 1]["total"]
        Vm = np.zeros((offV[t]["total"], ncol), dtype=np.complex128)
        for (cnode, p), rec in F.V[t].items():
            base = cnode * leaf if t == 1 else offV[t - 1][(2 * cnode, p >> 1)]
            r0 = offV[t][(cnode, p)]
            for i, sp in enumerate(rec.skelpos):
                Vm[r0 + i, base + sp] = 1.0
                Vm[r0 + i, base + rec.redpos] = rec.T[i]
        Vs.append(Vm)
        nrow = N if t == 1 else offU[t - 1]["total"]
        Um = np.zeros((nrow, offU[t]["total"]), dtype=np.complex128)
        for (r, p), rec in F.U[t].items():
            base = r * leaf if t == 1 else offU[t - 1][(2 * r, p >> 1)]
            c0 = offU[t][(r, p)]
            for i, sp in enumerate(rec.skelpos):
                Um[base + sp, c0 + i] = 1.0
                Um[base + rec.redpos, c0 + i] = rec.T[i]
        Us.append(Um)
    d, sh = F.d, F.d - F.H
    Sm = np.zeros((offU[H]["total"], offV[H]["total"]), dtype=np.complex128)
    for (r, cc), blk in F.S.items():
        r0 = offU[H][(r, cc >> sh)]
        c0 = offV[H][(cc, r >> sh)]
        Sm[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk
    return Us + [Sm] + Vs[::-1]
