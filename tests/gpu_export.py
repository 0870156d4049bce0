"""Test helper: the GPU construction's factors, exported through the C ABI
(idbf_batch_export, idbf_middle_export), in the oracle's terms.

The index algebra that names each ID's candidate and allowed sets is the
tree algebra of Sections 2.2-2.4 (the same one ``oracle.build`` follows); here
it is applied to the GPU's own skeletons, so an ID can be recomputed by the
oracle on exactly the sets the GPU saw, and the exported factors can be
applied by ``oracle.apply``.  Only tests import this module.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle.idbf import IDRecord


class GpuLevels:
    """Exported per-level arrays of a Factorization."""

    def __init__(self, fac, with_T: bool = True):
        from paper_1809_10573_amd import binding as B
        info = fac.info()
        self.N, self.leaf, self.L, self.H = info["N"], info["leaf"], info["L"], info["H"]
        self.batches = {}
        self._bits = {}
        for t in range(1, self.H + 1):
            for side in (B.SIDE_U, B.SIDE_V):
                b = fac.batch(side, t)
                offs = np.concatenate([[0], np.cumsum(b.rank, dtype=np.int64)])
                self.batches[(side, t)] = (b, offs)
        self.SIDE_U, self.SIDE_V = B.SIDE_U, B.SIDE_V

    def bits(self, side: int, t: int) -> np.ndarray:
        """(n_ids, 128) bool: candidate l of ID q is a skeleton (the 128-bit masks)."""
        if (side, t) not in self._bits:
            b, _ = self.batches[(side, t)]
            m = np.ascontiguousarray(b.mask, dtype=np.uint64).view(np.uint8).reshape(len(b.rank), 16)
            self._bits[(side, t)] = np.unpackbits(m, axis=1, bitorder="little").astype(bool)
        return self._bits[(side, t)]

    def skel(self, side: int, t: int, node: int, partner: int) -> np.ndarray:
        b, offs = self.batches[(side, t)]
        q = partner * (1 << (self.L - t + 1)) + node
        return b.skel[offs[q]:offs[q + 1]]

    def cand(self, side: int, t: int, q: int) -> np.ndarray:
        nn = 1 << (self.L - t + 1)
        node, p = q % nn, q // nn
        if t == 1:
            return np.arange(node * self.leaf, (node + 1) * self.leaf)
        return np.concatenate([self.skel(side, t - 1, 2 * node, p >> 1),
                               self.skel(side, t - 1, 2 * node + 1, p >> 1)])

    def sets(self, side: int, t: int, q: int):
        """(cand, allowed) global index sets of ID q = partner 2^(L-t+1) + node."""
        N, L, leaf = self.N, self.L, self.leaf
        nn = 1 << (L - t + 1)
        node, p = q % nn, q // nn
        if t == 1:
            cand = np.arange(node * leaf, (node + 1) * leaf)
        else:
            cand = np.concatenate([self.skel(side, t - 1, 2 * node, p >> 1),
                                   self.skel(side, t - 1, 2 * node + 1, p >> 1)])
        # the allowed set joins the skeletons of 2^sh consecutive IDs of the
        # other side (nodes p 2^sh .. (p + 1) 2^sh - 1, one partner): in the ID
        # numbering partner * nodes + node they are one contiguous run
        if side == self.SIDE_U:
            if t == 1:
                allowed = np.arange(p * (N // 2), (p + 1) * (N // 2))
            else:
                sh = L - 2 * t + 2
                allowed = self.run(self.SIDE_V, t - 1, (node >> sh) * (2 * nn) + (p << sh), 1 << sh)
        else:
            sh = L - 2 * t + 1
            allowed = self.run(self.SIDE_U, t, (node >> sh) * nn + (p << sh), 1 << sh)
        return cand, allowed

    def run(self, side: int, t: int, q0: int, count: int) -> np.ndarray:
        """Skeletons of IDs q0 .. q0 + count - 1 of one level, joined in order."""
        b, offs = self.batches[(side, t)]
        return b.skel[offs[q0]:offs[q0 + count]]

    def record(self, side: int, t: int, q: int) -> IDRecord:
        """ID q as an oracle record (T as (k, c - k), rows ascending skeletons)."""
        b, offs = self.batches[(side, t)]
        cand = self.cand(side, t, q)
        c, k = int(b.cand_len[q]), int(b.rank[q])
        bits = self.bits(side, t)[q, :c]
        skelpos, redpos = np.nonzero(bits)[0], np.nonzero(~bits)[0]
        r = c - k
        flat = b.T[b.T_off[q]:b.T_off[q] + k * r]
        T = flat.reshape(r, k).T if side == self.SIDE_V else flat.reshape(k, r)
        return IDRecord(cand=cand, skel=b.skel[offs[q]:offs[q + 1]], skelpos=skelpos, redpos=redpos,
                        T=T, nsamples=0, rdiag=np.zeros(0))


def to_oracle_factors(fac, tol: float) -> oracle.Factors:
    """The GPU's factors as an oracle.Factors (for oracle.apply)."""
    G = GpuLevels(fac)
    F = oracle.Factors(N=G.N, leaf=G.leaf, L=G.L, H=G.H, tol=tol)
    if G.H == 0:
        S, off = fac.middle()
        F.dense = S[:G.N * G.N].reshape(G.N, G.N).T.copy()
        return F
    for t in range(1, G.H + 1):
        nn, npart = 1 << (G.L - t + 1), 1 << t
        for side, store in ((G.SIDE_U, F.U), (G.SIDE_V, F.V)):
            store[t] = {(q % nn, q // nn): G.record(side, t, q) for q in range(nn * npart)}
    S, off = fac.middle()
    d, H = F.d, F.H
    sh = d - H
    for r in range(1 << d):
        for cc in range(1 << d):
            rl = len(F.U[H][(r, cc >> sh)].skel)
            cl = len(F.V[H][(cc, r >> sh)].skel)
            b = ((cc >> sh) * (1 << d) + r) * (1 << sh) + (cc & ((1 << sh) - 1))
            F.S[(r, cc)] = S[off[b]:off[b] + rl * cl].reshape(cl, rl).T
    return F


def same_factors(a, b):
    """Two factorizations hold the same factors bit for bit (entries in use)."""
    from paper_1809_10573_amd import binding as B
    ia, ib = a.info(), b.info()
    for key in ("L", "H", "nnz_T", "nnz_S", "n_skel", "rank_max", "rank_min"):
        assert ia[key] == ib[key], key
    for side in (B.SIDE_U, B.SIDE_V):
        for t in range(1, ia["H"] + 1):
            x, y = a.batch(side, t), b.batch(side, t)
            for f in ("rank", "cand_len", "mask", "skel", "T_off"):
                assert np.array_equal(getattr(x, f), getattr(y, f)), (side, t, f)
            # T entries in use (each ID reserves an upper bound; the tail is never written)
            for q in range(len(x.rank)):
                n = int(x.rank[q]) * int(x.cand_len[q] - x.rank[q])
                o = int(x.T_off[q])
                assert np.array_equal(x.T[o:o + n], y.T[o:o + n]), (side, t, q)
    Sa, oa = a.middle()
    Sb, ob = b.middle()
    assert np.array_equal(oa, ob)
    ends = np.append(oa[1:], len(Sa))
    for o, e in zip(oa, ends):  # a block's reservation is rounded up to even: skip its last slot
        assert np.array_equal(Sa[o:e - 1], Sb[o:e - 1])
