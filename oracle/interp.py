"""Linear-scaling interpolative decomposition (oracle; test infrastructure).

Section 2.1, Lemma 2.1 and eqs. pivotedQR / pivotedQR2 / acc / R2:

  A_{s,:} Lambda = Q [R_1 R_2]   (rank-revealing QR of the sampled rows)
  k_eps  from the diagonal of R_1                                (eq. acc)
  T      = R_1(1:k,1:k)^{-1} [R_1(1:k, k+1:) R_2(1:k, :)]        (eq. R2)
  A     ~= A_{:,q} [I T] Lambda^*                                (column ID)

The rank-revealing QR is Householder QR with column pivoting, written out
here step by step.  Readings taken where the paper leaves details open:

* Pivot rule.  At step j the remaining columns' residual norms (recomputed
  from scratch, rows j..s-1) are nu_l; M = max nu_l.  The pivot is the column
  with the smallest original index among those with nu_l >= (1 - PIVOT_TIE_REL) M.
  For matrices whose residual norms are distinct by more than that relative
  gap this is LAPACK ?geqp3's choice; the band makes the choice reproducible
  when norms tie in exact arithmetic (every column of a unimodular kernel
  block has the same norm, so the first pivot is always such a tie).
* epsilon-rank (eq. acc).  The factorization stops before step j >= 1 when
  M <= eps * |R_00| (M is |R_jj| up to the tie band), so k_eps counts the
  diagonal entries above eps |R_00|.  Read literally, eq. acc would also keep
  the first entry that falls below eps |R_00|; that makes R_1(1:k,1:k)
  singular on exactly rank-deficient blocks, so the count excludes it.
  k_eps >= 1; an all-zero block keeps its first column with T = 0.
* Rank cap.  ``kmax > 0`` stops after kmax steps (the "rank parameter k").
* Skeleton order.  The skeleton set q and the redundant set p are returned
  in ascending position order, with the rows and columns of T permuted to
  match.  This does not change A_{:,q} [I T] Lambda^*.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_triangular

PIVOT_TIE_REL = 1e-8


@dataclass
class ColumnID:
    """Column ID of a matrix B (s x c): B[:, red] ~= B[:, skel] @ T."""

    skel: np.ndarray      # ascending positions of skeleton columns, length k
    red: np.ndarray       # ascending positions of redundant columns, length c - k
    T: np.ndarray         # (k, c - k) complex128, rows follow skel, columns follow red
    pivots: np.ndarray    # positions in the order the QR picked them (length k)
    rdiag: np.ndarray     # |R_jj| for j < k

    @property
    def rank(self) -> int:
        return len(self.skel)


def column_id(B, tol: float, kmax: int = 0, among=None) -> ColumnID:
    """(tol, kmax)-cID of B by column-pivoted Householder QR (Lemma 2.1, eqs. acc, R2).

    ``among`` (positions; the learned skeleton proposal, not in the paper)
    restricts the pivot search to those columns: the same steps, the
    eps-rank rule still taken against the largest column norm of all of B
    (|R_00| of the unrestricted QR), and at most len(among) steps.  If no
    column of ``among`` is above that threshold the proposal is unusable:
    None."""
    R = np.array(B, dtype=np.complex128, copy=True)
    s, c = R.shape
    if s == 0 or c == 0:
        raise ValueError("column_id needs a non-empty matrix")
    kcap = min(s, c) if kmax <= 0 else min(s, c, kmax)
    if among is not None:
        among = np.asarray(among, dtype=np.int64)
        if len(among) < 1 or len(np.unique(among)) != len(among) or among.min() < 0 or among.max() >= c:
            raise ValueError("among must name distinct columns of B")
        kcap = min(kcap, len(among))
    order = np.arange(c)           # order[p]: original position of the column now at p
    r00 = 0.0
    rdiag = []
    k = 0
    for j in range(kcap):
        nu = np.linalg.norm(R[j:, j:], axis=0)          # residual norms of columns j..c-1
        if j == 0:
            r00 = nu.max()
            if r00 == 0.0:
                break
        if among is not None:
            nu = np.where(np.isin(order[j:], among), nu, -1.0)
        M = nu.max()
        if (j > 0 or among is not None) and M <= tol * r00:
            break
        near = np.nonzero(nu >= (1.0 - PIVOT_TIE_REL) * M)[0]
        p = j + near[np.argmin(order[j + near])]
        if p != j:
            R[:, [j, p]] = R[:, [p, j]]
            order[[j, p]] = order[[p, j]]
        # Householder reflector H = I - 2 v v^H / (v^H v) with H x = alpha e_1.
        x = R[j:, j].copy()
        xnorm = np.linalg.norm(x)
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -phase * xnorm
        v = x.copy()
        v[0] -= alpha
        vv = np.vdot(v, v).real
        if vv > 0.0:
            R[j:, j:] -= np.outer(v, (2.0 / vv) * (v.conj() @ R[j:, j:]))
        R[j, j] = alpha
        R[j + 1:, j] = 0.0
        rdiag.append(abs(alpha))
        k = j + 1
    if k == 0:
        if r00 > 0.0:               # a restriction none of whose columns is kept
            return None
        skel = np.array([0])        # all-zero block: keep the first column, T = 0
        red = np.arange(1, c)
        return ColumnID(skel, red, np.zeros((1, c - 1), dtype=np.complex128),
                        np.array([0]), np.array([0.0]))
    T_piv = solve_triangular(R[:k, :k], R[:k, k:]) if k < c else np.zeros((k, 0), np.complex128)
    piv = order[:k].copy()
    rest = order[k:]
    skel = np.sort(piv)
    red = np.sort(rest)
    rows = np.argsort(piv)          # pivot-order row of each ascending skeleton
    cols = np.argsort(rest)         # current column of each ascending redundant position
    T = T_piv[rows][:, cols]
    return ColumnID(skel, red, T, piv, np.array(rdiag))
