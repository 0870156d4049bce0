"""CPU FP64 reference ("oracle") for the interpolative decomposition butterfly
factorization (IDBF) of Pang, Ho and Yang, arXiv:1809.10573.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
it shares no code with that path: the two meet only through the seeded inputs
of ``paper_1809_10573_amd/inputs.py``, which hold none of the method's arithmetic.

Everything here is plain NumPy/SciPy in float64 / complex128, slow and written
to be checked against the paper by eye:

* ``kernel``   -- entries of K(x, xi) = exp(2 pi i Phi(x, xi)) (Introduction;
                  Example 1), the dense O(N^2) matvec, and the closed forms
                  (DFT, constant-c FIO) that pin it.
* ``interp``   -- the interpolative decomposition by column-pivoted Householder
                  QR of Lemma 2.1 and the epsilon-rank / truncated interpolation
                  solve of Section 2.1 (eqs. pivotedQR2, acc, R2); row IDs as
                  column IDs of the transpose; the ID on a given skeleton
                  (the learned proposal's accept path).
* ``sampling`` -- Mock-Chebyshev sample selection (Section 2.1).
* ``idbf``     -- the level-by-level construction (LRCS, MSCS, recursive MSCS
                  of Sections 2.2-2.4) and the factor-by-factor apply
                  (eq. finishIDBF) and its adjoint, plus ``densify`` for
                  small N.
* ``bessel``   -- J_0 for Example 2's Schloemilch kernel (Miller's backward
                  recurrence below 25, Hankel's expansion above).
* ``mlp``      -- not in the paper: the rank-proposal network (forward,
                  backpropagation, Adam), the randomized residual acceptance
                  test and the SplitMix64 counter generator of the check rows.

Readings of the paper where it is silent, ambiguous or garbled are listed in
the module docstrings where they apply.

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, LAPACK, SVD bounds, brute force or exactness identities.  The
Mock-Chebyshev rule (``sampling.mock_chebyshev``), which the paper cites
without stating, is pinned by the published definition's closed form on
equispaced grids (rounded Chebyshev-Lobatto points, from 60-digit cosines),
the stability of interpolation on its subsets, exact affine invariance and
hand-worked collision cases.
"""
from .kernel import (PHASE_DFT, PHASE_FIO, PHASE_J0, amplitude_shift, phase_mod1, entries,
                     matvec_rows, dense_matvec, dft_closed_form, fio_const_closed_form,
                     relative_error)
from .interp import PIVOT_TIE_REL, column_id, ColumnID
from .sampling import chebyshev_fraction, mock_chebyshev
from .idbf import Factors, build, apply, apply_adjoint, densify, tree_sizes, factor_matrices, sample_count
from . import bessel, mlp

__all__ = [
    "PHASE_DFT", "PHASE_FIO", "PHASE_J0", "amplitude_shift", "phase_mod1", "entries",
    "matvec_rows", "dense_matvec", "dft_closed_form", "fio_const_closed_form",
    "relative_error", "PIVOT_TIE_REL", "column_id", "ColumnID",
    "chebyshev_fraction", "mock_chebyshev", "Factors", "build", "apply",
    "apply_adjoint", "densify", "tree_sizes", "factor_matrices", "sample_count", "bessel", "mlp",
]
