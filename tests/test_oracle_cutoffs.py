"""Singular-value gaps at the two truncation cut-offs (CPU only).

The check-to-equivalent pseudoinverses drop singular values of K(uc, ue)
below tau sigma_1 (tau = 1e-7), and the compressed M2L keeps the left singular
vectors of [M2L(d_1) ... M2L(d_316)] with sigma >= m2l_rtol sigma_1
(m2l_rtol = 1e-6).  Two correct implementations can keep different ranks only
if a singular value sits next to the cut, so the kept ranks are pinned by
showing that none does: the last kept value is at least 2 % above the cut and
the first dropped one at least 2 % below it (measured margins: 8 % at
p = 7 for tau, 3 % at p = 8 for the M2L basis), far beyond FP64 rounding of
either decomposition.
"""
import numpy as np
import pytest

from oracle.operators import RHO_UC, RHO_UE, TAU, Operators, kernel_matrix, pinv_truncated, surface

GAP = 0.02


def gaps(S, cut):
    r = S / (cut * S[0])
    k = int(np.sum(r >= 1.0))
    last = r[k - 1]
    first = r[k] if k < len(S) else 0.0
    return k, last, first


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_pseudoinverse_cut_has_a_gap(p):
    A = kernel_matrix(surface(p, RHO_UC, 0, 1.0), surface(p, RHO_UE, 0, 1.0), 1.0)
    _, rank, S = pinv_truncated(A, TAU)
    k, last, first = gaps(S, TAU)
    assert k == rank
    assert last >= 1 + GAP and first <= 1 - GAP, (p, last, first)


@pytest.mark.parametrize("p,rank", [(4, 56), (6, 116), (8, 124)])
def test_m2l_basis_cut_has_a_gap(p, rank):
    ops = Operators(p, 1.0, 1.0, TAU, 1e-6)
    Q, S = ops.m2l_basis(0)
    k, last, first = gaps(S, 1e-6)
    assert k == Q.shape[1] == rank
    assert last >= 1 + GAP and first <= 1 - GAP, (p, last, first)
