"""The oracle's discrete adjoint of the force-matching loss against finite
differences at 65,536 points (the adjoint workload's generator at the reduced
size its specification allows when the oracle is slow at full size).

The differences are stored in ``golden/fd_adjoint_65536.txt``, written by
``golden/make_fd_adjoint.py`` from the oracle alone (central differences at
two steps combined by Richardson extrapolation, tree frozen).  The loss is a
quartic polynomial in one charge, so there the combination is exact up to
rounding; in a position it leaves an O(h^4) term.
"""
import os

import numpy as np
import pytest

import workloads
from oracle import kifmm

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "fd_adjoint_65536.txt")
N, P_ORDER, LEAF, M2L_RTOL = 65536, 6, 128, 1e-6


def load_fd():
    xs, qs = [], []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        kind, k, a, r = line.split()[:4]
        (xs if kind == "x" else qs).append((int(k), int(a), float(r)))
    return xs, qs


def loss_gradient_oracle(points):
    """dL/dq and dL/dx of L = sum |q E - Ft|^2 at caller indices ``points``."""
    w = workloads.make(4, n=N)
    qt = workloads.adjoint_target_charges(w.charges, seed=4401)
    P = kifmm.plan(w.positions, w.kernel, P_ORDER, LEAF, True, 21, w.root, m2l_rtol=M2L_RTOL)
    _, Et = kifmm.forward(P, qt)
    _, E = kifmm.forward(P, w.charges)
    R = w.charges[:, None] * E - qt[:, None] * Et
    qb, xb = kifmm.vjp(P, w.charges, np.zeros(N), 2.0 * w.charges[:, None] * R, targets=points)
    qb = qb + 2.0 * np.sum(R[points] * E[points], axis=1)
    return qb, xb


def test_golden_file_shape():
    xs, qs = load_fd()
    assert len(xs) == 64 and len(qs) == 64
    assert all(0 <= k < N and 0 <= a < 3 for k, a, _ in xs)


@pytest.mark.slow
def test_oracle_adjoint_matches_finite_differences():
    xs, qs = load_fd()
    pts = np.unique([k for k, _, _ in xs] + [k for k, _, _ in qs])
    qb, xb = loss_gradient_oracle(pts)
    at = {int(k): i for i, k in enumerate(pts)}
    gx = np.array([xb[at[k], a] for k, a, _ in xs])
    fx = np.array([r for _, _, r in xs])
    gq = np.array([qb[at[k]] for k, _, _ in qs])
    fq = np.array([r for _, _, r in qs])
    ex = np.linalg.norm(gx - fx) / np.linalg.norm(fx)
    eq = np.linalg.norm(gq - fq) / np.linalg.norm(fq)
    print(f"rel-L2 against finite differences: dL/dx {ex:.2e}, dL/dq {eq:.2e}")
    # measured 7e-8 (x: the O(h^4) remainder) and 4e-9 (q: the rounding of the
    # loss differences, each a sum over all 65,536 points)
    assert ex < 1e-6 and eq < 1e-8
