"""Pins of the oracle's periodic sums (Section 2.4: periodic boundaries,
neutral cells for the Laplace lattice sum).

The Ewald sum is pinned by the Madelung constants of NaCl and CsCl, the
vanishing field at ion sites of a cubic crystal, independence of the
splitting parameter (which a wrong prefactor, self or background term
breaks) and invariance under a translation wrapped into the cell.  The
periodic fast method is then pinned by the Ewald sum, by its convergence in
p, by exactly-once coverage of the 27 near images by the periodic lists, and
its adjoint by exact differences.
"""
import math
import os

import numpy as np
import pytest

from oracle import kifmm, periodic as per
from oracle import tree as T

HERE = os.path.dirname(__file__)
C = 1.0 / (4.0 * math.pi)     # the Laplace constant of the oracle's "laplace" kernel
CELL = ((0.0, 0.0, 0.0), 1.0)


def madelung():
    out = {}
    for line in open(os.path.join(HERE, "golden", "madelung.txt")):
        if line.strip() and not line.startswith("#"):
            name, val = line.split()
            out[name] = float(val)
    return out


def test_ewald_madelung_nacl():
    # conventional cube of side 1 holding 8 ions on a grid of spacing d = 1/2
    x, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                x.append((0.5 * i, 0.5 * j, 0.5 * k))
                q.append((-1.0) ** (i + j + k))
    x = np.array(x) + 0.13
    q = np.array(q)
    u, E = per.ewald(x, q, 1.0)
    alpha = madelung()["NaCl"]
    np.testing.assert_allclose(u / C, -q * alpha / 0.5, rtol=1e-13)
    assert np.abs(E).max() / C < 1e-12


def test_ewald_madelung_cscl():
    x = np.array([[0.2, 0.3, 0.4], [0.7, 0.8, 0.9]])
    q = np.array([1.0, -1.0])
    u, E = per.ewald(x, q, 1.0)
    alpha = madelung()["CsCl"]
    np.testing.assert_allclose(u / C, -q * alpha / (math.sqrt(3.0) / 2.0), rtol=1e-12)
    assert np.abs(E).max() / C < 1e-12


@pytest.mark.parametrize("neutral", [True, False])
def test_ewald_independent_of_splitting(neutral):
    rng = np.random.default_rng(7)
    x = rng.random((120, 3)) * 2.0
    q = rng.standard_normal(120)
    if neutral:
        q -= q.mean()
    u1, E1 = per.ewald(x, q, 2.0, alpha=1.6)
    u2, E2 = per.ewald(x, q, 2.0, alpha=4.0)
    assert np.abs(u1 - u2).max() <= 1e-12 * np.abs(u1).max()
    assert np.abs(E1 - E2).max() <= 1e-12 * np.abs(E1).max()


def test_ewald_translation_wrapped_into_the_cell():
    rng = np.random.default_rng(8)
    x = rng.random((100, 3))
    q = rng.standard_normal(100)
    q -= q.mean()
    u1, E1 = per.ewald(x, q, 1.0)
    u2, E2 = per.ewald(np.mod(x + np.array([0.37, -0.81, 0.55]), 1.0), q, 1.0)
    assert np.abs(u1 - u2).max() <= 1e-12 * np.abs(u1).max()
    assert np.abs(E1 - E2).max() <= 1e-12 * np.abs(E1).max()


def test_lattice_kernel_even_harmonic_and_splitting_free():
    rng = np.random.default_rng(9)
    r = rng.uniform(-0.9, 0.9, (40, 3))
    F = per.lattice_far(r, 1.0)
    np.testing.assert_allclose(per.lattice_far(-r, 1.0), F, rtol=0, atol=1e-13)
    np.testing.assert_allclose(per.lattice_far(r, 1.0, alpha=3.5), F, rtol=0, atol=1e-13)
    # seven-point Laplacian vanishes (the removed |r|^2 term carries the background)
    h = 1e-2
    lap = -6.0 * F
    for a in range(3):
        for sgn in (1.0, -1.0):
            e = np.zeros(3)
            e[a] = sgn * h
            lap = lap + per.lattice_far(r + e, 1.0)
    assert np.abs(lap / h ** 2).max() < 1e-6 * np.abs(F).max() / h ** 2 + 1e-7


def _coverage_periodic(t, L):
    """Count, for every target leaf, source leaf and near image s of the
    cell, the interaction paths that reach it."""
    leaves = [int(b) for b in t.leaves()]
    pos = {b: i for i, b in enumerate(leaves)}
    nl = len(leaves)
    cnt = np.zeros((nl, nl, 27), dtype=int)
    memo = {}

    def dl(a):
        if a not in memo:
            memo[a] = [a] if t.is_leaf[a] else [l for c in t.children[a] if c >= 0 for l in dl(int(c))]
        return memo[a]

    def code(s):
        return int(9 * (s[0] + 1) + 3 * (s[1] + 1) + s[2] + 1)

    for B in leaves:
        i = pos[B]
        anc = []
        a = B
        while a >= 0:
            anc.append(a)
            a = int(t.parent[a])
        for e in L.U[B]:
            A, s = T.decode(e)
            cnt[i, pos[A], code(s)] += 1
        for e in L.W[B]:
            A, s = T.decode(e)
            for l in dl(A):
                cnt[i, pos[l], code(s)] += 1
        for a in anc:
            for e in L.V[a]:
                A, s = T.decode(e)
                for l in dl(A):
                    cnt[i, pos[l], code(s)] += 1
            for e in L.X[a]:
                A, s = T.decode(e)
                cnt[i, pos[A], code(s)] += 1
    return cnt


@pytest.mark.parametrize("adaptive,leaf", [(True, 8), (False, 16)])
def test_periodic_lists_cover_the_near_images_exactly_once(adaptive, leaf):
    # every (target leaf, source leaf, image within one cell) is reached
    # exactly once; images further away belong to the root's lattice term
    rng = np.random.default_rng(10)
    x = np.concatenate([rng.random((300, 3)), 0.02 * rng.standard_normal((200, 3)) % 1.0])
    t = T.build_tree(x, leaf, adaptive, 21, CELL)
    L = T.build_lists(t, periodic=True)
    assert sum(len(L.X[b]) for b in range(t.nboxes)) > 0 or not adaptive
    cnt = _coverage_periodic(t, L)
    assert np.all(cnt == 1)
    # free-space entries are plain indices; periodic ones decode to valid boxes
    for rows in (L.U, L.V, L.W, L.X):
        for r in rows:
            for e in r:
                b, s = T.decode(e)
                assert 0 <= b < t.nboxes and np.all(np.abs(s) <= 1)
                assert T.encode(b, s) == e


def test_periodic_single_leaf_lists():
    # a root that is a leaf: U(root) is the 27 images of the root itself
    x = np.random.default_rng(11).random((20, 3))
    t = T.build_tree(x, 64, True, 21, CELL)
    L = T.build_lists(t, periodic=True)
    assert t.nboxes == 1
    assert sorted(L.U[0]) == sorted(T.encode(0, s) for s in np.ndindex(3, 3, 3) for s in [np.array(s) - 1])


@pytest.fixture(scope="module")
def neutral_cell():
    rng = np.random.default_rng(12)
    n = 700
    # two dense clusters and a uniform background, net charge zero, a net dipole
    x = np.concatenate([rng.random((300, 3)),
                        (np.array([0.2, 0.3, 0.8]) + 0.05 * rng.standard_normal((200, 3))) % 1.0,
                        (np.array([0.9, 0.6, 0.1]) + 0.05 * rng.standard_normal((200, 3))) % 1.0])
    q = rng.standard_normal(n)
    q[300:500] += 0.5
    q[500:] -= 0.5
    q -= q.mean()
    ue, Ee = per.ewald(x, q, 1.0)
    return x, q, ue, Ee


def test_periodic_fmm_matches_ewald(neutral_cell):
    x, q, ue, Ee = neutral_cell
    errs = []
    for p in (4, 6):
        P = kifmm.plan(x, "laplace", p, 16, True, 21, CELL, periodic=True)
        u, E = kifmm.forward(P, q)
        errs.append((np.linalg.norm(u - ue) / np.linalg.norm(ue), np.linalg.norm(E - Ee) / np.linalg.norm(Ee)))
    assert errs[1][0] < 3e-5 and errs[1][1] < 3e-5
    assert errs[1][0] < 0.2 * errs[0][0] and errs[1][1] < 0.2 * errs[0][1]


def test_periodic_fmm_non_neutral_cell_matches_background_convention():
    rng = np.random.default_rng(13)
    x = rng.random((400, 3))
    q = rng.random(400)       # all positive: the Ewald sum with a uniform background
    ue, Ee = per.ewald(x, q, 1.0)
    # the field of a one-signed set is a difference of large opposing parts, so
    # its relative error at p = 6 is a few 1e-5; p = 8 brings it to a few 1e-6
    P = kifmm.plan(x, "laplace", 8, 16, True, 21, CELL, periodic=True)
    u, E = kifmm.forward(P, q)
    assert np.linalg.norm(E - Ee) / np.linalg.norm(Ee) < 1e-5
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 1e-5


def test_periodic_adjoint_exact_differences():
    # L = ubar.u + Ebar.E is linear in q: central differences are exact up to rounding;
    # in x the tree is frozen and Richardson differences remove the O(h^2) term
    rng = np.random.default_rng(14)
    n = 300
    x = rng.random((n, 3)) * 0.98 + 0.01
    q = rng.standard_normal(n)
    q -= q.mean()
    P = kifmm.plan(x, "laplace", 4, 16, True, 21, CELL, periodic=True)
    ub = rng.standard_normal(n)
    Eb = rng.standard_normal((n, 3))

    def loss(PP, qq):
        u, E = kifmm.forward(PP, qq)
        return float(ub @ u + np.sum(Eb * E))

    qb, xb = kifmm.vjp(P, q, ub, Eb)
    for k in (0, 77, 211):
        # a unit step: the loss is linear in q, and a large step keeps rounding small
        dq = np.zeros(n)
        dq[k] = 1.0
        fd = (loss(P, q + dq) - loss(P, q - dq)) / 2.0
        assert abs(fd - qb[k]) <= 1e-9 * max(1.0, abs(qb[k]))
    # the periodic operator is symmetric (reciprocity)
    q1, q2 = rng.standard_normal(n), rng.standard_normal(n)
    u1, _ = kifmm.forward(P, q1)
    u2, _ = kifmm.forward(P, q2)
    assert abs(q2 @ u1 - q1 @ u2) <= 1e-9 * abs(q2 @ u1)
    for k, a in ((5, 0), (150, 2)):
        def at(h):
            xx = x.copy()
            xx[k, a] += h
            return loss(P.with_positions(xx), q)
        h = 1e-4
        d1 = (at(h) - at(-h)) / (2 * h)
        d2 = (at(h / 2) - at(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
        assert abs(fd - xb[k, a]) <= 1e-6 * max(1.0, np.abs(xb).max())


def test_periodic_uniform_tree_list_sizes_closed_form():
    # a full uniform tree of depth 2 in a periodic cell: every box below the
    # root sees 8 x 27 - 27 = 189 far children of its parent's 27 neighbour
    # images, every leaf its 27 neighbour images, and there is no W or X
    x = np.random.default_rng(15).random((4096, 3))
    t = T.build_tree(x, 64, False, 21, CELL)
    L = T.build_lists(t, periodic=True)
    assert t.depth == 2 and t.nboxes == 73
    assert all(len(L.V[b]) == (189 if b > 0 else 0) for b in range(t.nboxes))
    assert all(len(L.U[b]) == 27 for b in t.leaves())
    assert sum(len(r) for r in L.W) == 0 and sum(len(r) for r in L.X) == 0
