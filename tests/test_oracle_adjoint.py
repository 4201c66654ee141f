"""Pins for the oracle's discrete adjoint and clump reduction (CPU only)."""
import numpy as np
import pytest

import workloads
from oracle import closed_forms as cf
from oracle import clump, direct, kifmm


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def small_plan():
    w = workloads.make(4, n=1500)
    P = kifmm.plan(w.positions, "laplace", 4, 16, True, 21, w.root)
    rng = np.random.default_rng(7)
    ub = rng.standard_normal(w.n)
    Eb = rng.standard_normal((w.n, 3))
    qb, xb = kifmm.vjp(P, w.charges, ub, Eb)
    return w, P, ub, Eb, qb, xb


def _loss(P, q, ub, Eb, x=None):
    PP = P if x is None else P.with_positions(x)
    u, E = kifmm.forward(PP, q)
    return u, E


def test_adjoint_in_q_is_exact(small_plan):
    # L = ub.u + Eb.E is linear in q, so a central difference with step 1 is exact
    w, P, ub, Eb, qb, xb = small_plan
    for j in (0, 700, 1499):
        e = np.zeros(w.n); e[j] = 1.0
        up, Ep = _loss(P, w.charges + e, ub, Eb)
        um, Em = _loss(P, w.charges - e, ub, Eb)
        fd = 0.5 * (np.dot(ub, up - um) + np.sum(Eb * (Ep - Em)))
        assert fd == pytest.approx(qb[j], rel=1e-9, abs=1e-9 * np.abs(qb).max())


def test_adjoint_in_x_matches_richardson_fd(small_plan):
    # frozen tree, FP64 central differences at h and h/2 with Richardson extrapolation
    w, P, ub, Eb, qb, xb = small_plan
    h = 2.0 ** -20
    for k, a in ((5, 0), (333, 1), (1200, 2)):
        def d(hh):
            xp = w.positions.copy(); xp[k, a] += hh
            xm = w.positions.copy(); xm[k, a] -= hh
            up, Ep = _loss(P, w.charges, ub, Eb, xp)
            um, Em = _loss(P, w.charges, ub, Eb, xm)
            return (np.dot(ub, up - um) + np.sum(Eb * (Ep - Em))) / (2 * hh)
        rich = (4 * d(h / 2) - d(h)) / 3
        assert rich == pytest.approx(xb[k, a], rel=1e-6, abs=1e-7 * np.abs(xb).max())


def test_adjoint_close_to_direct_sum_gradient(small_plan):
    w, P, ub, Eb, qb, xb = small_plan
    qd, xd = direct.vjp(w.positions, w.charges, ub, Eb)
    assert rel(qb, qd) < 2e-3 and rel(xb, xd) < 2e-3


def test_clump_dipoles_far_apart_match_point_dipoles():
    # two 3-pebble dipole clumps (charges -1, 0, +1 on a line; Section 3.2 geometry,
    # spacing shrunk so that the finite-size correction (l/d)^2 stays below 1e-4)
    l = 0.002
    c1 = np.array([0.3, 0.5, 0.5])
    c2 = np.array([0.7, 0.5, 0.52])
    d1 = np.array([1.0, 0.0, 0.0])
    d2 = np.array([0.0, 0.6, 0.8])
    x = np.concatenate([c1 + np.outer([-1, 0, 1], d1) * l, c2 + np.outer([-1, 0, 1], d2) * l])
    q = np.array([-1.0, 0.0, 1.0, -1.0, 0.0, 1.0])
    u, E, _ = direct.potential_field(x, q)
    F, Tq = clump.clump_reduce(x, q, E, np.array([0, 3, 6]), np.stack([c1, c2]))
    p1, p2 = 2 * l * d1, 2 * l * d2
    E2_at_1 = cf.dipole_field(p2, (c1 - c2)[None, :])[0]
    # torque on dipole 1 in the field of dipole 2 ~ p1 x E
    np.testing.assert_allclose(Tq[0], np.cross(p1, E2_at_1), rtol=2e-3, atol=1e-6 * np.abs(Tq).max())
    # forces are equal and opposite (intra-clump pairs cancel to rounding of the pebble forces)
    fmax = np.abs(q[:, None] * E).max()
    np.testing.assert_allclose(F[0], -F[1], rtol=0, atol=1e-14 * fmax)


def test_clump_in_uniform_field_has_torque_p_cross_E():
    # a dipole clump between two distant large plates of charge sees a nearly uniform field
    l = 0.001
    d = np.array([0.0, 1.0, 0.0])
    cen = np.array([0.0, 0.0, 0.0])
    x_clump = cen + np.outer([-1, 0, 1], d) * l
    q_clump = np.array([-1.0, 0.0, 1.0])
    # uniform field E0 along x from the exact formula applied pebble by pebble
    E0 = np.array([2.0, 0.0, 0.0])
    E = np.tile(E0, (3, 1))
    F, Tq = clump.clump_reduce(x_clump, q_clump, E, np.array([0, 3]), cen[None, :])
    p = 2 * l * d
    np.testing.assert_allclose(F[0], 0.0, atol=1e-15)
    np.testing.assert_allclose(Tq[0], np.cross(p, E0), rtol=1e-14)


def _clump_case(seed=7, C=5, per=(1, 4)):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(per[0], per[1] + 1, C)
    off = np.concatenate([[0], np.cumsum(sizes)])
    N = int(off[-1]) + 3          # three pebbles outside every clump
    x = rng.standard_normal((N, 3))
    q = rng.standard_normal(N)
    E = rng.standard_normal((N, 3))
    cen = rng.standard_normal((C, 3))
    return x, q, E, off, cen


def test_clump_vjp_matches_central_differences():
    # L = Fbar.F + Tbar.T is bilinear in (q, E) and affine in x and X for fixed
    # (q, E): central differences are exact up to rounding.
    x, q, E, off, cen = _clump_case()
    C = len(off) - 1
    rng = np.random.default_rng(8)
    Fb = rng.standard_normal((C, 3))
    Tb = rng.standard_normal((C, 3))

    def L(x_, q_, E_, c_):
        F, T = clump.clump_reduce(x_, q_, E_, off, c_)
        return float(np.sum(Fb * F) + np.sum(Tb * T))

    qb, Eb, xb, Xb = clump.clump_vjp(x, q, E, off, cen, Fb, Tb)
    h = 1e-6
    for k in range(x.shape[0]):
        dq = np.zeros_like(q)
        dq[k] = h
        assert abs((L(x, q + dq, E, cen) - L(x, q - dq, E, cen)) / (2 * h) - qb[k]) < 1e-7
        for d in range(3):
            dE = np.zeros_like(E)
            dE[k, d] = h
            assert abs((L(x, q, E + dE, cen) - L(x, q, E - dE, cen)) / (2 * h) - Eb[k, d]) < 1e-7
            dx = np.zeros_like(x)
            dx[k, d] = h
            assert abs((L(x + dx, q, E, cen) - L(x - dx, q, E, cen)) / (2 * h) - xb[k, d]) < 1e-7
    for c in range(C):
        for d in range(3):
            dc = np.zeros_like(cen)
            dc[c, d] = h
            assert abs((L(x, q, E, cen + dc) - L(x, q, E, cen - dc)) / (2 * h) - Xb[c, d]) < 1e-7
    # pebbles outside every clump receive nothing
    n_in = int(off[-1])
    assert not qb[n_in:].any() and not Eb[n_in:].any() and not xb[n_in:].any()


def test_clump_vjp_single_pebble_closed_form():
    # one pebble at r from the centre in a field E, torque-only loss along z:
    # T_z = q (r_x E_y - r_y E_x), so dL/dx = q (E_y, -E_x, 0) and dL/dq = T_z / q
    x = np.array([[0.3, -0.2, 0.5]])
    cen = np.zeros((1, 3))
    q = np.array([2.0])
    E = np.array([[1.0, 4.0, -3.0]])
    qb, Eb, xb, Xb = clump.clump_vjp(x, q, E, np.array([0, 1]), cen, np.zeros((1, 3)), np.array([[0, 0, 1.0]]))
    np.testing.assert_allclose(xb[0], [2 * 4.0, -2 * 1.0, 0.0])
    np.testing.assert_allclose(qb[0], 0.3 * 4.0 - (-0.2) * 1.0)
    np.testing.assert_allclose(Eb[0], 2.0 * np.array([0.2, 0.3, 0.0]))   # q (z x r)
    np.testing.assert_allclose(Xb[0], -xb[0])
