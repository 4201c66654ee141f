"""Pins for the oracle's exact direct sum (CPU only).

The paper prints no worked numbers, so the direct sum is pinned by the pair
force of eq. (3), the sign of eq. (4), the shell theorem, Newton's third law,
reciprocity and an independent pure-Python double loop.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import direct, pairsum


def test_coulomb_pair_eq3():
    # eq. (3): F_12 = r q1 q2 / (4 pi r^3) with r = x1 - x2 (repulsive for like charges)
    x = np.array([[0.1, 0.2, 0.3], [0.4, -0.1, 0.7]])
    q = np.array([1.5, -0.5])
    u, E, _ = direct.potential_field(x, q, "laplace")
    F1 = q[0] * E[0]
    np.testing.assert_allclose(F1, cf.coulomb_force(q[0], q[1], x[0], x[1]), rtol=1e-14)
    r = np.linalg.norm(x[0] - x[1])
    assert u[0] == pytest.approx(q[1] / (4 * math.pi * r), rel=1e-14)
    # like charges repel: force on 1 points away from 2
    u, E, _ = direct.potential_field(x, np.array([1.0, 1.0]), "laplace")
    assert np.dot(E[0], x[0] - x[1]) > 0


def test_gravity_attracts_eq4():
    # eq. (4) with G = 1: |F| = m1 m2 / r^2, directed from 1 towards 2
    x = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    m = np.array([3.0, 5.0])
    u, E, _ = direct.potential_field(x, m, "gravity")
    F1 = m[0] * E[0]
    np.testing.assert_allclose(F1, [15.0 / 4.0, 0.0, 0.0], rtol=1e-15)
    assert u[0] == pytest.approx(-5.0 / 2.0, rel=1e-15)


def test_shell_theorem():
    Q, R = 2.0, 0.3
    n = 20000
    ys = cf.fibonacci_sphere(n, R)
    qs = np.full(n, Q / n)
    rng = np.random.default_rng(1)
    inside = rng.standard_normal((50, 3))
    inside *= (0.5 * R * rng.random(50) / np.linalg.norm(inside, axis=1))[:, None]
    outside = rng.standard_normal((50, 3))
    outside *= ((2.0 + 3.0 * rng.random(50)) * R / np.linalg.norm(outside, axis=1))[:, None]
    for pts in (inside, outside):
        u, E, _ = pairsum.direct(pts, ys, qs, None, direct.KERNELS["laplace"])
        r = np.linalg.norm(pts, axis=1)
        np.testing.assert_allclose(u, cf.shell_potential(Q, R, r), rtol=2e-4)
        Eref = cf.shell_field(Q, R, pts)
        scale = Q * cf.C_LAPLACE / R ** 2
        assert np.max(np.abs(E - Eref)) < 2e-3 * scale


def test_newton_third_law_and_reciprocity():
    rng = np.random.default_rng(2)
    x = rng.random((500, 3))
    q1 = rng.standard_normal(500)
    q2 = rng.standard_normal(500)
    _, E, _ = direct.potential_field(x, q1, "laplace")
    F = q1[:, None] * E
    assert np.max(np.abs(F.sum(axis=0))) < 1e-12 * np.max(np.abs(F)) * 500
    u2, _, _ = direct.potential_field(x, q2, "laplace")
    u1, _, _ = direct.potential_field(x, q1, "laplace")
    assert np.dot(q1, u2) == pytest.approx(np.dot(q2, u1), rel=1e-12)


def test_c_helper_matches_python_double_loop_with_coincident_points():
    rng = np.random.default_rng(3)
    x = rng.random((30, 3))
    x[7] = x[3]                     # coincident pair is skipped like the self pair
    q = rng.standard_normal(30)
    u, E, _ = direct.potential_field(x, q, "laplace")
    up, Ep = direct.brute_force_python(x.tolist(), q.tolist(), "laplace")
    np.testing.assert_allclose(u, up, rtol=1e-13)
    np.testing.assert_allclose(E, Ep, rtol=1e-12, atol=1e-12 * np.abs(Ep).max())


def test_hessian_traceless_and_matches_field_difference():
    rng = np.random.default_rng(4)
    x = rng.random((200, 3))
    q = rng.standard_normal(200)
    _, E, H = direct.potential_field(x, q, "laplace", hess=True)
    tr = H[:, 0] + H[:, 1] + H[:, 2]
    assert np.max(np.abs(tr)) < 1e-9 * np.max(np.abs(H))
    # H = -dE/dx (central difference of the field of the other points at x_0)
    h = 1e-6
    for a in range(3):
        xp = x[:1].copy(); xp[0, a] += h
        xm = x[:1].copy(); xm[0, a] -= h
        _, Ep, _ = pairsum.direct(xp, x[1:], q[1:], None, direct.KERNELS["laplace"])
        _, Em, _ = pairsum.direct(xm, x[1:], q[1:], None, direct.KERNELS["laplace"])
        col = -(Ep[0] - Em[0]) / (2 * h)
        Hfull = np.array([[H[0, 0], H[0, 3], H[0, 4]], [H[0, 3], H[0, 1], H[0, 5]],
                          [H[0, 4], H[0, 5], H[0, 2]]])
        np.testing.assert_allclose(col, Hfull[:, a], rtol=1e-6, atol=1e-6 * np.abs(Hfull).max())


def test_dipole_source_matches_point_dipole():
    p = np.array([0.3, -0.2, 0.5])
    rng = np.random.default_rng(5)
    xt = rng.standard_normal((40, 3))
    # the helper's dipole source m makes psi = -m.G(r) (a derivative w.r.t. the
    # source position), i.e. the physical dipole p = -m
    u, E, _ = pairsum.direct(xt, np.zeros((1, 3)), np.zeros(1), -p[None, :], cf.C_LAPLACE)
    np.testing.assert_allclose(u, cf.dipole_potential(p, xt), rtol=1e-12)
    np.testing.assert_allclose(E, cf.dipole_field(p, xt), rtol=1e-11, atol=1e-13)


def test_direct_vjp_matches_finite_differences():
    rng = np.random.default_rng(6)
    n = 40
    x = rng.random((n, 3))
    q = rng.standard_normal(n)
    ub = rng.standard_normal(n)
    Eb = rng.standard_normal((n, 3))
    qb, xb = direct.vjp(x, q, ub, Eb, "laplace")

    def L(q_, x_):
        u, E, _ = direct.potential_field(x_, q_, "laplace")
        return np.dot(ub, u) + np.sum(Eb * E)

    for j in (0, 13, 39):
        e = np.zeros(n); e[j] = 1.0
        assert (L(q + e, x) - L(q - e, x)) / 2 == pytest.approx(qb[j], rel=1e-10)
    h = 1e-5
    for k, a in ((3, 0), (17, 2), (31, 1)):
        xp = x.copy(); xp[k, a] += h
        xm = x.copy(); xm[k, a] -= h
        xp2 = x.copy(); xp2[k, a] += h / 2
        xm2 = x.copy(); xm2[k, a] -= h / 2
        d1 = (L(q, xp) - L(q, xm)) / (2 * h)
        d2 = (L(q, xp2) - L(q, xm2)) / h
        rich = (4 * d2 - d1) / 3
        assert rich == pytest.approx(xb[k, a], rel=1e-7)


def test_dipole_field_gradient_matches_differences_and_is_traceless():
    # dE/dx of monopoles plus dipoles: central differences of the field at
    # displaced targets (Richardson), and zero trace (harmonic away from sources)
    from oracle import pairsum
    rng = np.random.default_rng(31)
    ys = rng.random((40, 3))
    s = rng.standard_normal(40)
    m = rng.standard_normal((40, 3))
    xt = rng.random((5, 3)) + 1.5          # targets away from the sources
    c = 1.0 / (4.0 * np.pi)
    _, _, H = pairsum.direct(xt, ys, s, m, c, True)
    G = -H
    comps = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]

    def field(x):
        return pairsum.direct(x, ys, s, m, c, False)[1]

    h = 1e-3
    for k, (a, b) in enumerate(comps):
        e = np.zeros(3)
        e[b] = h
        d1 = (field(xt + e)[:, a] - field(xt - e)[:, a]) / (2 * h)
        d2 = (field(xt + e / 2)[:, a] - field(xt - e / 2)[:, a]) / h
        np.testing.assert_allclose((4 * d2 - d1) / 3, G[:, k], rtol=1e-7, atol=1e-9 * np.abs(G).max())
    np.testing.assert_allclose(G[:, 0] + G[:, 1] + G[:, 2], 0.0, atol=1e-12 * np.abs(G).max())
