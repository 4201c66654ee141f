"""Pins for the oracle's operators and FMM sweep (CPU only).

KIFMM is an approximation, so it is pinned by what must hold exactly (a
single leaf is the direct sum; the discrete operator is symmetric, linear and
scale-covariant; pseudoinverses are projectors; transposition identities of
the surfaces) and by its approach to the exact direct sum as p grows.
"""
import numpy as np
import pytest

import workloads
from oracle import direct, kifmm
from oracle import operators as O


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_surface_count_matches_p4_56():
    assert O.n_surface(4) == 56 == O.surface_grid(4).shape[0]
    for p in (2, 3, 5, 6, 8):
        g = O.surface_grid(p)
        assert g.shape[0] == O.n_surface(p)
        assert np.all((g.min(axis=1) == 0) | (g.max(axis=1) == 1))


@pytest.mark.parametrize("p", [4, 6])
def test_pseudoinverse_is_projector_and_transposes(p):
    ops = O.Operators(p, direct.KERNELS["laplace"], 1.0)
    for l in (2, 3):
        w = ops.w(l)
        A = O.kernel_matrix(O.surface(p, O.RHO_UC, 0, w), O.surface(p, O.RHO_UE, 0, w), ops.c)
        P = ops.uc2e(l) @ A
        np.testing.assert_allclose(P @ P, P, atol=1e-6)
        # DC2E is built independently from K(dc, de); the surfaces make it UC2E^T
        np.testing.assert_allclose(ops.dc2e(l), ops.uc2e(l).T, rtol=0,
                                   atol=1e-6 * np.abs(ops.uc2e(l)).max())
        # scale covariance: K at side w/2 is 2 K at side w, so the inverse halves
        np.testing.assert_allclose(ops.uc2e(l + 1), ops.uc2e(l) / 2, rtol=0,
                                   atol=1e-6 * np.abs(ops.uc2e(l)).max())
        for o in range(8):
            np.testing.assert_allclose(ops.l2l(l, o), ops.m2m(l, o).T, rtol=1e-14)
        for d in [(2, 0, 0), (3, -1, 2), (-2, -2, -3)]:
            md = tuple(-v for v in d)
            np.testing.assert_allclose(ops.m2l(l, d), ops.m2l(l, md).T, rtol=1e-14)


def test_equivalent_density_reproduces_far_field():
    # P2M + UC2E of a box's points, evaluated beyond the check surface
    p, c = 6, direct.KERNELS["laplace"]
    ops = O.Operators(p, c, 1.0)
    rng = np.random.default_rng(0)
    w = ops.w(3)
    pts = (rng.random((100, 3)) - 0.5) * w
    q = rng.standard_normal(100)
    psi = O.kernel_matrix(O.surface(p, O.RHO_UC, 0, w), pts, c) @ q
    phi = ops.uc2e(3) @ psi
    far = rng.standard_normal((50, 3))
    far *= (2.5 * w / np.abs(far).max(axis=1))[:, None]
    ref = O.kernel_matrix(far, pts, c) @ q
    approx = O.kernel_matrix(far, O.surface(p, O.RHO_UE, 0, w), c) @ phi
    assert rel(approx, ref) < 1e-5


def test_single_leaf_is_direct_sum():
    w = workloads.make(4, n=100)
    P = kifmm.plan(w.positions, "laplace", 6, 128)
    u, E = kifmm.forward(P, w.charges)
    ud, Ed, _ = direct.potential_field(w.positions, w.charges)
    np.testing.assert_allclose(u, ud, rtol=1e-12)
    np.testing.assert_allclose(E, Ed, rtol=1e-11)


def test_error_decays_with_order():
    w = workloads.make(1, n=2048)
    ud, Ed, _ = direct.potential_field(w.positions, w.charges)
    errs = []
    for p in (2, 3, 4, 5, 6):
        P = kifmm.plan(w.positions, "laplace", p, 32, False, 21, w.root)
        u, E = kifmm.forward(P, w.charges)
        errs.append(rel(E, Ed))
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 2e-5


def test_uniform_4096_accuracy_p4():
    w = workloads.make(1)
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root)
    u, E = kifmm.forward(P, w.charges)
    ud, Ed, _ = direct.potential_field(w.positions, w.charges)
    assert rel(u, ud) < 3e-4 and rel(E, Ed) < 5e-4


def test_adaptive_accuracy_and_reciprocity():
    w = workloads.make(2, n=6000)
    P = kifmm.plan(w.positions, "laplace", 6, 32, True, 21, w.root)
    assert sum(len(x) for x in P.lists.X) > 0
    u, E = kifmm.forward(P, w.charges)
    ud, Ed, _ = direct.potential_field(w.positions, w.charges)
    assert rel(u, ud) < 2e-5 and rel(E, Ed) < 2e-5
    rng = np.random.default_rng(1)
    q2 = rng.standard_normal(w.n)
    u2, _ = kifmm.forward(P, q2)
    # q1^T A q2 = q2^T A q1: the discrete operator is symmetric
    a, b = np.dot(w.charges, u2), np.dot(q2, u)
    assert abs(a - b) <= 1e-10 * max(abs(a), np.linalg.norm(w.charges) * np.linalg.norm(u2))
    # linearity
    u3, E3 = kifmm.forward(P, 2.0 * w.charges - 3.0 * q2)
    _, E2 = kifmm.forward(P, q2)
    np.testing.assert_allclose(E3, 2 * E - 3 * E2, rtol=0, atol=1e-9 * np.abs(E3).max())


def test_scaling_covariance():
    w = workloads.make(4, n=3000)
    P1 = kifmm.plan(w.positions, "laplace", 4, 32, True, 21, ((0, 0, 0), 1.0))
    P2 = kifmm.plan(2.0 * w.positions, "laplace", 4, 32, True, 21, ((0, 0, 0), 2.0))
    np.testing.assert_array_equal(P1.tree.perm, P2.tree.perm)
    np.testing.assert_array_equal(P1.tree.begin, P2.tree.begin)
    u1, E1 = kifmm.forward(P1, w.charges)
    u2, E2 = kifmm.forward(P2, w.charges)
    np.testing.assert_allclose(u2, u1 / 2, rtol=1e-9)
    np.testing.assert_allclose(E2, E1 / 4, rtol=1e-9, atol=1e-12 * np.abs(E1).max())


def test_gravity_plummer_accuracy():
    w = workloads.make(5, n=5000)
    P = kifmm.plan(w.positions, w.kernel, 6, 64, True, w.max_depth, w.root)
    u, E = kifmm.forward(P, w.charges)
    ud, Ed, _ = direct.potential_field(w.positions, w.charges, "gravity")
    assert rel(u, ud) < 1e-5 and rel(E, Ed) < 2e-5
    # unit masses attract: the potential is negative everywhere
    assert np.all(u < 0)


def test_sampled_targets_match_full_evaluation():
    w = workloads.make(2, n=5000)
    P = kifmm.plan(w.positions, "laplace", 4, 32, True, 21, w.root)
    u, E = kifmm.forward(P, w.charges)
    idx = np.random.default_rng(2).choice(w.n, 97, replace=False)
    us, Es = kifmm.forward(P, w.charges, targets=idx)
    # same arithmetic up to BLAS blocking of differently sized batches
    np.testing.assert_allclose(us, u[idx], rtol=0, atol=1e-11 * np.abs(u).max())
    np.testing.assert_allclose(Es, E[idx], rtol=0, atol=1e-11 * np.abs(E).max())


def test_dipole_sources_accuracy_and_linearity():
    # monopoles plus dipoles on the clustered shape: the KIFMM sweep with dipole
    # parts converges to the direct sum, and the map is linear in (q, m)
    w = workloads.make(2, n=3000)
    rng = np.random.default_rng(41)
    m = rng.standard_normal((w.n, 3)) * 1e-3
    P = kifmm.plan(w.positions, "laplace", 6, 48, True, 21, w.root)
    u, E = kifmm.forward_dipoles(P, w.charges, m)
    ud, Ed = direct.dipole_potential_field(w.positions, w.charges, m)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-5
    assert np.linalg.norm(E - Ed) / np.linalg.norm(Ed) < 1e-4
    u1, E1 = kifmm.forward_dipoles(P, None, m)
    u2, E2 = kifmm.forward(P, w.charges)
    # FP64 rounding carried through the truncated pseudoinverse (amplification
    # up to 1/tau = 1e7) bounds the difference by about 1e-9 of the largest value
    np.testing.assert_allclose(u1 + u2, u, rtol=0, atol=1e-9 * np.abs(u).max())
    np.testing.assert_allclose(E1 + E2, E, rtol=0, atol=1e-9 * np.abs(E).max())
    # a lone dipole field: sampled targets equal the full evaluation
    t = np.array([3, 77, 2999])
    ut, Et = kifmm.forward_dipoles(P, None, m, targets=t)
    np.testing.assert_allclose(ut, u1[t], rtol=0, atol=1e-11 * np.abs(u1).max())
    np.testing.assert_allclose(Et, E1[t], rtol=0, atol=1e-11 * np.abs(E1).max())


def test_field_gradient_accuracy_with_dipoles():
    # dE/dx of monopoles plus dipoles through the sweep (monopole equivalent
    # densities, dipole parts in the near field) against the direct sum
    w = workloads.make(2, n=3000)
    rng = np.random.default_rng(42)
    m = rng.standard_normal((w.n, 3)) * 1e-3
    P = kifmm.plan(w.positions, "laplace", 6, 48, True, 21, w.root)
    u, E, G = kifmm.forward_dipoles(P, w.charges, m, grad=True)
    ud, Ed, Gd = direct.dipole_potential_field(w.positions, w.charges, m, grad=True)
    assert np.linalg.norm(G - Gd) / np.linalg.norm(Gd) < 1e-5
    # p = 8 is closer (the method converges in p)
    P8 = kifmm.plan(w.positions, "laplace", 8, 48, True, 21, w.root)
    _, _, G8 = kifmm.forward_dipoles(P8, w.charges, m, grad=True)
    assert np.linalg.norm(G8 - Gd) < 0.3 * np.linalg.norm(G - Gd)
    # no dipoles: the same call on the charges alone
    u0, E0, G0 = kifmm.forward_dipoles(P, w.charges, None, grad=True)
    uf, Ef = kifmm.forward(P, w.charges)
    np.testing.assert_allclose(u0, uf, rtol=0, atol=1e-12 * np.abs(uf).max())


def test_compressed_m2l_bound_and_symmetry():
    # M2L in the truncated common basis Q: within 2 tau sigma_1(H) of the exact
    # operator in the spectral norm (one-sided truncation error on each side),
    # and M2L_c(-d) = M2L_c(d)^T, which the adjoint needs
    from oracle import operators as O
    tau = 1e-6
    ops = O.Operators(6, 1.0, 1.0, m2l_rtol=tau)
    Q, S = ops.m2l_basis(2)
    assert Q.shape == (152, int(np.sum(S >= tau * S[0])))
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
    for d in [(2, 0, 0), (-3, 1, 2), (3, 3, 3), (0, -2, 1)]:
        M, Mc = ops.m2l_exact(2, d), ops.m2l(2, d)
        assert np.linalg.norm(M - Mc, 2) <= 2 * tau * S[0] * (1 + 1e-9)
        Mm = ops.m2l(2, tuple(-v for v in d))
        np.testing.assert_allclose(Mm, Mc.T, rtol=0, atol=1e-12 * np.abs(Mc).max())
    exact = O.Operators(6, 1.0, 1.0)
    np.testing.assert_array_equal(exact.m2l(2, (2, 1, 0)), exact.m2l_exact(2, (2, 1, 0)))


def test_compressed_m2l_forward_and_adjoint():
    # the compressed sweep stays within about 1e-6 of the exact one on the
    # clustered shape, and its adjoint is still exact (unit steps in q)
    w = workloads.make(2, n=6000)
    P0 = kifmm.plan(w.positions, "laplace", 6, 48, True, 21, w.root)
    P1 = kifmm.plan(w.positions, "laplace", 6, 48, True, 21, w.root, m2l_rtol=1e-6)
    u0, E0 = kifmm.forward(P0, w.charges)
    u1, E1 = kifmm.forward(P1, w.charges)
    assert np.linalg.norm(u1 - u0) / np.linalg.norm(u0) < 2e-6
    assert np.linalg.norm(E1 - E0) / np.linalg.norm(E0) < 2e-6
    rng = np.random.default_rng(45)
    ub = rng.standard_normal(w.n)
    Eb = rng.standard_normal((w.n, 3))
    qb, _ = kifmm.vjp(P1, w.charges, ub, Eb)

    def loss(q):
        u, E = kifmm.forward(P1, q)
        return float(ub @ u + np.sum(Eb * E))

    for k in (3, 2999):
        dq = np.zeros(w.n)
        dq[k] = 1.0
        fd = (loss(w.charges + dq) - loss(w.charges - dq)) / 2.0
        assert abs(fd - qb[k]) <= 1e-8 * max(1.0, abs(qb[k]))


def test_small_leaf_w_x_pairs_are_direct():
    """A W/X pair whose finer box F is a leaf of at most n points is summed point
    to point in both directions (the reading of the oracle's header): with
    charges only in one X-list source A of such a leaf, the potential and field
    at F's points are the direct sum over A's points to rounding, and with
    charges only in F, those at A's points are (the W direction).  An expansion
    would leave an error of order 1e-6 here."""
    from oracle.tree import decode
    w = workloads.make(2, n=3000)
    P = kifmm.plan(w.positions, "laplace", 4, 16, True, 21, w.root)
    t, L = P.tree, P.lists
    n = P.ops.n
    cases = [(f, decode(e)[0]) for f in range(t.nboxes) if L.X[f] and kifmm.direct_xw(P, f)
             for e in L.X[f][:1]]
    assert len(cases) >= 3
    rng = np.random.default_rng(4)
    for f, a in cases[:3]:
        assert t.is_leaf[f] and t.end[f] - t.begin[f] <= n
        for src, dst in ((a, f), (f, a)):
            q = np.zeros(w.n)
            ids = t.perm[t.begin[src]:t.end[src]]
            q[ids] = rng.standard_normal(ids.shape[0])
            u, E = kifmm.forward(P, q)
            ud, Ed, _ = direct.potential_field(w.positions, q)
            tid = t.perm[t.begin[dst]:t.end[dst]]
            assert rel(u[tid], ud[tid]) < 1e-12 and rel(E[tid], Ed[tid]) < 1e-12


def test_far_and_near_parts_add_up():
    """The near part at a target is the direct sum over the points of its
    leaf's near-list boxes (brute force here); far and near add up to the
    whole evaluation."""
    w = workloads.make(2, n=3000)
    P = kifmm.plan(w.positions, "laplace", 4, 32, True, 21, w.root)
    idx = np.random.default_rng(4).choice(w.n, 40, replace=False)
    u, E = kifmm.forward(P, w.charges, targets=idx)
    uf, Ef = kifmm.forward(P, w.charges, targets=idx, part="far")
    un, En = kifmm.forward(P, w.charges, targets=idx, part="near")
    np.testing.assert_allclose(uf + un, u, rtol=0, atol=1e-12 * np.abs(u).max())
    np.testing.assert_allclose(Ef + En, E, rtol=0, atol=1e-12 * np.abs(E).max())
    assert np.abs(uf).max() > 1e-3 * np.abs(u).max()
    t = P.tree
    inv = np.empty_like(t.perm)
    inv[t.perm] = np.arange(P.n)
    qs = np.asarray(w.charges, dtype=np.float64)[t.perm]
    leaves = t.leaves()
    near = kifmm.near_lists(P)
    for k, i in enumerate(idx):
        si = inv[i]
        leaf = next(int(b) for b in leaves if t.begin[b] <= si < t.end[b])
        src = np.concatenate([np.arange(t.begin[a], t.end[a]) for a in (kifmm.decode(e)[0] for e in near[leaf])])
        r = P.x[si] - P.x[src]
        d = np.linalg.norm(r, axis=1)
        keep = d > 0
        assert np.isclose(un[k], P.c * np.sum(qs[src][keep] / d[keep]), rtol=1e-12)
        np.testing.assert_allclose(En[k], P.c * (qs[src][keep, None] * r[keep] / d[keep, None] ** 3).sum(axis=0),
                                   rtol=1e-11, atol=1e-12 * np.abs(En[k]).max())


def test_unknown_part_is_refused():
    w = workloads.make(4, n=100)
    P = kifmm.plan(w.positions, "laplace", 4, 128)
    with pytest.raises(ValueError):
        kifmm.forward(P, w.charges, part="middle")
