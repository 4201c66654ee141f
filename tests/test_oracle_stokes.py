"""Pins of the Stokeslet oracle (CPU only): the direct sum against closed
forms of Stokes flow, the divergence-free velocity, the pressure through the
Stokes equations, the velocity gradient as the velocity's derivative, the
kernel's symmetry, and the harmonic decomposition that the fast evaluation
uses."""
import math

import numpy as np

import workloads
from oracle import direct, kifmm, stokes
from oracle.closed_forms import fibonacci_sphere


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_single_force_is_the_stokeslet():
    f = np.array([[0.3, -1.2, 0.7], [0.0, 0.0, 0.0]])
    x = np.array([[0.1, 0.2, 0.3], [0.6, -0.1, 0.5]])
    u = stokes.direct(x, f, mu=2.0)
    r = x[1] - x[0]
    d = np.linalg.norm(r)
    ref = (f[0] / d + np.dot(r, f[0]) * r / d ** 3) / (8 * math.pi * 2.0)
    np.testing.assert_allclose(u[1], ref, rtol=1e-14)
    assert np.all(u[0] == 0.0)   # no force at point 1, no self term at point 0


def test_sphere_with_uniform_traction():
    """A sphere of radius a carrying the uniform traction 3 mu U / (2a) (the
    surface force of a sphere translating with velocity U in Stokes flow)
    moves its interior rigidly with U and makes outside the flow
    (3a/4)(U/r + (U.r) r/r^3) + (a^3/4)(U/r^3 - 3 (U.r) r/r^5); here as point
    forces on a 4,000-point Fibonacci sphere."""
    mu, a, N = 1.3, 0.2, 4000
    c = np.array([0.5, 0.5, 0.5])
    U = np.array([0.3, -0.2, 0.5])
    y = fibonacci_sphere(N, a, c)
    f = np.tile(6 * math.pi * mu * a * U / N, (N, 1))
    dirs = np.array([[1.0, 0, 0], [0.3, 0.4, 0.866], [0, -1.0, 0]])
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    inside = c + np.array([[0.0, 0, 0], [0.05, 0.02, -0.03], [0.0, 0.09, 0.0]])
    outside = c + dirs * np.array([[2 * a], [3 * a], [1.5 * a]])
    X = np.concatenate([y, inside, outside])
    F = np.concatenate([f, np.zeros((6, 3))])
    u = stokes.direct(X, F, mu, targets=np.arange(N, N + 6))

    def flow(p):
        r = p - c
        d = np.linalg.norm(r)
        return 0.75 * a * (U / d + np.dot(U, r) * r / d ** 3) + 0.25 * a ** 3 * (U / d ** 3 - 3 * np.dot(U, r) * r / d ** 5)

    ref = np.concatenate([np.tile(U, (3, 1)), np.array([flow(p) for p in outside])])
    assert np.abs(u - ref).max() <= 1e-5 * np.linalg.norm(U)


def test_velocity_is_divergence_free():
    rng = np.random.default_rng(4)
    x = rng.random((200, 3))
    f = rng.standard_normal((200, 3))
    probes = rng.random((5, 3)) * 0.2 + 1.2          # away from every source
    h = 1e-4
    div = []
    scale = []
    for p in probes:
        d = 0.0
        g = 0.0
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            X = np.concatenate([x, [p + e], [p - e]])
            F = np.concatenate([f, np.zeros((2, 3))])
            up, um = stokes.direct(X, F, targets=[200, 201])
            d += (up[k] - um[k]) / (2 * h)
            g = max(g, np.abs(up - um).max() / (2 * h))
        div.append(d)
        scale.append(g)
    assert np.max(np.abs(div)) <= 1e-7 * np.max(scale)


def _richardson(fun, p, h):
    """Central-difference gradient and Laplacian of ``fun`` (values [m] at a
    point) at p, Richardson-extrapolated from steps 2h and h."""
    def diffs(hh):
        f0 = fun(p)
        g, lap = [], 0.0
        for k in range(3):
            e = np.zeros(3)
            e[k] = hh
            fp, fm = fun(p + e), fun(p - e)
            g.append((fp - fm) / (2 * hh))
            lap = lap + (fp - 2 * f0 + fm) / hh ** 2
        return np.array(g), lap
    g2, l2 = diffs(2 * h)
    g1, l1 = diffs(h)
    return (4 * g1 - g2) / 3, (4 * l1 - l2) / 3


def test_pressure_satisfies_the_stokes_equations():
    """Away from the forces the direct velocity and pressure satisfy
    mu lap u = grad p, and p is harmonic (finite differences of the direct
    sums, Richardson-extrapolated); a wrong factor or sign in either sum
    leaves a residual of the size of grad p."""
    rng = np.random.default_rng(14)
    x = rng.random((150, 3))
    f = rng.standard_normal((150, 3))
    mu, h = 0.7, 2e-3
    X = np.concatenate([x, np.zeros((1, 3))])
    F = np.concatenate([f, np.zeros((1, 3))])

    def at(p, which):
        X[-1] = p
        if which == "u":
            return stokes.direct(X, F, mu, targets=[150])[0]
        return stokes.pressure_direct(X, F, targets=[150])

    for p in rng.random((4, 3)) * 0.3 + 1.25:          # at least 0.25 from every force
        _, lap_u = _richardson(lambda q: at(q, "u"), p, h)
        grad_p, lap_p = _richardson(lambda q: at(q, "p"), p, h)
        grad_p = grad_p[:, 0]
        scale = np.linalg.norm(grad_p)
        assert np.linalg.norm(mu * lap_u - grad_p) <= 1e-6 * scale
        assert abs(lap_p[0]) <= 1e-6 * scale / 0.25


def test_velocity_gradient_is_the_derivative_of_the_velocity():
    """The direct velocity gradient equals Richardson differences of the
    direct velocity, and its trace (the divergence) vanishes."""
    rng = np.random.default_rng(15)
    x = rng.random((120, 3))
    f = rng.standard_normal((120, 3))
    mu = 0.7
    X = np.concatenate([x, np.zeros((1, 3))])
    F = np.concatenate([f, np.zeros((1, 3))])

    def vel(q):
        X[-1] = q
        return stokes.direct(X, F, mu, targets=[120])[0]

    for p in rng.random((3, 3)) * 0.3 + 1.25:
        fd, _ = _richardson(vel, p, 2e-3)
        X[-1] = p
        g = stokes.gradient_direct(X, F, mu, targets=[120])[0]
        assert np.abs(fd.T - g).max() <= 1e-8 * np.abs(g).max()
        assert abs(np.trace(g)) <= 1e-12 * np.abs(g).max()


def test_kifmm_velocity_gradient_converges_to_the_direct_sum():
    """The oracle KIFMM's velocity gradient (fields and field gradients of
    the four harmonic charges) converges to the direct one with p."""
    w = workloads.make(2, n=3000)
    f = workloads.round_f32(np.random.default_rng(16).standard_normal((w.n, 3)))
    idx = np.arange(0, w.n, 23)
    gd = stokes.gradient_direct(w.positions, f, 0.7, targets=idx)
    err = []
    for p in (4, 6, 8):
        P = kifmm.plan(w.positions, "laplace", p, 64, True, 21, w.root)
        err.append(rel(stokes.kifmm(P, f, 0.7, targets=idx, grad=True)[1], gd))
    assert err[0] > 10 * err[1] > 5 * err[2]
    assert err[1] < 5e-5 and err[2] < 5e-6


def test_symmetry_of_the_kernel():
    rng = np.random.default_rng(5)
    x = rng.random((400, 3))
    f = rng.standard_normal((400, 3))
    g = rng.standard_normal((400, 3))
    a = float(np.sum(g * stokes.direct(x, f)))
    b = float(np.sum(f * stokes.direct(x, g)))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_far_field_of_a_compact_cluster():
    rng = np.random.default_rng(6)
    c = np.array([0.1, 0.2, 0.3])
    s = 0.01
    y = c + s * (rng.random((50, 3)) - 0.5)
    f = rng.standard_normal((50, 3))
    p = c + np.array([0.8, -0.3, 0.5])
    u = stokes.direct(np.concatenate([y, [p]]), np.concatenate([f, [[0, 0, 0]]]), targets=[50])[0]
    F = f.sum(axis=0)
    r = p - c
    d = np.linalg.norm(r)
    ref = (F / d + np.dot(r, F) * r / d ** 3) / (8 * math.pi)
    # the first neglected (moment) term is of relative size s / d times the
    # ratio of the force magnitudes to their sum
    assert np.linalg.norm(u - ref) <= 3 * (s / d) * np.abs(f).sum(axis=0).max() / (8 * math.pi * d)


def test_harmonic_decomposition_with_direct_laplace_sums():
    rng = np.random.default_rng(7)
    x = rng.random((300, 3))
    f = rng.standard_normal((300, 3))
    o = np.array([0.5, 0.5, 0.5])
    xp = x - o
    res = [direct.potential_field(x, q) for q in (f[:, 0], f[:, 1], f[:, 2], np.einsum("ij,ij->i", xp, f))]
    u = np.stack([res[k][0] for k in range(3)], axis=1) + sum(xp[:, k:k + 1] * res[k][1] for k in range(3))
    u = (u - res[3][1]) / (8 * math.pi / (4 * math.pi))
    assert rel(u, stokes.direct(x, f)) <= 1e-13
    # the pressure is the trace of the first three charges' fields
    pr = sum(res[k][1][:, k] for k in range(3))
    assert rel(pr, stokes.pressure_direct(x, f)) <= 1e-13


def test_kifmm_stokes_converges_to_the_direct_sum():
    w = workloads.make(2, n=6000)
    f = workloads.round_f32(np.random.default_rng(8).standard_normal((w.n, 3)))
    ud = stokes.direct(w.positions, f)
    pd = stokes.pressure_direct(w.positions, f)
    err, perr = [], []
    for p in (4, 6, 8):
        P = kifmm.plan(w.positions, "laplace", p, 64, True, 21, w.root)
        u, pr = stokes.kifmm(P, f, pressure=True)
        err.append(rel(u, ud))
        perr.append(rel(pr, pd))
    assert err[0] > 10 * err[1] > 10 * err[2]
    assert err[1] < 5e-5 and err[2] < 5e-6
    # the pressure (fields only: 9.7e-5, 1.8e-6, 1.6e-7 at p = 4, 6, 8)
    assert perr[0] > 10 * perr[1] > 5 * perr[2]
    assert perr[1] < 1e-5 and perr[2] < 1e-6


def test_kifmm_stokes_terms_bound_the_far_velocity():
    """With terms, the same velocity, and magnitudes that bound its far part
    (the velocity minus the Stokeslet summed directly over the near lists)
    term by term, about the root's centre and about each target's leaf
    centre."""
    w = workloads.make(2, n=4000)
    f = workloads.round_f32(np.random.default_rng(9).standard_normal((w.n, 3)))
    P = kifmm.plan(w.positions, "laplace", 4, 32, True, 21, w.root)
    idx = np.random.default_rng(10).choice(w.n, 30, replace=False)
    u = stokes.kifmm(P, f, 0.7, targets=idx)
    u2, mag = stokes.kifmm(P, f, 0.7, targets=idx, terms=True)
    u3, mag_leaf = stokes.kifmm(P, f, 0.7, targets=idx, terms=True, frame="leaf")
    assert np.array_equal(u, u2) and np.array_equal(u, u3)
    c = stokes.leaf_centres(P, idx)
    t = P.tree
    inv = np.empty_like(t.perm)
    inv[t.perm] = np.arange(P.n)
    leaves = t.leaves()
    near = kifmm.near_lists(P)
    for k, i in enumerate(idx):
        si = inv[i]
        leaf = next(int(b) for b in leaves if t.begin[b] <= si < t.end[b])
        src = np.concatenate([np.arange(t.begin[a], t.end[a]) for a in (kifmm.decode(e)[0] for e in near[leaf])])
        # caller indices of the near sources (the direct sum skips the target itself)
        un = stokes.direct(np.concatenate([w.positions[t.perm[src]], w.positions[i:i + 1]]),
                           np.concatenate([f[t.perm[src]], np.zeros((1, 3))]), 0.7, targets=[len(src)])[0]
        far = u[k] - un
        assert np.all(np.abs(far) <= mag[k] * (1 + 1e-9) + 1e-12 * np.abs(u[k]).max())
        assert np.all(np.abs(far) <= mag_leaf[k] * (1 + 1e-9) + 1e-12 * np.abs(u[k]).max())
        assert np.abs(far).max() > 1e-3 * np.abs(u[k]).max()
        # the leaf frame's origin is the centre of the target's own leaf
        wl = P.tree.width(int(P.tree.level[leaf]))
        np.testing.assert_allclose(c[k], P.tree.center(leaf), rtol=0, atol=1e-15)
        assert np.all(np.abs(w.positions[i] - c[k]) <= 0.5 * wl * (1 + 1e-12))


def test_harmonic_decomposition_is_frame_independent():
    """The identity the per-box frames rest on, with direct Laplace sums: the
    fourth potential about any centre c equals that about o plus (o - c)
    times the three force potentials (and so for the fields), and the
    velocity combined about a per-target centre c (x' = x - c, the fourth
    charge (y - c).f) is the direct Stokeslet sum."""
    rng = np.random.default_rng(14)
    x = rng.random((250, 3))
    f = rng.standard_normal((250, 3))
    o = np.array([0.5, 0.5, 0.5])
    c = np.array([0.13, 0.71, 0.42])
    pot = [direct.potential_field(x, f[:, k]) for k in range(3)]
    p4o = direct.potential_field(x, np.einsum("ij,ij->i", x - o, f))
    p4c = direct.potential_field(x, np.einsum("ij,ij->i", x - c, f))
    shifted_u = p4o[0] + sum((o - c)[k] * pot[k][0] for k in range(3))
    shifted_E = p4o[1] + sum((o - c)[k] * pot[k][1] for k in range(3))
    assert rel(shifted_u, p4c[0]) <= 1e-12 and rel(shifted_E, p4c[1]) <= 1e-12
    # every target about its own centre (a different c per target)
    cs = x + 0.05 * rng.standard_normal(x.shape)
    u = np.zeros((250, 3))
    for i in range(250):
        q4 = np.einsum("ij,ij->i", x - cs[i], f)   # the fourth charge about this target's centre
        keep = np.arange(250) != i
        r = x[i] - x[keep]
        d = np.linalg.norm(r, axis=1)
        e4 = (q4[keep][:, None] * r / d[:, None] ** 3).sum(0) / (4 * math.pi)   # its field at x_i
        u[i] = np.array([pot[a][0][i] for a in range(3)]) - e4
        for k in range(3):
            u[i] += (x[i] - cs[i])[k] * pot[k][1][i]
    u /= 8 * math.pi / (4 * math.pi)
    assert rel(u, stokes.direct(x, f)) <= 1e-12
