"""Stokes flow of point forces -- TEST INFRASTRUCTURE ONLY.

The sum of eq. (1) in Section 2.2 with a tensor kernel: the paper names
vector and tensor kernels (and periodic Stokes sums in Section 2.4) among what
the kernel-independent method evaluates.  For point forces f_j at x_j in a
fluid of viscosity mu, the velocity at each point is the Stokeslet sum

    u(x_i) = 1/(8 pi mu) sum_{j : x_j != x_i} [ f_j / r + (r . f_j) r / r^3 ],
    r = x_i - x_j,  r = |r|.

``direct`` is that definition written out (O(N^2), FP64).

``kifmm`` evaluates the same sum with the plan's Laplace KIFMM: the Stokeslet
is a combination of harmonic potentials and their gradients (the harmonic
decomposition of Tornberg and Greengard, J. Comput. Phys. 227 (2008)): with
x' = x - o for a fixed origin o,

    phi_k(x) = sum_j f_{j,k} / r  (k = 1, 2, 3),   phi_4(x) = sum_j (x'_j . f_j) / r,
    sum_j S(r) f_j = phi - x'_k grad phi_k + grad phi_4,

since -x'_k d_a(f_k/r) + d_a((x'_j . f)/r) = (r . f) r_a / r^3 for each pair.
Each phi is one charge evaluation of the plan (charges f_x, f_y, f_z and
x'.f); the origin is the root cube's centre.

The pressure that goes with this velocity (the Stokes equations
mu lap u = grad p, div u = 0 hold away from the forces) is

    p(x_i) = 1/(4 pi) sum_{j : x_j != x_i} (r . f_j) / r^3,

``pressure_direct`` written out; through the same decomposition it is
-(1/4 pi) sum_k d_k phi_k, the trace of the fields of the first three
charges, which ``kifmm`` returns with ``pressure``.

The velocity gradient g_ab = d u_a / d x_b of the Stokeslet sum,

    g_ab = 1/(8 pi mu) sum_j [ (f_b r_a - f_a r_b + (r . f) delta_ab) / r^3
                               - 3 (r . f) r_a r_b / r^5 ],

is ``gradient_direct``; differentiating the decomposition gives
g_ab = (-E(a)_b + E(b)_a + x'_k dE(k)_a/dx_b - dE(4)_a/dx_b) / (8 pi mu c),
the fields and field gradients of the four charges, which ``kifmm`` returns
with ``grad``.
"""
from __future__ import annotations

import math

import numpy as np


def direct(x, f, mu=1.0, targets=None, chunk=512):
    """Velocity [nt, 3] at the points ``targets`` (all by default)."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64).reshape(-1, 3)
    t = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((t.shape[0], 3))
    for a in range(0, t.shape[0], chunk):
        xt = x[t[a:a + chunk]]
        r = xt[:, None, :] - x[None, :, :]
        r2 = np.einsum("ijk,ijk->ij", r, r)
        inv = np.zeros_like(r2)
        nz = r2 > 0
        inv[nz] = 1.0 / np.sqrt(r2[nz])
        rf = np.einsum("ijk,jk->ij", r, f)
        out[a:a + chunk] = np.einsum("ij,jk->ik", inv, f) + np.einsum("ij,ijk->ik", rf * inv ** 3, r)
    return out / (8.0 * math.pi * mu)


def pressure_direct(x, f, targets=None, chunk=512):
    """Pressure [nt] at the points ``targets`` (all by default)."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64).reshape(-1, 3)
    t = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros(t.shape[0])
    for a in range(0, t.shape[0], chunk):
        xt = x[t[a:a + chunk]]
        r = xt[:, None, :] - x[None, :, :]
        r2 = np.einsum("ijk,ijk->ij", r, r)
        inv3 = np.zeros_like(r2)
        nz = r2 > 0
        inv3[nz] = r2[nz] ** -1.5
        out[a:a + chunk] = np.einsum("ij,ij->i", np.einsum("ijk,jk->ij", r, f), inv3)
    return out / (4.0 * math.pi)


def gradient_direct(x, f, mu=1.0, targets=None, chunk=256):
    """Velocity gradient [nt, 3, 3], entry [a, b] = d u_a / d x_b, at the
    points ``targets`` (all by default)."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64).reshape(-1, 3)
    t = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((t.shape[0], 3, 3))
    eye = np.eye(3)
    for a in range(0, t.shape[0], chunk):
        xt = x[t[a:a + chunk]]
        r = xt[:, None, :] - x[None, :, :]
        r2 = np.einsum("ijk,ijk->ij", r, r)
        inv3 = np.zeros_like(r2)
        nz = r2 > 0
        inv3[nz] = r2[nz] ** -1.5
        inv5 = np.zeros_like(r2)
        inv5[nz] = r2[nz] ** -2.5
        rf = np.einsum("ijk,jk->ij", r, f)
        g = (np.einsum("ij,jb,ija->iab", inv3, f, r) - np.einsum("ij,ja,ijb->iab", inv3, f, r)
             + np.einsum("ij,ab->iab", rf * inv3, eye) - 3.0 * np.einsum("ij,ija,ijb->iab", rf * inv5, r, r))
        out[a:a + chunk] = g
    return out / (8.0 * math.pi * mu)


def origin(P):
    """The fixed origin of the decomposition: the root cube's centre."""
    return P.tree.lo + 0.5 * P.tree.s


def leaf_centres(P, targets=None):
    """Centre of the leaf holding each point (caller order, or at caller
    indices ``targets``)."""
    t = P.tree
    leaf_of = np.empty(P.n, dtype=np.int64)
    for b in t.leaves():
        leaf_of[t.begin[b]:t.end[b]] = b
    inv = np.empty_like(t.perm)
    inv[t.perm] = np.arange(P.n)
    idx = inv if targets is None else inv[np.asarray(targets)]
    return np.array([t.center(int(b)) for b in leaf_of[idx]]).reshape(-1, 3)


def kifmm(P, f, mu=1.0, targets=None, terms=False, frame="root", pressure=False, grad=False):
    """The Stokeslet sum through four Laplace evaluations of the oracle plan
    ``P`` (its kernel constant c = P.c): u = (1/(8 pi mu c)) [psi_a +
    x'_k E(k)_a - E(4)_a], psi_k and E(k) = -grad psi_k the plan's potential
    and field of the charges f_k (k = 1, 2, 3) and x'.f (k = 4).

    With ``terms`` also the sum of the magnitudes of the far-field parts of
    those terms (the expansions' share of each evaluation, its whole minus its
    near-list sum), scaled alike: its ratio to |u| bounds how much the
    combination amplifies relative errors of the four far fields (the terms
    grow as |x'| over the distance to the sources, u does not).  ``frame``
    names the origin of those terms: "root" (the one origin used here) or
    "leaf", each target's leaf centre c, for which the fourth field is
    E(4) + (o - c)_k E(k) and x' = x - c (the same velocity).

    With ``pressure`` the pressure p = (1/(4 pi c)) sum_k E(k)_k (k = 1, 2,
    3) is returned after those; with ``grad`` last the velocity gradient
    [.., 3, 3] (entry [a, b] = d u_a / d x_b) from the four charges' fields
    and field gradients (one sweep with the field gradient per charge)."""
    from . import kifmm as K
    f = np.asarray(f, dtype=np.float64).reshape(-1, 3)
    o = origin(P)
    xs = P.x[np.argsort(P.tree.perm)]          # caller order
    xp = xs - o
    charges = [f[:, 0], f[:, 1], f[:, 2], np.einsum("ij,ij->i", xp, f)]
    if grad:
        res = [K.forward_dipoles(P, q, None, targets=targets, grad=True) for q in charges]
    else:
        res = [K.forward(P, q, targets=targets) for q in charges]
    xt = xp if targets is None else xp[np.asarray(targets)]
    u = np.stack([res[a][0] for a in range(3)], axis=1)
    for k in range(3):
        u += xt[:, k:k + 1] * res[k][1]
    u -= res[3][1]
    s = 1.0 / (8.0 * math.pi * mu * P.c)
    extra = ()
    if pressure:
        extra = (sum(res[k][1][:, k] for k in range(3)) / (4.0 * math.pi * P.c),)
    if grad:
        def full(G6):
            # (xx yy zz xy xz yz) -> symmetric [.., 3, 3]
            G = np.empty(G6.shape[:-1] + (3, 3))
            for a, b, c in ((0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 1, 3), (0, 2, 4), (1, 2, 5)):
                G[..., a, b] = G[..., b, a] = G6[..., c]
            return G
        E = [res[k][1] for k in range(4)]
        Gk = [full(res[k][2]) for k in range(4)]
        g = np.zeros(E[0].shape[:-1] + (3, 3))
        for a in range(3):
            for b in range(3):
                g[:, a, b] = -E[a][:, b] + E[b][:, a] - Gk[3][:, a, b]
        for k in range(3):
            g += xt[:, k, None, None] * Gk[k]
        extra = extra + (g * s,)
    if not terms:
        return (u * s,) + extra if extra else u * s
    if frame not in ("root", "leaf"):
        raise ValueError(f"unknown frame {frame!r}")
    near = [K.forward(P, q, targets=targets, part="near") for q in charges]
    far = [(r[0] - n[0], r[1] - n[1]) for r, n in zip(res, near)]
    e4, xf = far[3][1], xt
    if frame == "leaf":
        c = leaf_centres(P, targets)
        e4 = e4 + sum((o[k] - c[:, k:k + 1]) * far[k][1] for k in range(3))
        xf = xt + o - c
    mag = np.abs(np.stack([far[a][0] for a in range(3)], axis=1)) + np.abs(e4)
    for k in range(3):
        mag += np.abs(xf[:, k:k + 1] * far[k][1])
    return (u * s, mag * abs(s)) + extra
