"""Exact O(N^2) sums -- TEST INFRASTRUCTURE ONLY.

The quantity the fast method approximates (eq. (1) of Section 2.2 with
sources equal to targets): for every point i,

    u_i = sum_{j : x_j != x_i} K(x_i - x_j) q_j,    E_i = -grad u at x_i,

with K(r) = c/|r|.  The Laplace/Coulomb constant c = 1/(4 pi) makes q_i E_i
the pair force of eq. (3); the gravity constant c = -1 (G = 1) makes m_i E_i
the attractive force of eq. (4).  The potential energy is U = 1/2 sum q_i u_i.
"""
from __future__ import annotations

import math

import numpy as np

from . import pairsum

KERNELS = {"laplace": 1.0 / (4.0 * math.pi), "gravity": -1.0}


def kernel_constant(kernel: str) -> float:
    return KERNELS[kernel]


def potential_field(x, q, kernel="laplace", targets=None, hess=False):
    """u, E (and the Hessian of u, 6 components xx,yy,zz,xy,xz,yz) by direct sum.

    ``targets`` optionally restricts the outputs to those point indices.
    """
    x = np.asarray(x, dtype=np.float64)
    xt = x if targets is None else x[np.asarray(targets)]
    return pairsum.direct(xt, x, q, None, KERNELS[kernel], hess)


def dipole_potential_field(x, q, m, kernel="laplace", grad=False):
    """u, E of monopoles q (or none) and dipoles m by direct sum; with ``grad``
    also dE_a/dx_b = -Hess u (xx, yy, zz, xy, xz, yz)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros(x.shape[0]) if q is None else q
    u, E, H = pairsum.direct(x, x, s, np.asarray(m, dtype=np.float64).reshape(-1, 3), KERNELS[kernel], grad)
    return (u, E, -H) if grad else (u, E)


def energy(x, q, kernel="laplace"):
    u, _, _ = potential_field(x, q, kernel)
    return 0.5 * float(np.dot(q, u))


def vjp(x, q, ubar, Ebar, kernel="laplace"):
    """Exact gradient of L = sum_i (ubar_i u_i + Ebar_i . E_i) w.r.t. q and x.

    Written out from the pair sums: with r = x_i - x_j,
      dL/dq_j = sum_i ubar_i K(r) + Ebar_i . G(r)        (r = x_i - x_j)
      dL/dx_k = -ubar_k E_k - H_k Ebar_k + q_k grad psi(x_k),
    where psi(x) = sum_j ubar_j K(x - x_j) - Ebar_j . G(x - x_j) and H_k is the
    Hessian of u at x_k.  (The second form follows from the first by the
    symmetry K(x_i - x_j) = K(x_j - x_i).)
    """
    c = KERNELS[kernel]
    x = np.asarray(x, dtype=np.float64)
    _, E, H = pairsum.direct(x, x, q, None, c, True)
    psi, Epsi, _ = pairsum.direct(x, x, ubar, Ebar, c, False)
    HE = hess_times(H, Ebar)
    qbar = psi
    xbar = -ubar[:, None] * E - HE - q[:, None] * Epsi
    return qbar, xbar


def hess_times(H, v):
    """Symmetric 3x3 matrices given as (xx,yy,zz,xy,xz,yz) times vectors v."""
    out = np.empty_like(v)
    out[:, 0] = H[:, 0] * v[:, 0] + H[:, 3] * v[:, 1] + H[:, 4] * v[:, 2]
    out[:, 1] = H[:, 3] * v[:, 0] + H[:, 1] * v[:, 1] + H[:, 5] * v[:, 2]
    out[:, 2] = H[:, 4] * v[:, 0] + H[:, 5] * v[:, 1] + H[:, 2] * v[:, 2]
    return out


def brute_force_python(x, q, kernel="laplace"):
    """Pure-Python double loop, independent of the C helper (tiny inputs only)."""
    c = KERNELS[kernel]
    n = len(q)
    u = [0.0] * n
    E = [[0.0, 0.0, 0.0] for _ in range(n)]
    for i in range(n):
        for j in range(n):
            r = [x[i][k] - x[j][k] for k in range(3)]
            d = math.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
            if d == 0.0:
                continue
            u[i] += c * q[j] / d
            for k in range(3):
                E[i][k] += c * q[j] * r[k] / d ** 3
    return np.array(u), np.array(E)
