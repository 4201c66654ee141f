"""Per-clump force and torque -- TEST INFRASTRUCTURE ONLY.

Section 2.4: the long-range forces are applied to the pebbles and then the
forces and moments on the pebbles are summed into the force and torque of
each clump.  With F_k = q_k E_k on pebble k and the clump reference point X_c
(its centre of mass, supplied by the caller):

    F_c = sum_{k in c} F_k,     T_c = sum_{k in c} (x_k - X_c) x F_k,

accumulated in FP64 over the pebbles in caller order.  Point charges carry no
moment of their own.

``clump_vjp`` is the vector-Jacobian product of that map for given dL/dF_c
and dL/dT_c (r_k = x_k - X_c; a . (b x c) = c . (a x b)):

    dL/dq_k = Fbar_c . E_k + Tbar_c . (r_k x E_k)
    dL/dE_k = q_k (Fbar_c + Tbar_c x r_k)
    dL/dx_k = q_k (E_k x Tbar_c)
    dL/dX_c = - sum_{k in c} q_k (E_k x Tbar_c)

Pebbles outside every clump get zero.
"""
from __future__ import annotations

import numpy as np


def clump_reduce(x, q, E, offsets, centers):
    x = np.asarray(x, dtype=np.float64)
    F = np.asarray(q, dtype=np.float64)[:, None] * np.asarray(E, dtype=np.float64)
    C = len(offsets) - 1
    Fc = np.zeros((C, 3))
    Tc = np.zeros((C, 3))
    for c in range(C):
        for k in range(int(offsets[c]), int(offsets[c + 1])):
            Fc[c] += F[k]
            Tc[c] += np.cross(x[k] - centers[c], F[k])
    return Fc, Tc


def clump_vjp(x, q, E, offsets, centers, Fbar, Tbar):
    """(dL/dq [N], dL/dE [N,3], dL/dx [N,3], dL/dX [C,3]) for dL/dF_c = Fbar, dL/dT_c = Tbar."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    Fbar = np.asarray(Fbar, dtype=np.float64)
    Tbar = np.asarray(Tbar, dtype=np.float64)
    N = x.shape[0]
    C = len(offsets) - 1
    qb = np.zeros(N)
    Eb = np.zeros((N, 3))
    xb = np.zeros((N, 3))
    Xb = np.zeros((C, 3))
    for c in range(C):
        for k in range(int(offsets[c]), int(offsets[c + 1])):
            r = x[k] - centers[c]
            qb[k] = Fbar[c] @ E[k] + Tbar[c] @ np.cross(r, E[k])
            Eb[k] = q[k] * (Fbar[c] + np.cross(Tbar[c], r))
            xb[k] = q[k] * np.cross(E[k], Tbar[c])
            Xb[c] -= xb[k]
    return qb, Eb, xb, Xb
