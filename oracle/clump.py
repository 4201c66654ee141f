"""Per-clump force and torque -- TEST INFRASTRUCTURE ONLY.

Section 2.4: the long-range forces are applied to the pebbles and then the
forces and moments on the pebbles are summed into the force and torque of
each clump.  With F_k = q_k E_k on pebble k and the clump reference point X_c
(its centre of mass, supplied by the caller):

    F_c = sum_{k in c} F_k,     T_c = sum_{k in c} (x_k - X_c) x F_k,

accumulated in FP64 over the pebbles in caller order.  Point charges carry no
moment of their own.
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
