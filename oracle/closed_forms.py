"""Closed-form references used to pin the oracle -- TEST INFRASTRUCTURE ONLY.

* Two point charges (eq. (3)): F = q1 q2 r / (4 pi |r|^3) on charge 1.
* A uniformly charged spherical shell of total charge Q and radius R
  (shell theorem): u = Q/(4 pi R) and E = 0 inside, u = Q/(4 pi r) and
  E = Q r_hat/(4 pi r^2) outside.
* A point dipole p at the origin: u(x) = p.x / (4 pi |x|^3),
  E(x) = (3 (p.x_hat) x_hat - p) / (4 pi |x|^3).
* A dipole in a uniform field E0: force 0, torque p x E0.
"""
from __future__ import annotations

import math

import numpy as np

C_LAPLACE = 1.0 / (4.0 * math.pi)


def fibonacci_sphere(n: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    i = np.arange(n) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / n)
    theta = math.pi * (1.0 + 5.0 ** 0.5) * i
    pts = np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], axis=1)
    return np.asarray(center) + radius * pts


def shell_potential(Q: float, R: float, r: np.ndarray) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < R, Q * C_LAPLACE / R, Q * C_LAPLACE / np.maximum(r, 1e-300))


def shell_field(Q: float, R: float, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x, axis=1)
    out = Q * C_LAPLACE * x / np.maximum(r, 1e-300)[:, None] ** 3
    out[r < R] = 0.0
    return out


def coulomb_force(q1, q2, x1, x2):
    r = np.asarray(x1, dtype=np.float64) - np.asarray(x2, dtype=np.float64)
    return C_LAPLACE * q1 * q2 * r / np.linalg.norm(r) ** 3


def dipole_potential(p, x):
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x, axis=1)
    return C_LAPLACE * (x @ np.asarray(p)) / r ** 3


def dipole_field(p, x):
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    r = np.linalg.norm(x, axis=1)
    xh = x / r[:, None]
    return C_LAPLACE * (3.0 * (xh @ p)[:, None] * xh - p[None, :]) / r[:, None] ** 3
