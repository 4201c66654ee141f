"""Periodic Laplace sums over a cubic cell -- TEST INFRASTRUCTURE ONLY.

Section 2.4 allows periodic boundaries in the long-range solver and notes that
the Laplace lattice sum converges only for a charge-neutral cell (after de
Leeuw et al.).  The paper fixes no summation order or boundary term; the
reading used here is the Ewald sum with conducting ("tin-foil") boundary,
no surface term, and for a cell with net charge Q the implicit uniform
neutralising background (the sum is then still well defined).  For points
x_i and charges q_j in a cube of side L (volume V = L^3), with K = c/|r|:

    u_i = c sum_n sum_j' q_j / |x_i - x_j + n L|           (' : skip j = i at n = 0)

evaluated as the sum of

    real space   c sum_j sum_n' q_j erfc(a R)/R,   R = |x_i - x_j + n L|
    reciprocal   c (4 pi / V) sum_{k != 0} exp(-k^2/(4 a^2)) / k^2 sum_j q_j cos(k . (x_i - x_j))
    self         -c (2 a / sqrt(pi)) q_i
    background   -c pi Q / (a^2 V)

with k = 2 pi m / L, m integer; E = -grad u.  The result does not depend on
the splitting parameter a (one of the pins).

``lattice_far`` is the kernel the periodic fast method needs at the root:
the part of the periodic Green's function due to every image at cube distance
two or more, with its non-harmonic part removed:

    F(r) = G(r) - (2 pi / (3 V)) |r|^2 - sum_{|n|_inf <= 1} 1/|r + n L|,

G the Ewald Green's function of a unit charge (the four terms above with
q = 1 and no self term).  F is harmonic near r = 0, so a root equivalent
density reproduces it; the removed part sums in closed form over the sources
(``moment_correction``).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .direct import KERNELS

# Cut-offs: erfc(a R) is below 1e-16 for a R > 5.9 (real space) and
# exp(-k^2 / (4 a^2)) for k > 2 a 5.9 (reciprocal space).  With a L = 6.5 the
# real-space sum of a pair inside one cell needs the images |n|_inf <= 1 only.
_AL = 6.5          # a L
_CUT = 5.9


def _recip_vectors(L, a):
    mc = int(math.ceil(a * L * _CUT / math.pi)) + 1
    m = np.arange(-mc, mc + 1)
    g = np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3)
    # one of each pair +-m (the sum is even in k), m = 0 excluded
    keep = (g[:, 0] > 0) | ((g[:, 0] == 0) & (g[:, 1] > 0)) | ((g[:, 0] == 0) & (g[:, 1] == 0) & (g[:, 2] > 0))
    return 2.0 * math.pi * g[keep].astype(np.float64) / L


def _images(nmax):
    n = np.arange(-nmax, nmax + 1)
    return np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)


def ewald(x, q, L, kernel="laplace", targets=None, alpha=None, chunk=64):
    """Periodic potential and field at the points (or at ``targets``), tin-foil Ewald sum.

    x: [N,3] inside one cell of side L; q: [N].  Returns (u [nt], E [nt,3]).
    """
    c = KERNELS[kernel]
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    a = _AL / L if alpha is None else float(alpha)
    V = L ** 3
    tid = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    xt = x[tid]
    nt = xt.shape[0]
    u = np.zeros(nt)
    E = np.zeros((nt, 3))
    # real space: for |r|_inf < L only images with |n|_inf <= ceil(R_cut / L) can come within R_cut
    nimg = max(1, int(math.ceil(_CUT / (a * L))))
    imgs = _images(nimg) * L
    for s in range(0, nt, chunk):
        xi = xt[s:s + chunk]
        r = xi[:, None, None, :] - x[None, :, None, :] + imgs[None, None, :, :]
        R = np.sqrt(np.einsum("ijkl,ijkl->ijk", r, r))
        zero = R == 0.0
        R = np.where(zero, 1.0, R)
        ec = erfc(a * R) / R
        g = (ec + 2.0 * a / math.sqrt(math.pi) * np.exp(-(a * R) ** 2)) / (R * R)
        ec[zero] = 0.0
        g[zero] = 0.0
        u[s:s + chunk] += np.einsum("ijk,j->i", ec, q)
        E[s:s + chunk] += np.einsum("ijk,ijkl,j->il", g, r, q)
    # reciprocal space: structure factor per k, then both signs of k
    kv = _recip_vectors(L, a)
    k2 = np.einsum("ij,ij->i", kv, kv)
    w = 2.0 * (4.0 * math.pi / V) * np.exp(-k2 / (4.0 * a * a)) / k2
    ph = x @ kv.T                                   # [N, K]
    C = np.cos(ph).T @ q
    S = np.sin(ph).T @ q
    pt = xt @ kv.T                                  # [nt, K]
    ct, st = np.cos(pt), np.sin(pt)
    # sum_j q_j cos(k.(x - x_j)) = cos(k.x) C + sin(k.x) S
    u += (ct * C + st * S) @ w
    # -grad of the above: k (sin(k.x) C - cos(k.x) S)
    E += ((st * C - ct * S) * w) @ kv
    u += -2.0 * a / math.sqrt(math.pi) * q[tid] - math.pi * q.sum() / (a * a * V)
    return c * u, c * E


def lattice_far(r, L, alpha=None):
    """F(r) of the module docstring for rows of r ([M,3], |r|_inf < 1.5 L); kernel constant 1."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    a = _AL / L if alpha is None else float(alpha)
    V = L ** 3
    out = np.zeros(r.shape[0])
    rmax = float(np.abs(r).max()) / L if r.size else 0.0
    nimg = max(1, int(math.ceil(rmax + _CUT / (a * L))))
    imgs = _images(nimg) * L
    near = np.max(np.abs(imgs), axis=1) <= 1.0 * L + 1e-9 * L
    for s in range(0, r.shape[0], 256):
        rr = r[s:s + 256, None, :] + imgs[None, :, :]
        R = np.sqrt(np.einsum("ijk,ijk->ij", rr, rr))
        # near images: erfc(aR)/R - 1/R = -erf(aR)/R (finite at R = 0)
        Rs = np.where(R == 0.0, 1.0, R)
        t_far = np.where(near[None, :], 0.0, erfc(a * R) / Rs)
        t_near = np.where(near[None, :], -(1.0 - erfc(a * Rs)) / Rs, 0.0)
        t_near = np.where(R == 0.0, -2.0 * a / math.sqrt(math.pi), t_near)
        out[s:s + 256] = t_far.sum(1) + t_near.sum(1)
    kv = _recip_vectors(L, a)
    k2 = np.einsum("ij,ij->i", kv, kv)
    w = 2.0 * (4.0 * math.pi / V) * np.exp(-k2 / (4.0 * a * a)) / k2
    for s in range(0, r.shape[0], 1024):
        out[s:s + 1024] += np.cos(r[s:s + 1024] @ kv.T) @ w
    out += -math.pi / (a * a * V) - (2.0 * math.pi / (3.0 * V)) * np.einsum("ij,ij->i", r, r)
    return out


def moment_correction(xt, x, q, m, L, c):
    """u and E at targets xt of the removed part (2 pi c/(3V)) |x - y|^2 of the
    periodic kernel, summed over monopoles q and dipoles m (a dipole m at y
    contributes m . grad_x of the kernel, consistent with psi = -m . G).
    Coordinates relative to any common origin."""
    V = L ** 3
    k = 2.0 * math.pi * c / (3.0 * V)
    xt = np.asarray(xt, dtype=np.float64).reshape(-1, 3)
    x = np.asarray(x, dtype=np.float64)
    q = np.zeros(x.shape[0]) if q is None else np.asarray(q, dtype=np.float64)
    Q = q.sum()
    M = q @ x
    S2 = q @ np.einsum("ij,ij->i", x, x)
    u = k * (Q * np.einsum("ij,ij->i", xt, xt) - 2.0 * xt @ M + S2)
    E = -k * (2.0 * Q * xt - 2.0 * M)
    if m is not None:
        m = np.asarray(m, dtype=np.float64).reshape(-1, 3)
        D = m.sum(0)
        u += k * 2.0 * (xt @ D - np.einsum("ij,ij->", m, x))
        E += -k * 2.0 * D
    return u, E
