"""Surfaces, kernel matrices and check-to-equivalent pseudoinverses -- TEST INFRASTRUCTURE ONLY.

Section 2.2: a box's far field (and its local field) is represented by a
density on samples of an equivalent surface, the approximation at y being
sum_i phi_i K(x_i, y); the M2M, L2L and M2L operators are matrices computed
from the kernel.  The paper leaves the surfaces and the regularisation open;
the readings used here are:

* Surface of a box with centre c and side w:  c + rho w (g - 1/2), g the
  boundary points of the p^3 grid {i/(p-1)}^3 (i slowest, k fastest),
  n = 6 (p-1)^2 + 2 points (56 at p = 4).
* rho = 1.05 for the upward equivalent and downward check surfaces,
  rho = 2.95 for the upward check and downward equivalent surfaces.
* Check-to-equivalent maps: truncated-SVD pseudoinverses in FP64 that drop
  singular values below tau * sigma_1 (tau = 1e-7 by default):
    UC2E = pinv_tau(K(uc, ue)),   DC2E = pinv_tau(K(dc, de)).
"""
from __future__ import annotations

import functools

import numpy as np

RHO_UE = 1.05
RHO_UC = 2.95
RHO_DE = 2.95
RHO_DC = 1.05
TAU = 1e-7


@functools.lru_cache(maxsize=None)
def _surface_grid(p: int) -> np.ndarray:
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if min(i, j, k) == 0 or max(i, j, k) == p - 1:
                    pts.append((i / (p - 1), j / (p - 1), k / (p - 1)))
    g = np.array(pts, dtype=np.float64)
    g.setflags(write=False)
    return g


def surface_grid(p: int) -> np.ndarray:
    """Boundary points of the p^3 grid in [0,1]^3, i slowest and k fastest."""
    return _surface_grid(p)


def n_surface(p: int) -> int:
    return 6 * (p - 1) ** 2 + 2


def surface(p: int, rho: float, center, w: float) -> np.ndarray:
    return np.asarray(center, dtype=np.float64) + rho * w * (surface_grid(p) - 0.5)


def kernel_matrix(trg: np.ndarray, src: np.ndarray, c: float) -> np.ndarray:
    """K[i, j] = c / |trg_i - src_j|."""
    d = trg[:, None, :] - src[None, :, :]
    return c / np.sqrt(np.einsum("ijk,ijk->ij", d, d))


def field_matrices(trg: np.ndarray, src: np.ndarray, c: float):
    """G[a][i, j] = c (trg_i - src_j)_a / |trg_i - src_j|^3  (= -grad_trg K)."""
    d = trg[:, None, :] - src[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    ri3 = r2 ** -1.5
    return [c * d[:, :, a] * ri3 for a in range(3)]


def hessian_matrices(trg: np.ndarray, src: np.ndarray, c: float):
    """Hessian of K w.r.t. the target, (xx,yy,zz,xy,xz,yz), each [nt, ns]."""
    d = trg[:, None, :] - src[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    ri3 = r2 ** -1.5
    ri5 = r2 ** -2.5
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    out = []
    for a, b in pairs:
        m = 3.0 * d[:, :, a] * d[:, :, b] * ri5
        if a == b:
            m = m - ri3
        out.append(c * m)
    return out


def pinv_truncated(A: np.ndarray, tau: float = TAU):
    """Pseudoinverse from the SVD, dropping sigma_k < tau * sigma_1.

    Returns (P, kept rank, singular values).
    """
    U, S, Vt = np.linalg.svd(A)
    keep = S >= tau * S[0]
    P = (Vt[keep].T / S[keep]) @ U[:, keep].T
    return P, int(keep.sum()), S


class Operators:
    """Per-level FP64 operators for a root cube of side s (built lazily).

    ``m2l_rtol`` > 0 applies every M2L operator in a truncated common basis
    (a reading; the paper does not say how its M2L is applied).  Because
    M2L(-d) = M2L(d)^T, the left singular vectors of H = [M2L(d_1) ... M2L(d_316)]
    also span the right ones of the stacked operators, so one basis Q (the left
    singular vectors with sigma >= m2l_rtol * sigma_1) serves both sides:
        M2L_c(d) = Q (Q^T M2L(d) Q) Q^T,
    which keeps M2L_c(-d) = M2L_c(d)^T (the adjoint stays exact) and differs
    from M2L(d) by at most 2 m2l_rtol sigma_1(H) in the spectral norm.
    """

    def __init__(self, p: int, c: float, s: float, tau: float = TAU, m2l_rtol: float = 0.0):
        self.p, self.c, self.s, self.tau = p, c, s, tau
        self.m2l_rtol = float(m2l_rtol)
        self.n = n_surface(p)
        self._cache = {}

    def w(self, l):
        return self.s / (1 << l)

    def uc2e(self, l):
        key = ("uc2e", l)
        if key not in self._cache:
            w = self.w(l)
            A = kernel_matrix(surface(self.p, RHO_UC, 0, w), surface(self.p, RHO_UE, 0, w), self.c)
            self._cache[key] = pinv_truncated(A, self.tau)[0]
        return self._cache[key]

    def dc2e(self, l):
        key = ("dc2e", l)
        if key not in self._cache:
            w = self.w(l)
            A = kernel_matrix(surface(self.p, RHO_DC, 0, w), surface(self.p, RHO_DE, 0, w), self.c)
            self._cache[key] = pinv_truncated(A, self.tau)[0]
        return self._cache[key]

    @staticmethod
    def octant_offset(o):
        """Child-centre offset (in parent widths) of octant o: +-1/4 per axis."""
        return np.array([((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5]) * 0.5

    def m2m(self, l, o):
        """K(uc of a parent at level l, ue of its child at octant o)."""
        key = ("m2m", l, o)
        if key not in self._cache:
            w = self.w(l)
            trg = surface(self.p, RHO_UC, 0, w)
            src = surface(self.p, RHO_UE, self.octant_offset(o) * w, w / 2)
            self._cache[key] = kernel_matrix(trg, src, self.c)
        return self._cache[key]

    def l2l(self, l, o):
        """K(dc of a child at octant o, de of its parent at level l)."""
        key = ("l2l", l, o)
        if key not in self._cache:
            w = self.w(l)
            trg = surface(self.p, RHO_DC, self.octant_offset(o) * w, w / 2)
            src = surface(self.p, RHO_DE, 0, w)
            self._cache[key] = kernel_matrix(trg, src, self.c)
        return self._cache[key]

    def m2l_exact(self, l, d):
        """K(dc of a target box at level l, ue of the source box at offset d)."""
        w = self.w(l)
        trg = surface(self.p, RHO_DC, 0, w)
        src = surface(self.p, RHO_UE, np.asarray(d, dtype=np.float64) * w, w)
        return kernel_matrix(trg, src, self.c)

    def m2l_basis(self, l):
        """(Q, singular values of H) of the truncated common M2L basis at level l."""
        key = ("m2l_basis", l)
        if key not in self._cache:
            H = np.hstack([self.m2l_exact(l, d) for d in far_offsets()])
            U, S, _ = np.linalg.svd(H, full_matrices=False)
            k = int(np.sum(S >= self.m2l_rtol * S[0]))
            self._cache[key] = (U[:, :k], S)
        return self._cache[key]

    def m2l(self, l, d):
        """The M2L operator as the sweep applies it (compressed when m2l_rtol > 0)."""
        M = self.m2l_exact(l, d)
        if self.m2l_rtol <= 0.0:
            return M
        Q, _ = self.m2l_basis(l)
        return Q @ (Q.T @ M @ Q) @ Q.T


def far_offsets():
    """The 316 offsets of [-3,3]^3 outside [-1,1]^3, lexicographic (dx, dy, dz)."""
    return [(dx, dy, dz) for dx in range(-3, 4) for dy in range(-3, 4) for dz in range(-3, 4)
            if max(abs(dx), abs(dy), abs(dz)) > 1]
