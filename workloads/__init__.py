"""Seeded synthetic inputs for the KIFMM hot path.

This module only draws random numbers and lays out particle sets; it holds
none of the method's arithmetic.  Both the CPU oracle (in tests) and the GPU
library (in tests, ``smoke()`` and ``bench.py``) take their inputs from here,
so that the two sides see bit-identical positions and charges.

Every position and charge is rounded to FP32 and handed out as FP64, so the
FP32 GPU path and the FP64 oracle start from the same numbers.

The five workloads stand in for the paper's application examples (Section 3:
charged particles in a box, dipole clumps, clumped platelets, gravitational
collapse); the paper uses no public dataset.

  1  Laplace, uniform unit cube, charges U[-1,1], p=4, leaf 64, uniform tree
  2  Laplace, 60 % uniform + 40 % in 20 Gaussian clusters (sigma 0.02),
        charges N(0,1) with the mean removed, p=6, leaf 128, adaptive tree
  3  rigid clumps of 8 pebbles on the corners of a cube of edge 0.6 R,
        R lognormal(ln 0.003, 0.3) rescaled to 30 % bounding-sphere volume
        fraction, random rotations, random sequential addition packing,
        pebble charges N(0,1), p=6, leaf 128, adaptive tree
  4  Laplace, uniform unit cube, charges N(0,1), p=6, leaf 128, adaptive;
        adjoint loss target built from charges + 0.1 N(0,1)
  5  gravity, Plummer sphere (a = 0.1, truncated at r = 10 a), unit
        masses, p=8, leaf 256, adaptive tree, depth <= 12, root [-1,1)^3
  6  periodic unit cell (Laplace): co-oriented hexagonal two-layer
        platelets of 2 x 547 pebbles (N = 14 rings, spacing 0.01), one
        layer charged +1 and the other -1 (zero net charge, a dipole each),
        placed at random without overlap and wrapped into the cell, p=6,
        leaf 64, adaptive tree (the periodic platelet example of Section 3
        has 50 such platelets)
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = ["Workload", "make", "FULL_N", "SEED_BASE", "round_f32", "uniform_cube",
           "clustered", "plummer", "clumps", "platelets", "adjoint_target_charges"]

SEED_BASE = 9478
FULL_N = {1: 4096, 2: 1_048_576, 3: 1_600_000, 4: 524_288, 5: 8_388_608, 6: 54_700}


@dataclasses.dataclass
class Workload:
    name: str
    positions: np.ndarray            # [N,3] float64, FP32-representable
    charges: np.ndarray              # [N] float64, FP32-representable
    kernel: str                      # "laplace" or "gravity"
    p: int
    leaf_size: int
    adaptive: bool
    max_depth: int
    root: Optional[tuple]            # (lo[3], side) or None for automatic
    clump_offsets: Optional[np.ndarray] = None   # [C+1] int64, CSR over caller order
    clump_centers: Optional[np.ndarray] = None   # [C,3] float64
    periodic: bool = False           # the root cube is the unit cell of a periodic system

    @property
    def n(self) -> int:
        return int(self.positions.shape[0])


def round_f32(a: np.ndarray) -> np.ndarray:
    """Round to the nearest FP32 value and return it as FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _rng(k: int, seed: Optional[int]) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k if seed is None else seed)


def uniform_cube(rng: np.random.Generator, n: int) -> np.ndarray:
    x = round_f32(rng.random((n, 3)))
    return np.minimum(x, np.nextafter(1.0, 0.0))   # stay inside [0,1)


def clustered(rng: np.random.Generator, n: int, n_clusters: int = 20,
              sigma: float = 0.02, frac_uniform: float = 0.6) -> np.ndarray:
    nu = int(round(frac_uniform * n))
    nc = n - nu
    xu = rng.random((nu, 3))
    centres = rng.random((n_clusters, 3))
    which = rng.integers(0, n_clusters, size=nc)
    xc = centres[which] + sigma * rng.standard_normal((nc, 3))
    bad = np.any((xc < 0.0) | (xc >= 1.0), axis=1)
    while bad.any():                        # resample the tails back into the cube
        k = int(bad.sum())
        xc[bad] = centres[which[bad]] + sigma * rng.standard_normal((k, 3))
        bad = np.any((xc < 0.0) | (xc >= 1.0), axis=1)
    x = np.concatenate([xu, xc], axis=0)
    x = round_f32(x)
    return np.minimum(x, np.nextafter(1.0, 0.0))


def plummer(rng: np.random.Generator, n: int, a: float = 0.1, rmax: float = 1.0) -> np.ndarray:
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = int((n - out.shape[0]) * 1.05) + 16
        u = rng.random(m)
        u = u[u > 0.0]
        r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        r = r[r <= rmax]
        d = rng.standard_normal((r.shape[0], 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        out = np.concatenate([out, d * r[:, None]], axis=0)
    return round_f32(out[:n])


def _random_rotations(rng: np.random.Generator, k: int) -> np.ndarray:
    """Uniform random rotation matrices from uniform unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random(k), rng.random(k), rng.random(k)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    w = a * np.sin(2 * np.pi * u2)
    x = a * np.cos(2 * np.pi * u2)
    y = b * np.sin(2 * np.pi * u3)
    z = b * np.cos(2 * np.pi * u3)
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _rsa_pack(rng: np.random.Generator, radii: np.ndarray, batch: int = 1024,
              max_rounds: int = 4000, cap: int = 160) -> np.ndarray:
    """Random sequential addition of spheres (largest first) inside the unit cube.

    Spheres are taken in groups (at most ``batch``, radii within 5 % of the
    group's largest) in decreasing radius; a group is placed completely before
    the next one starts.  Each round proposes one uniform position for every
    unplaced sphere of the group and accepts a proposal when it overlaps
    neither a placed sphere nor an earlier proposal accepted in the same round.
    A uniform cell grid of side >= 2*max(radii) (at most ``cap`` spheres per
    cell) bounds the overlap checks.  Returns the centres in the order of
    ``radii``.
    """
    order = np.argsort(-radii, kind="stable")
    rmax = float(radii.max())
    g = max(1, int(1.0 / (2.0 * rmax)))
    cell = 1.0 / g
    n = radii.shape[0]
    cen = np.zeros((n, 3))
    # grid[cell, k] = placement slot of the k-th sphere in that cell
    grid = np.full((g * g * g + 1, cap), n, dtype=np.int64)   # row g^3 is an empty sentinel
    gcnt = np.zeros(g * g * g + 1, dtype=np.int64)
    pc = np.full((n + 1, 3), 1e9)         # slot n is a far-away sentinel
    pr = np.zeros(n + 1)
    npl = 0
    offs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    groups = []
    i = 0
    while i < n:
        j = i + 1
        while j < n and j - i < batch and radii[order[j]] >= 0.95 * radii[order[i]]:
            j += 1
        groups.append(order[i:j])
        i = j
    for grp in groups:
        todo = np.asarray(grp)
        rounds = 0
        while todo.size:
            rounds += 1
            if rounds > max_rounds:
                raise RuntimeError("random sequential addition did not converge")
            r = radii[todo]
            c = r[:, None] + (1.0 - 2.0 * r[:, None]) * rng.random((todo.size, 3))
            ci = np.minimum((c / cell).astype(np.int64), g - 1)
            nb = ci[:, None, :] + offs[None, :, :]                      # [K,27,3]
            inside = np.all((nb >= 0) & (nb < g), axis=2)
            cid = np.where(inside, (nb[..., 0] * g + nb[..., 1]) * g + nb[..., 2], g * g * g)
            m = max(1, int(gcnt.max()))
            slots = grid[cid][:, :, :m].reshape(todo.size, -1)           # [K, 27*m]
            d2 = np.sum((pc[slots] - c[:, None, :]) ** 2, axis=2)
            ok = ~np.any(d2 < (pr[slots] + r[:, None]) ** 2, axis=1)
            # proposals of this batch against the earlier accepted ones (in order)
            acc = []
            for t in np.nonzero(ok)[0]:
                if acc:
                    a = np.asarray(acc)
                    if np.any(np.sum((c[a] - c[t]) ** 2, axis=1) < (r[a] + r[t]) ** 2):
                        ok[t] = False
                        continue
                acc.append(t)
            for t in acc:
                q = int((ci[t, 0] * g + ci[t, 1]) * g + ci[t, 2])
                if gcnt[q] >= cap:
                    raise RuntimeError("packing grid cell overflow")
                grid[q, gcnt[q]] = npl
                gcnt[q] += 1
                pc[npl] = c[t]
                pr[npl] = r[t]
                npl += 1
                cen[todo[t]] = c[t]
            todo = todo[~ok]
    return cen


def clumps(rng: np.random.Generator, n_clumps: int, phi: float = 0.30,
           mu: float = math.log(0.003), sigma: float = 0.3):
    """Rigid 8-pebble clumps (cube corners, edge 0.6 R) packed at volume fraction phi.

    The drawn radii are rescaled by (phi / phi_drawn)^(1/3) so that the bounding
    spheres fill the requested fraction of the unit cube.
    Returns (positions [8C,3], offsets [C+1], centres [C,3]).
    """
    R = rng.lognormal(mu, sigma, size=n_clumps)
    phi_drawn = float(np.sum(4.0 / 3.0 * np.pi * R ** 3))
    R = R * (phi / phi_drawn) ** (1.0 / 3.0)
    centres = _rsa_pack(rng, R)
    rot = _random_rotations(rng, n_clumps)
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                       dtype=np.float64) * 0.3
    local = corners[None, :, :] * R[:, None, None]                 # [C,8,3]
    pts = centres[:, None, :] + np.einsum("cij,ckj->cki", rot, local)
    pos = round_f32(pts.reshape(-1, 3))
    pos = np.clip(pos, 0.0, np.nextafter(1.0, 0.0))
    offsets = np.arange(0, 8 * n_clumps + 1, 8, dtype=np.int64)
    return pos, offsets, round_f32(centres)


def _hex_layer(rings: int, spacing: float) -> np.ndarray:
    """Triangular-lattice points within hexagonal distance rings-1 of the origin (z = 0)."""
    m = rings - 1
    pts = []
    for i in range(-m, m + 1):
        for j in range(-m, m + 1):
            if abs(i + j) <= m:
                pts.append((spacing * (i + 0.5 * j), spacing * (math.sqrt(3.0) / 2.0) * j, 0.0))
    return np.array(pts, dtype=np.float64)


def platelets(rng: np.random.Generator, n_platelets: int, rings: int = 14, spacing: float = 0.01):
    """Co-oriented two-layer close-packed platelets in the periodic unit cell.

    Layer A at height 0 carries +1, layer B (shifted to the hollow sites, at
    height spacing * sqrt(2/3)) carries -1.  Centres are drawn uniformly and
    rejected while a platelet's bounding cylinder overlaps another's under
    the minimum-image convention.  Returns (positions [2 k n_platelets, 3]
    in [0, 1), charges).
    """
    a = _hex_layer(rings, spacing)
    b = a + np.array([0.5 * spacing, spacing / (2.0 * math.sqrt(3.0)), spacing * math.sqrt(2.0 / 3.0)])
    rad = spacing * (rings - 1) + spacing      # bounding radius, with margin
    thick = 2.0 * spacing * math.sqrt(2.0 / 3.0) + spacing
    cen = []
    while len(cen) < n_platelets:
        c = rng.random(3)
        ok = True
        for d in cen:
            dd = c - d
            dd -= np.round(dd)
            if math.hypot(dd[0], dd[1]) < 2.0 * rad and abs(dd[2]) < thick:
                ok = False
                break
        if ok:
            cen.append(c)
    cen = np.array(cen)
    one = np.concatenate([a, b])
    pos = (cen[:, None, :] + one[None, :, :]).reshape(-1, 3) % 1.0
    pos = round_f32(pos)
    pos = np.where(pos >= 1.0, 0.0, pos)
    q = np.tile(np.concatenate([np.ones(a.shape[0]), -np.ones(b.shape[0])]), n_platelets)
    return pos, q


def adjoint_target_charges(charges: np.ndarray, seed: int) -> np.ndarray:
    """Charges perturbed by 0.1 * N(0,1); the field they produce is the loss target."""
    rng = np.random.default_rng(seed)
    return round_f32(charges + 0.1 * rng.standard_normal(charges.shape[0]))


def make(k: int, n: Optional[int] = None, seed: Optional[int] = None) -> Workload:
    """Build workload ``k`` (1..6) with ``n`` points (default: the full size; the
    platelet cell rounds down to whole platelets and is periodic)."""
    rng = _rng(k, seed)
    N = FULL_N[k] if n is None else int(n)
    if k == 1:
        x = uniform_cube(rng, N)
        q = round_f32(rng.uniform(-1.0, 1.0, N))
        return Workload("uniform_4096_p4", x, q, "laplace", 4, 64, False, 21,
                        ((0.0, 0.0, 0.0), 1.0))
    if k == 2:
        x = clustered(rng, N)
        q = rng.standard_normal(N)
        q = round_f32(q - q.mean())
        return Workload("clustered_1M_p6", x, q, "laplace", 6, 128, True, 21,
                        ((0.0, 0.0, 0.0), 1.0))
    if k == 3:
        C = max(1, N // 8)
        x, off, cen = clumps(rng, C)
        q = round_f32(rng.standard_normal(x.shape[0]))
        return Workload("clumps_200k_p6", x, q, "laplace", 6, 128, True, 21,
                        ((0.0, 0.0, 0.0), 1.0), off, cen)
    if k == 4:
        x = uniform_cube(rng, N)
        q = round_f32(rng.standard_normal(N))
        return Workload("uniform_524k_p6", x, q, "laplace", 6, 128, True, 21,
                        ((0.0, 0.0, 0.0), 1.0))
    if k == 5:
        x = plummer(rng, N)
        q = np.ones(N)
        return Workload("plummer_8M_p8", x, q, "gravity", 8, 256, True, 12,
                        ((-1.0, -1.0, -1.0), 2.0))
    if k == 6:
        per = 2 * (1 + 3 * 14 * 13)
        x, q = platelets(rng, max(1, N // per))
        return Workload("platelets_periodic_p6", x, q, "laplace", 6, 64, True, 21,
                        ((0.0, 0.0, 0.0), 1.0), periodic=True)
    raise ValueError(f"unknown workload {k}")
