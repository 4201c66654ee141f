"""FP64 kernel-independent FMM and its discrete adjoint -- TEST INFRASTRUCTURE ONLY.

Follows the four steps of Section 2.2 in order:

1. octree (``tree.build_tree``) and lists (``tree.build_lists``);
2. upward pass, fine to coarse: a leaf's upward check potential comes from
   its points, a parent's from its children's equivalent densities (M2M);
   the upward equivalent density is UC2E applied to the check potential;
3. downward pass, coarse to fine, from level 2: the downward check potential
   of a box sums the V-list equivalent densities (M2L), the X-list points and
   (from level 3) the parent's downward equivalent density (L2L); the
   downward equivalent density is DC2E applied to it;
4. leaf evaluation: for a target in leaf B, the downward density of B (from
   level 2), the upward densities of the W-list boxes and the points of the
   U-list leaves (pairs at distance zero skipped).

A W/X pair links a box A and a finer box F (F in W(A), A in X(F)).  The paper
leaves open how such a pair is evaluated; the reading used here (see
``direct_xw``): when F is a leaf holding at most n points (n the surface
size) the pair is summed point to point in both directions, which costs
fewer kernel evaluations than n per point of the other box, and is exact;
otherwise A's points go onto F's downward check surface (X) and F's upward
density is evaluated at A's points (W).

Sources carry a monopole s_j and optionally a dipole m_j (the dipole sources
are what the adjoint needs); targets receive the potential, E = -grad and, on
request, the Hessian of the potential.

The discrete adjoint (``vjp``) uses that the discrete operator u = A(x) q is
symmetric under the chosen surfaces (uc and de coincide, ue and dc coincide,
DC2E = UC2E^T, M2M and L2L are transposes, V-list pairs come in +-d, W and X
are transposes, P2P is symmetric): for L = sum ubar.u + Ebar.E,
    qbar = psi,   xbar_k = -ubar_k E_k - H_k Ebar_k + q_k grad psi(x_k),
psi being the FMM of monopoles ubar and dipoles Ebar and H the FMM Hessian of
the forward potential.  Both are plain calls of the forward sweep.
"""
from __future__ import annotations

import dataclasses
from collections import defaultdict
from typing import Optional

import numpy as np

from . import pairsum
from .direct import KERNELS, hess_times
from .operators import (RHO_DC, RHO_DE, RHO_UC, RHO_UE, TAU, Operators, field_matrices,
                        hessian_matrices, kernel_matrix, surface)
from .periodic import lattice_far, moment_correction
from .tree import Lists, Tree, build_lists, build_tree, decode


@dataclasses.dataclass
class Plan:
    tree: Tree
    lists: Lists
    kernel: str
    c: float
    p: int
    tau: float
    ops: Operators
    x: np.ndarray            # sorted positions [N,3] FP64
    periodic: bool = False   # the root cube tiles space (Laplace, Ewald sum)

    @property
    def n(self):
        return self.x.shape[0]

    def with_positions(self, x_caller: np.ndarray) -> "Plan":
        """Same (frozen) tree, lists and operators; new positions."""
        xs = np.asarray(x_caller, dtype=np.float64)[self.tree.perm]
        return dataclasses.replace(self, x=xs)


def plan(x, kernel="laplace", p=6, leaf_size=128, adaptive=True, max_depth=21, root=None,
         tau=TAU, periodic=False, m2l_rtol=0.0) -> Plan:
    """``periodic``: the explicit root cube ``root`` = (lo, side) is the unit
    cell of a periodic system (Laplace only; every point inside the cell).
    ``m2l_rtol`` > 0: M2L in the truncated common basis (``Operators``)."""
    x = np.asarray(x, dtype=np.float64)
    if periodic and (root is None or kernel != "laplace"):
        raise ValueError("periodic sums need the Laplace kernel and the cell as an explicit root")
    t = build_tree(x, leaf_size, adaptive, max_depth, root)
    L = build_lists(t, periodic)
    c = KERNELS[kernel]
    return Plan(t, L, kernel, c, p, tau, Operators(p, c, t.s, tau, m2l_rtol), x[t.perm], periodic)


def _lowest(P: Plan) -> int:
    """Coarsest level with far-field interactions: 2 in free space; 0 when
    periodic (the root receives the images beyond its neighbours)."""
    return 0 if P.periodic else 2


def direct_xw(P: Plan, f: int) -> bool:
    """Whether the W/X pairs whose finer box is ``f`` are summed point to point:
    ``f`` is a leaf holding at most n points (the rule is symmetric, so the
    discrete operator stays symmetric)."""
    t = P.tree
    return bool(t.is_leaf[f]) and int(t.end[f] - t.begin[f]) <= P.ops.n


def near_lists(P: Plan):
    """Point-to-point source boxes of every box: the U list, the X list when the
    box itself is a direct finer box, and the W-list boxes that are.  Entries
    keep their image shift.  Returns a list of lists."""
    L = P.lists
    near = []
    for b in range(P.tree.nboxes):
        row = list(L.U[b])
        if L.X[b] and direct_xw(P, b):
            row.extend(L.X[b])
        row.extend(e for e in L.W[b] if direct_xw(P, decode(e)[0]))
        near.append(row)
    return near


def _image(P: Plan, e):
    """(box, displacement in length units) of a list entry."""
    b, sh = decode(e)
    return b, sh * P.tree.s


_LATTICE = {}


def lattice_operator(P: Plan) -> np.ndarray:
    """Root downward check potential from the root upward density for all
    images at cube distance >= 2: c F(dc_i - ue_j), F the harmonic lattice
    kernel (kept per (p, cell side, c) for the process)."""
    t = P.tree
    key = (P.p, float(t.s), float(P.c))
    if key not in _LATTICE:
        dc = surface(P.p, RHO_DC, 0, t.s)
        ue = surface(P.p, RHO_UE, 0, t.s)
        r = (dc[:, None, :] - ue[None, :, :]).reshape(-1, 3)
        _LATTICE[key] = P.c * lattice_far(r, t.s).reshape(dc.shape[0], ue.shape[0])
    return _LATTICE[key]


def _octant(anchor):
    return int(((anchor[0] & 1) << 2) | ((anchor[1] & 1) << 1) | (anchor[2] & 1))


def upward(P: Plan, s: np.ndarray, m: Optional[np.ndarray]) -> np.ndarray:
    """Upward equivalent densities phi_u [B, n] (zero above the coarsest far-field level)."""
    t, ops, c = P.tree, P.ops, P.c
    phi = np.zeros((t.nboxes, ops.n))
    for l in range(t.depth, _lowest(P) - 1, -1):
        w = ops.w(l)
        boxes = np.arange(t.level_start[l], t.level_start[l + 1])
        psi = np.zeros((boxes.shape[0], ops.n))
        for r, b in enumerate(boxes):
            if not t.is_leaf[b]:
                continue
            b0, b1 = t.begin[b], t.end[b]
            uc = surface(P.p, RHO_UC, t.center(b), w)
            # psi = K(uc, x_B) s_B (- the dipole part), summed point by point in C
            psi[r] = pairsum.direct(uc, P.x[b0:b1], s[b0:b1], None if m is None else m[b0:b1], c)[0]
        for o in range(8):
            ch = t.children[boxes, o]
            rows = np.nonzero(ch >= 0)[0]
            if rows.size:
                psi[rows] += phi[ch[rows]] @ ops.m2m(l, o).T
        phi[boxes] = psi @ ops.uc2e(l).T
    return phi


def downward(P: Plan, s, m, phi_u, needed: np.ndarray) -> np.ndarray:
    """Downward equivalent densities phi_d [B, n] for the boxes flagged in ``needed``."""
    t, ops, c, L = P.tree, P.ops, P.c, P.lists
    phi = np.zeros((t.nboxes, ops.n))
    l0 = _lowest(P)
    for l in range(l0, t.depth + 1):
        w = ops.w(l)
        boxes = np.arange(t.level_start[l], t.level_start[l + 1])
        boxes = boxes[needed[boxes]]
        if boxes.size == 0:
            continue
        psi = np.zeros((boxes.shape[0], ops.n))
        # V list, grouped by the offset between source and target
        groups = defaultdict(lambda: ([], []))
        for r, b in enumerate(boxes):
            for e in L.V[b]:
                a, sh = decode(e)
                d = tuple(int(v) for v in (t.anchor[a] + sh * (1 << l) - t.anchor[b]))
                groups[d][0].append(r)
                groups[d][1].append(a)
        for d, (rows, srcs) in groups.items():
            np.add.at(psi, np.array(rows), phi_u[np.array(srcs)] @ ops.m2l(l, d).T)
        # X list: source points straight onto the downward check surface
        # (unless the pairs are summed point to point)
        for r, b in enumerate(boxes):
            if not L.X[b] or direct_xw(P, b):
                continue
            dc = surface(P.p, RHO_DC, t.center(b), w)
            for e in L.X[b]:
                a, disp = _image(P, e)
                a0, a1 = t.begin[a], t.end[a]
                psi[r] += pairsum.direct(dc, P.x[a0:a1] + disp, s[a0:a1], None if m is None else m[a0:a1], c)[0]
        # periodic root: every image beyond the root's neighbours
        if l == 0 and P.periodic:
            psi += phi_u[boxes] @ lattice_operator(P).T
        # L2L from the parent
        if l > l0:
            par = t.parent[boxes]
            octs = np.array([_octant(t.anchor[b]) for b in boxes])
            for o in range(8):
                rows = np.nonzero(octs == o)[0]
                if rows.size:
                    psi[rows] += phi[par[rows]] @ ops.l2l(l - 1, o).T
        phi[boxes] = psi @ ops.dc2e(l).T
    return phi


def evaluate_sorted(P: Plan, s, m=None, targets=None, hess=False, part="all"):
    """FMM outputs at sorted targets (all points by default).

    Returns (u [nt], E [nt,3], H [nt,6] or None) for the sorted indices
    ``targets``; ``part`` "far" keeps only the expansions (local and W list),
    "near" only the point-to-point sum over the near lists.
    """
    if part not in ("all", "far", "near"):
        raise ValueError(f"unknown part {part!r}")
    t, ops, c, L = P.tree, P.ops, P.c, P.lists
    s = np.asarray(s, dtype=np.float64)
    m = None if m is None else np.asarray(m, dtype=np.float64)
    if targets is None:
        targets = np.arange(P.n)
    targets = np.asarray(targets, dtype=np.int64)
    nt = targets.shape[0]
    leaves = t.leaves()
    # leaf of each sorted point
    leaf_of = np.empty(P.n, dtype=np.int64)
    for b in leaves:
        leaf_of[t.begin[b]:t.end[b]] = b
    tleaf = leaf_of[targets]
    # boxes whose downward density is needed: ancestors of the target leaves
    needed = np.zeros(t.nboxes, dtype=bool)
    for b in np.unique(tleaf):
        a = int(b)
        while a >= 0 and not needed[a]:
            needed[a] = True
            a = int(t.parent[a])
    u = np.zeros(nt)
    E = np.zeros((nt, 3))
    H = np.zeros((nt, 6)) if hess else None
    if part != "near":
        phi_u = upward(P, s, m)
        phi_d = downward(P, s, m, phi_u, needed)
    order = np.argsort(tleaf, kind="stable")
    bounds = np.nonzero(np.diff(tleaf[order]))[0] + 1
    for grp in (np.split(order, bounds) if part != "near" else []):
        if grp.size == 0:
            continue
        b = int(tleaf[grp[0]])
        xt = P.x[targets[grp]]
        surf, dens = [], []
        lb = int(t.level[b])
        if lb >= _lowest(P):
            surf.append(surface(P.p, RHO_DE, t.center(b), ops.w(lb)))
            dens.append(phi_d[b])
        for e in L.W[b]:
            a, disp = _image(P, e)
            if direct_xw(P, a):
                continue   # summed point to point with the near field
            surf.append(surface(P.p, RHO_UE, t.center(a) + disp, ops.w(int(t.level[a]))))
            dens.append(phi_u[a])
        if not surf:
            continue
        S = np.concatenate(surf)
        D = np.concatenate(dens)
        # u = K(x, S) D, E = G(x, S) D, H = Hess K(x, S) D, summed point by point in C
        ul, El, Hl = pairsum.direct(xt, S, D, None, c, hess)
        u[grp] += ul
        E[grp] += El
        if hess:
            H[grp] += Hl

    def periodic_part():
        # the non-harmonic part of the periodic kernel, summed in closed form
        # (relative to the cell centre)
        o = t.lo + 0.5 * t.s
        uc, Ec = moment_correction(P.x[targets] - o, P.x - o, s, m, t.s, c)
        u[:] += uc
        E[:] += Ec
        if hess:
            # grad grad of (2 pi c / 3V) Q |x|^2
            H[:, :3] += 4.0 * np.pi * c / (3.0 * t.s ** 3) * s.sum()

    if part == "far":
        if P.periodic:
            periodic_part()
        return u, E, H
    near = near_lists(P)
    uoff = np.zeros(len(near) + 1, dtype=np.int64)
    uoff[1:] = np.cumsum([len(r) for r in near])
    uenc = np.array([e for r in near for e in r], dtype=np.int64)
    uidx = np.array([decode(e)[0] for e in uenc], dtype=np.int64)
    ushift = None
    if P.periodic:
        ushift = np.array([decode(e)[1] * t.s for e in uenc], dtype=np.float64).reshape(-1, 3)
    un, En, Hn = pairsum.p2p(targets, tleaf, t.begin, t.end, uoff, uidx, P.x, s, m, c, hess, ushift)
    u += un
    E += En
    if hess:
        H += Hn
    if P.periodic and part == "all":
        periodic_part()
    return u, E, H


def forward(P: Plan, q, targets=None, part="all"):
    """Potential and field in caller order (or at caller indices ``targets``);
    ``part`` as in ``evaluate_sorted``."""
    q = np.asarray(q, dtype=np.float64)
    inv = np.empty_like(P.tree.perm)
    inv[P.tree.perm] = np.arange(P.n)
    qs = q[P.tree.perm]
    if targets is None:
        u, E, _ = evaluate_sorted(P, qs, part=part)
        out_u = np.empty(P.n)
        out_E = np.empty((P.n, 3))
        out_u[P.tree.perm] = u
        out_E[P.tree.perm] = E
        return out_u, out_E
    u, E, _ = evaluate_sorted(P, qs, targets=inv[np.asarray(targets)], part=part)
    return u, E


def forward_dipoles(P: Plan, q, m, targets=None, grad=False):
    """Potential and field of monopoles q (or none) and dipoles m (or none; a
    dipole m at y makes psi(x) = -m . G(x - y)), in caller order or at caller
    indices ``targets``; the same sweep as the charges, with the dipole part in
    every point-to-surface and point-to-point sum.  With ``grad`` also the
    field gradient dE_a/dx_b = -Hess u (xx, yy, zz, xy, xz, yz)."""
    perm = P.tree.perm
    qs = np.zeros(P.n) if q is None else np.asarray(q, dtype=np.float64)[perm]
    ms = None if m is None else np.asarray(m, dtype=np.float64).reshape(-1, 3)[perm]
    if targets is None:
        u, E, H = evaluate_sorted(P, qs, ms, hess=grad)
        out_u = np.empty(P.n)
        out_E = np.empty((P.n, 3))
        out_u[perm] = u
        out_E[perm] = E
        if not grad:
            return out_u, out_E
        out_G = np.empty((P.n, 6))
        out_G[perm] = -H
        return out_u, out_E, out_G
    inv = np.empty_like(perm)
    inv[perm] = np.arange(P.n)
    u, E, H = evaluate_sorted(P, qs, ms, targets=inv[np.asarray(targets)], hess=grad)
    return (u, E, -H) if grad else (u, E)


def vjp(P: Plan, q, ubar, Ebar, targets=None):
    """Exact vector-Jacobian product of the discrete map (q, x) -> (u, E), frozen tree.

    Returns (qbar, xbar) in caller order: [N], [N,3], or at the caller indices
    ``targets`` only (every entry of the product is an evaluation at one point).
    """
    perm = P.tree.perm
    qs = np.asarray(q, dtype=np.float64)[perm]
    us = np.asarray(ubar, dtype=np.float64)[perm]
    Es = np.asarray(Ebar, dtype=np.float64).reshape(-1, 3)[perm]
    if targets is None:
        ts = None
        sel = slice(None)
    else:
        inv = np.empty_like(perm)
        inv[perm] = np.arange(P.n)
        ts = inv[np.asarray(targets)]
        sel = ts
    _, E, H = evaluate_sorted(P, qs, targets=ts, hess=True)
    psi, Epsi, _ = evaluate_sorted(P, us, Es, targets=ts)
    qbar_s = psi
    xbar_s = -us[sel, None] * E - hess_times(H, Es[sel]) - qs[sel, None] * Epsi
    if targets is not None:
        return qbar_s, xbar_s
    qbar = np.empty(P.n)
    xbar = np.empty((P.n, 3))
    qbar[perm] = qbar_s
    xbar[perm] = xbar_s
    return qbar, xbar
