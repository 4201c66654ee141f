"""Root cube, Morton keys, octree and interaction lists -- TEST INFRASTRUCTURE ONLY.

Section 2.2, first step: an octree whose leaves hold at most M points.  The
paper fixes nothing else about the tree, so the following readings are used
(each is restated in the design notes):

* Root cube: explicit (lo, s) with s a power of two, or automatic:
  s = 2^ceil(log2(extent (1 + 2^-10))), lo = floor(min 2^12 / s) s / 2^12.
* Keys: 21 bits per axis, k_d = clamp(floor((x_d - lo_d) 2^21 / s), 0, 2^21-1)
  in FP64; Morton bit 3b+2 = x bit b, 3b+1 = y bit b, 3b = z bit b.
* Order: stable sort by key (ties keep the input order).
* Boxes exist when non-empty and their parent is not a leaf.  Adaptive tree:
  a box is a leaf when it holds <= M points or sits at max_depth.  Uniform
  tree: every box at depth L_u = min(max_depth, min{L : M 8^L >= N}) is a leaf.
* Box numbering: level by level, Morton order inside a level.
* Lists (near and far zones of Section 2.2, in the usual KIFMM form), with
  adjacency = closed cubes that touch or overlap:
    U(B), leaf B: leaves adjacent to B (B included);
    V(B), level >= 2: children of the colleagues of parent(B) not adjacent to B;
    W(B), leaf B: descendants A of B's colleagues with A not adjacent to B and
          parent(A) adjacent to B;
    X(B) = {A : B in W(A)}.
  A colleague is a box of the same level adjacent to it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BITS = 21
NCELL = 1 << BITS


def root_box(x: np.ndarray, explicit=None):
    """Return (lo[3], s) for the root cube; raises ValueError for a bad input."""
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite position")
    if explicit is not None:
        lo = np.asarray(explicit[0], dtype=np.float64).reshape(3)
        s = float(explicit[1])
        m, _ = math.frexp(s)
        if not (s > 0 and m == 0.5):
            raise ValueError("root side must be a power of two")
        g = lo * 4096.0 / s
        if not np.all(g == np.floor(g)):
            raise ValueError("root corner must lie on the side/4096 grid")
        if x.size and (np.any(x < lo) or np.any(x > lo + s)):
            raise ValueError("point outside the explicit root")
        return lo, s
    mn = x.min(axis=0)
    mx = x.max(axis=0)
    ext = float(np.max(mx - mn))
    if ext == 0.0:
        s = 1.0
    else:
        t = ext * (1.0 + 2.0 ** -10)
        m, e = math.frexp(t)                 # t = m 2^e, 0.5 <= m < 1
        s = 2.0 ** (e - 1) if m == 0.5 else 2.0 ** e
    lo = np.floor(mn * 4096.0 / s) * s / 4096.0
    return lo, s


def quantise(x: np.ndarray, lo, s) -> np.ndarray:
    k = np.floor((np.asarray(x, dtype=np.float64) - lo) * (float(NCELL) / s))
    return np.clip(k, 0, NCELL - 1).astype(np.int64)


def morton(k: np.ndarray) -> np.ndarray:
    """Interleave per-axis integer coordinates [.,3] into 63-bit keys."""
    k = np.asarray(k, dtype=np.uint64)
    key = np.zeros(k.shape[0], dtype=np.uint64)
    for b in range(BITS):
        sh = np.uint64(b)
        one = np.uint64(1)
        key |= ((k[:, 0] >> sh) & one) << np.uint64(3 * b + 2)
        key |= ((k[:, 1] >> sh) & one) << np.uint64(3 * b + 1)
        key |= ((k[:, 2] >> sh) & one) << np.uint64(3 * b)
    return key


def uniform_depth(n: int, leaf_size: int, max_depth: int) -> int:
    L = 0
    while leaf_size * 8 ** L < n:
        L += 1
    return min(max_depth, L)


@dataclasses.dataclass
class Tree:
    lo: np.ndarray
    s: float
    keys: np.ndarray          # sorted 63-bit keys [N] uint64
    perm: np.ndarray          # sorted position -> input index [N]
    level: np.ndarray         # [B]
    anchor: np.ndarray        # [B,3] integer cell of the box at its level
    begin: np.ndarray         # [B] first sorted point
    end: np.ndarray           # [B] one past the last sorted point
    parent: np.ndarray        # [B] (-1 for the root)
    children: np.ndarray      # [B,8] by octant (x bit <<2 | y bit <<1 | z bit), -1 if absent
    is_leaf: np.ndarray       # [B] bool
    level_start: np.ndarray   # [depth+2] first box of each level

    @property
    def nboxes(self) -> int:
        return int(self.level.shape[0])

    @property
    def depth(self) -> int:
        return int(self.level.max())

    def width(self, l: int) -> float:
        return self.s / (1 << l)

    def center(self, b: int) -> np.ndarray:
        w = self.width(int(self.level[b]))
        return self.lo + (self.anchor[b] + 0.5) * w

    def leaves(self) -> np.ndarray:
        return np.nonzero(self.is_leaf)[0]


def build_tree(x: np.ndarray, leaf_size: int, adaptive: bool = True, max_depth: int = BITS,
               root=None) -> Tree:
    if leaf_size < 1 or not (0 <= max_depth <= BITS):
        raise ValueError("bad leaf size or depth")
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    lo, s = root_box(x, root)
    keys = morton(quantise(x, lo, s))
    perm = np.argsort(keys, kind="stable")
    keys = keys[perm]
    Lu = uniform_depth(n, leaf_size, max_depth)

    def prefix(d, b0, b1):
        return keys[b0:b1] >> np.uint64(3 * (BITS - d))

    level, anchor, begin, end, parent, is_leaf = [], [], [], [], [], []
    level_start = [0]
    # level 0: the root
    cur = [(np.zeros(3, dtype=np.int64), 0, n, -1)]
    d = 0
    while cur:
        next_level = []
        for (a, b0, b1, par) in cur:
            idx = len(level)
            cnt = b1 - b0
            if adaptive:
                leaf = cnt <= leaf_size or d == max_depth
            else:
                leaf = d == Lu
            level.append(d)
            anchor.append(a)
            begin.append(b0)
            end.append(b1)
            parent.append(par)
            is_leaf.append(leaf)
            if not leaf:
                pre = prefix(d + 1, b0, b1)
                starts = np.concatenate([[0], np.nonzero(pre[1:] != pre[:-1])[0] + 1, [cnt]])
                for t in range(len(starts) - 1):
                    c0, c1 = b0 + int(starts[t]), b0 + int(starts[t + 1])
                    o = int(pre[starts[t]] & np.uint64(7))
                    ca = 2 * a + np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1], dtype=np.int64)
                    next_level.append((ca, c0, c1, idx))
        level_start.append(len(level))
        cur = next_level
        d += 1
    B = len(level)
    level = np.array(level, dtype=np.int64)
    anchor = np.array(anchor, dtype=np.int64).reshape(B, 3)
    parent = np.array(parent, dtype=np.int64)
    children = -np.ones((B, 8), dtype=np.int64)
    for b in range(1, B):
        o = int(((anchor[b, 0] & 1) << 2) | ((anchor[b, 1] & 1) << 1) | (anchor[b, 2] & 1))
        children[parent[b], o] = b
    return Tree(lo, s, keys, perm, level, anchor, np.array(begin, dtype=np.int64),
                np.array(end, dtype=np.int64), parent, children,
                np.array(is_leaf, dtype=bool), np.array(level_start, dtype=np.int64))


# ----------------------------------------------------------------------------
# interaction lists

def _extent(tree: Tree, b: int):
    sh = BITS - int(tree.level[b])
    lo = tree.anchor[b] << sh
    return lo, lo + (1 << sh)


def adjacent(tree: Tree, a: int, b: int) -> bool:
    """Closed cubes of boxes a and b touch or overlap (finest-grid integers)."""
    la, ha = _extent(tree, a)
    lb, hb = _extent(tree, b)
    return bool(np.all(la <= hb) and np.all(lb <= ha))


def v_offset_index(d) -> int:
    """Index 0..315 of an offset d in [-3,3]^3 minus [-1,1]^3, lexicographic (dx,dy,dz)."""
    k = 0
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            for dz in range(-3, 4):
                if max(abs(dx), abs(dy), abs(dz)) <= 1:
                    continue
                if (dx, dy, dz) == tuple(int(v) for v in d):
                    return k
                k += 1
    raise ValueError("not a far offset")


# A list entry names a box and, with periodic images, which image of it:
# entry = box + code << SHIFT_BITS, the image shift s in {-1,0,1}^3 (in root
# widths) coded as code = (9 (sx+1) + 3 (sy+1) + (sz+1) + 14) mod 27, so that
# the unshifted image has code 0 and free-space lists are plain box indices.
SHIFT_BITS = 26


def encode(box: int, s) -> int:
    raw = 9 * (int(s[0]) + 1) + 3 * (int(s[1]) + 1) + (int(s[2]) + 1)
    return int(box) + (((raw + 14) % 27) << SHIFT_BITS)


def decode(e: int):
    """(box, shift as an int array of 3) of a list entry."""
    e = int(e)
    raw = ((e >> SHIFT_BITS) + 13) % 27
    return e & ((1 << SHIFT_BITS) - 1), np.array([raw // 9 - 1, (raw // 3) % 3 - 1, raw % 3 - 1], dtype=np.int64)


@dataclasses.dataclass
class Lists:
    U: List[list]          # per box (empty unless leaf)
    V: List[list]
    W: List[list]
    X: List[list]

    def csr(self, name):
        rows = getattr(self, name)
        off = np.zeros(len(rows) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(r) for r in rows])
        idx = np.array([a for r in rows for a in r], dtype=np.int64)
        return off, idx


def build_lists(tree: Tree, periodic: bool = False) -> Lists:
    """U, V, W, X of every box.  With ``periodic`` the root cube tiles space:
    neighbours wrap around at every level and each entry carries the image
    shift of its box (Section 2.4 allows periodic boundaries)."""
    B = tree.nboxes
    lookup = {}
    for b in range(B):
        lookup[(int(tree.level[b]),) + tuple(int(v) for v in tree.anchor[b])] = b
    # closed finest-grid extents of every box as plain ints (same test as adjacent())
    sh = (BITS - tree.level)[:, None]
    lo_all = (tree.anchor << sh).tolist()
    hi_all = ((tree.anchor << sh) + (1 << sh)).tolist()
    ext = [(l[0], l[1], l[2], h[0], h[1], h[2]) for l, h in zip(lo_all, hi_all)]

    def adj(a, sa, b):
        """Image sa of box a touches box b (unshifted)."""
        ea, eb = ext[a], ext[b]
        o = [int(v) * NCELL for v in sa]
        return (ea[0] + o[0] <= eb[3] and eb[0] <= ea[3] + o[0] and ea[1] + o[1] <= eb[4]
                and eb[1] <= ea[4] + o[1] and ea[2] + o[2] <= eb[5] and eb[2] <= ea[5] + o[2])

    def colleagues(b):
        """(box, image shift) of the same-level boxes touching b, b included."""
        l = int(tree.level[b])
        a = tree.anchor[b]
        lim = 1 << l
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    g = [int(a[0]) + dx, int(a[1]) + dy, int(a[2]) + dz]
                    s = [0, 0, 0]
                    if periodic:
                        s = [v // lim for v in g]        # floor division: -1, 0 or 1
                        g = [v % lim for v in g]
                    c = lookup.get((l, g[0], g[1], g[2]))
                    if c is not None:
                        out.append((c, tuple(s)))
        return out

    U = [[] for _ in range(B)]
    V = [[] for _ in range(B)]
    W = [[] for _ in range(B)]
    X = [[] for _ in range(B)]
    coll = [colleagues(b) for b in range(B)]

    for b in range(B):
        l = int(tree.level[b])
        if l >= 1:
            p = int(tree.parent[b])
            for c, sc in coll[p]:
                for ch in tree.children[c]:
                    if ch >= 0 and not adj(int(ch), sc, b):
                        V[b].append(encode(int(ch), sc))
        if not tree.is_leaf[b]:
            continue
        # same-level and finer adjacent leaves, and W, by descending the colleagues
        u, w = set(), set()

        def descend(a, sa):
            for ch in tree.children[a]:
                if ch < 0:
                    continue
                ch = int(ch)
                if adj(ch, sa, b):
                    if tree.is_leaf[ch]:
                        u.add(encode(ch, sa))
                    else:
                        descend(ch, sa)
                else:
                    w.add(encode(ch, sa))

        for c, sc in coll[b]:
            if tree.is_leaf[c]:
                u.add(encode(c, sc))
            else:
                descend(c, sc)
        # coarser adjacent leaves are colleagues of an ancestor
        a = int(tree.parent[b])
        while a >= 0:
            for c, sc in coll[a]:
                if tree.is_leaf[c] and adj(c, sc, b):
                    u.add(encode(c, sc))
            a = int(tree.parent[a])
        U[b] = sorted(u)
        W[b] = sorted(w)
    for b in range(B):
        for e in W[b]:
            a, sa = decode(e)
            X[a].append(encode(b, -sa))
    for b in range(B):
        V[b].sort()
        X[b].sort()
    return Lists(U, V, W, X)
