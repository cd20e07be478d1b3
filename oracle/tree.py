"""Adaptive octree and periodic interaction lists (oracle, plain Python).

Tree (Section 2, notation table: at most s points per leaf):
  * periodic coordinates are wrapped into [0, 1) (a wrapped value of exactly
    1.0 becomes 0.0); non-periodic coordinates must lie in the closed [0, 1];
  * each coordinate is quantised to 21 bits, k = min(floor(u * 2^21), 2^21 - 1),
    which is exact in float64;
  * the three 21-bit integers are bit-interleaved into a 63-bit Morton key
    (x bit above y bit above z bit at every level);
  * points are stably sorted by (key, input index);
  * a box is split into its non-empty octants while it holds more than s
    points (depth capped at 21).
Boxes are numbered level by level, in Morton order within a level.

Lists (Section 2: near field of a box = same-level adjacent boxes; the
adaptive U, V, W, X lists of kernel-independent FMM).  Adjacency is evaluated
with periodic wrap on periodic axes, and every list entry carries the image
shift p in {-1, 0, 1}^3 (source box translated by +p).  The near field of the
original box is therefore the images with |p|_inf <= 1; everything beyond is
the far field handled at the root.
  * colleagues(B): same-level boxes A with A + p adjacent to B (B itself included);
  * U(B), B leaf: every leaf A with A + p adjacent to B;
  * V(B): children of the colleagues of parent(B) that are not adjacent to B;
  * W(B), B leaf: descendants A of colleagues of B with parent(A) + p adjacent
    to B and A + p not adjacent to B;
  * X(B): every (A, p) with (B, -p) in W(A).
The root gets no V list (its far field is the periodic operator).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

MAXLEVEL = 21
QSCALE = float(1 << MAXLEVEL)


class OutOfBox(ValueError):
    pass


def wrap(points: np.ndarray, periodic_mask: int) -> np.ndarray:
    """Wrap periodic axes into [0, 1); check the others lie in [0, 1]."""
    u = np.array(points, dtype=np.float64, copy=True)
    if not np.all(np.isfinite(u)):
        raise OutOfBox("non-finite coordinate")
    for a in range(3):
        if periodic_mask & (1 << a):
            w = u[:, a] - np.floor(u[:, a])
            w[w >= 1.0] = 0.0
            u[:, a] = w
        else:
            if np.any(u[:, a] < 0.0) or np.any(u[:, a] > 1.0):
                raise OutOfBox("coordinate outside [0,1] on a non-periodic axis")
    return u


def quantise(u: np.ndarray) -> np.ndarray:
    q = np.floor(u * QSCALE).astype(np.int64)
    return np.minimum(q, (1 << MAXLEVEL) - 1)


def interleave(q: np.ndarray) -> np.ndarray:
    """63-bit Morton keys from [N, 3] 21-bit integers (x highest at each level)."""
    key = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(MAXLEVEL):
        for a in range(3):
            bit = (q[:, a].astype(np.uint64) >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + (2 - a))
    return key


@dataclass
class Tree:
    perm: np.ndarray          # sorted position -> input index
    keys: np.ndarray          # sorted Morton keys
    level: List[int] = field(default_factory=list)
    coord: List[Tuple[int, int, int]] = field(default_factory=list)
    begin: List[int] = field(default_factory=list)
    end: List[int] = field(default_factory=list)
    parent: List[int] = field(default_factory=list)
    children: List[List[int]] = field(default_factory=list)   # 8 entries, -1 if absent

    @property
    def nbox(self) -> int:
        return len(self.level)

    def is_leaf(self, b: int) -> bool:
        return all(c < 0 for c in self.children[b])

    def centre(self, b: int) -> np.ndarray:
        h = 0.5 ** self.level[b]
        return (np.array(self.coord[b], dtype=np.float64) + 0.5) * h

    def edge(self, b: int) -> float:
        return 0.5 ** self.level[b]

    def leaves(self) -> List[int]:
        return [b for b in range(self.nbox) if self.is_leaf(b)]

    def depth(self) -> int:
        return max(self.level)


def build_tree(u: np.ndarray, s: int) -> Tree:
    """Sort by (Morton key, input index) and split boxes holding more than s points."""
    if s < 1:
        raise ValueError("s must be positive")
    keys = interleave(quantise(u))
    perm = np.argsort(keys, kind="stable")
    skeys = keys[perm]
    t = Tree(perm=perm, keys=skeys)
    t.level.append(0); t.coord.append((0, 0, 0)); t.begin.append(0); t.end.append(len(skeys))
    t.parent.append(-1); t.children.append([-1] * 8)
    frontier = [0]
    lvl = 0
    while frontier and lvl < MAXLEVEL:
        nxt = []
        for b in frontier:
            if t.end[b] - t.begin[b] <= s:
                continue
            cx, cy, cz = t.coord[b]
            for o in range(8):
                ox, oy, oz = (o >> 2) & 1, (o >> 1) & 1, o & 1
                child = (2 * cx + ox, 2 * cy + oy, 2 * cz + oz)
                prefix = (int(interleave(np.array([child], dtype=np.int64))[0]))
                sh = 3 * (MAXLEVEL - (lvl + 1))
                # prefix above was built from level-(lvl+1) integers placed in the low bits;
                lo = np.uint64(prefix << sh)
                hi = np.uint64(((prefix + 1) << sh) - 1)
                i0 = int(np.searchsorted(skeys, lo, side="left"))
                i1 = int(np.searchsorted(skeys, hi, side="right"))
                if i1 <= i0:
                    continue
                c = t.nbox
                t.level.append(lvl + 1); t.coord.append(child); t.begin.append(i0); t.end.append(i1)
                t.parent.append(b); t.children.append([-1] * 8)
                t.children[b][o] = c
                nxt.append(c)
        frontier = nxt
        lvl += 1
    return t


def _adjacent(la, a, p, lb, b) -> bool:
    """Closed boxes A + p (level la, integer coords a) and B (level lb, coords b) touch or overlap."""
    m = max(la, lb)
    sa, sb = 1 << (m - la), 1 << (m - lb)
    per = 1 << m
    for c in range(3):
        alo = a[c] * sa + p[c] * per
        ahi = alo + sa
        blo = b[c] * sb
        bhi = blo + sb
        if alo > bhi or blo > ahi:
            return False
    return True


@dataclass
class Lists:
    U: Dict[int, List[Tuple[int, Tuple[int, int, int]]]]
    V: Dict[int, List[Tuple[int, Tuple[int, int, int]]]]
    W: Dict[int, List[Tuple[int, Tuple[int, int, int]]]]
    X: Dict[int, List[Tuple[int, Tuple[int, int, int]]]]


def build_lists(t: Tree, periodic_mask: int, near_layers: int = 1) -> Lists:
    """The adaptive lists.  With near_layers l > 1 (Section 3.6: the near field spans l layers of
    images) the root also gets a V list: its own images with 2 <= |p|_inf <= l along the periodic
    axes, which act on it through its upward equivalent density."""
    lookup = {(t.level[b],) + tuple(t.coord[b]): b for b in range(t.nbox)}

    def adj(a, p, b):
        return _adjacent(t.level[a], t.coord[a], p, t.level[b], t.coord[b])

    def colleagues(b):
        lv = t.level[b]
        n = 1 << lv
        out = []
        for off in itertools.product((-1, 0, 1), repeat=3):
            g = [t.coord[b][c] + off[c] for c in range(3)]
            shift = [0, 0, 0]
            ok = True
            for c in range(3):
                if 0 <= g[c] < n:
                    continue
                if periodic_mask & (1 << c):
                    shift[c] = g[c] // n
                    g[c] -= shift[c] * n
                else:
                    ok = False
            if not ok:
                continue
            a = lookup.get((lv, g[0], g[1], g[2]))
            if a is not None:
                out.append((a, tuple(shift)))
        return out

    coll = [colleagues(b) for b in range(t.nbox)]
    U, V, W, X = {}, {}, {}, {}
    for b in range(t.nbox):
        if t.level[b] >= 1:
            vl = []
            for (pa, p) in coll[t.parent[b]]:
                for a in t.children[pa]:
                    if a >= 0 and not adj(a, p, b):
                        vl.append((a, p))
            V[b] = sorted(vl)
        if t.is_leaf(b):
            ul, wl = [], []
            # same level and finer: descend through adjacent non-leaf colleagues
            stack = list(coll[b])
            while stack:
                a, p = stack.pop()
                if t.is_leaf(a):
                    ul.append((a, p))
                    continue
                for c in t.children[a]:
                    if c < 0:
                        continue
                    if adj(c, p, b):
                        stack.append((c, p))
                    else:
                        wl.append((c, p))
            # coarser leaves: colleagues of ancestors that are leaves and adjacent to b
            anc = t.parent[b]
            while anc >= 0:
                for (a, p) in coll[anc]:
                    if t.is_leaf(a) and adj(a, p, b):
                        ul.append((a, p))
                anc = t.parent[anc]
            U[b] = sorted(set(ul))
            W[b] = sorted(set(wl))
    for b in range(t.nbox):
        X[b] = []
    for a, wl in W.items():
        for (b, p) in wl:
            X[b].append((a, (-p[0], -p[1], -p[2])))
    for b in X:
        X[b] = sorted(X[b])
    if near_layers > 1 and periodic_mask:
        rng = [range(-near_layers, near_layers + 1) if periodic_mask & (1 << c) else (0,) for c in range(3)]
        V[0] = sorted((0, p) for p in itertools.product(*rng) if max(abs(c) for c in p) >= 2)
    return Lists(U=U, V=V, W=W, X=X)
