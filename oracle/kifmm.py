"""Plain FP64 periodic kernel-independent FMM (the oracle's second tier).

This follows Algorithm 2 of the paper (Section 2, near/far split with a
precomputed periodic M2L operator), with its step d folded into the tree's
downward pass as the paper suggests at the end of that algorithm's
discussion:

  Stage 1 (operators, unit box, scaled by 2^l at level l since the kernels
  are homogeneous of degree -1):
    * upward / downward check-to-equivalent solves from the SVD A = U S V^T,
      applied as (V S_eps^+)(U^T q) (Appendix B, the backward-stable solver),
      with S_eps^+ dropping singular values at or below 1e-11 * s_max (the
      paper leaves this cutoff free).  Directions with smaller singular values
      carry no information that survives the rounding of the check potentials
      (sums with cancellation, tens of ulps): kept, they turn that rounding into
      equivalent-density noise (two SVD drivers, or two summation orders, then
      disagree at 1e-9 for Stokes at p = 8) and cost accuracy against the exact
      periodic sums (Stokes TP p = 8: 1.9e-5 with Table 1's rank criterion
      eps * s_max * dim(A), 5.2e-6 with 1e-11);
    * M2M, L2L for the eight octants and M2L for the 316 offsets in
      [-3,3]^3 \\ [-1,1]^3, from the free-space kernel between surfaces;
    * the periodic root operator M_root = K^{P,F}(x^{B0,d}, y^{B0,u}) over
      images with |p|_inf >= 2 (Eq. M2Lsolve's right-hand side).
  Stage 2 (evaluation):
    a. S2M at leaves, then M2M and upward solves up to the root density
       phi^{B0,u} (Algorithm 2, steps a and b);
    b. q^{B0,d} = M_root phi^{B0,u}  (step c, folded: the root's downward
       check potential rather than a separate far-field loop at targets);
    c. V-list M2L and X-list S2L into downward check potentials, L2L and the
       downward solves from the root to the leaves;
    d. at leaves: L2T from phi^{B,d}, W-list M2T from phi^{A,u} and the
       U-list direct sums over adjacent leaves and their periodic images.
  A W-list box that is a leaf with no more points than a surface has acts on
  the targets directly (its points instead of its upward surface), and a leaf
  with no more points than a surface has takes its X list directly (the
  sources straight to its points instead of through its downward surface):
  the cheaper form of the same interaction, and exact.

Every direct sum goes through the oracle's plain C loop; every dense
operator product is a numpy matmul.  Test infrastructure only.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np

from . import tree as otree
from . import periodic
from ._native import direct
from .kernels import (LAPLACE, STOKES, INNER, OUTER, kdim, unit_surface, kernel_matrix)

EPS = np.finfo(np.float64).eps


@dataclass
class Pinv:
    Ut: np.ndarray      # [r, kn]
    VS: np.ndarray      # [kn, r]

    def apply(self, q: np.ndarray) -> np.ndarray:
        """(V S^+)(U^T q) -- the backward-stable order of Appendix B."""
        return self.VS @ (self.Ut @ q)


DEFAULT_CUTOFF = 1e-11


def rank_threshold(A: np.ndarray) -> float:
    """Relative singular-value cutoff eps * dim(A): the rank criterion of Table 1."""
    return EPS * max(A.shape)


def pinv_factors(A: np.ndarray, rel_threshold: Optional[float] = None) -> Pinv:
    U, s, Vt = np.linalg.svd(A)
    thr = DEFAULT_CUTOFF if rel_threshold is None else rel_threshold
    keep = s > thr * s[0]
    return Pinv(Ut=U[:, keep].T.copy(), VS=(Vt[keep].T / s[keep][None, :]).copy())


def octant_offset(o: int) -> np.ndarray:
    return np.array([((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5]) * 0.5


M2L_OFFSETS = [d for d in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in d) >= 2]


class Operators:
    """Unit-box operators for one (kernel, periodicity, p)."""

    def __init__(self, kernel: int, mask: int, p: int, rel_threshold: Optional[float] = None,
                 near_layers: int = 1):
        self.kernel, self.mask, self.p = kernel, mask, p
        self.k = kdim(kernel)
        u = unit_surface(p)
        self.n = u.shape[0]
        self.inner = 0.5 * INNER * u      # unit box centred at 0
        self.outer = 0.5 * OUTER * u
        K = lambda X, Y: kernel_matrix(kernel, X, Y)
        self.up = pinv_factors(K(self.outer, self.inner), rel_threshold)
        self.down = pinv_factors(K(self.inner, self.outer), rel_threshold)
        self.m2m = [K(self.outer, octant_offset(o) + 0.5 * self.inner) for o in range(8)]
        self.l2l = [K(octant_offset(o) + 0.5 * self.inner, self.outer) for o in range(8)]
        self._m2l: Dict[tuple, np.ndarray] = {}
        self.mroot = periodic.far_kernel_matrix(kernel, mask, self.inner + 0.5, self.inner + 0.5,
                                                near_layers=near_layers)

    def m2l(self, delta) -> np.ndarray:
        delta = tuple(int(c) for c in delta)
        if delta not in self._m2l:
            self._m2l[delta] = kernel_matrix(self.kernel, self.inner,
                                             np.array(delta, dtype=np.float64) + self.inner)
        return self._m2l[delta]


_OPS_CACHE: Dict[tuple, Operators] = {}


def operators(kernel: int, mask: int, p: int, rel_threshold: Optional[float] = None,
              near_layers: int = 1) -> Operators:
    key = (kernel, mask, p, rel_threshold, near_layers)
    if key not in _OPS_CACHE:
        _OPS_CACHE[key] = Operators(kernel, mask, p, rel_threshold, near_layers)
    return _OPS_CACHE[key]


class KIFMM:
    """One problem: tree, lists and the evaluation pass."""

    def __init__(self, kernel: int, mask: int, p: int, s: int, points: np.ndarray,
                 rel_threshold: Optional[float] = None, box_length: float = 1.0,
                 targets: Optional[np.ndarray] = None, near_layers: int = 1):
        """points: the sources (also the targets unless `targets` is given).  With separate
        targets (Section 2's problem: T targets, S sources) the tree is built over the union of
        both sets, points [0, S) being the sources and [S, S + T) the targets; a target-only point
        carries zero density, so it adds nothing to any sum, and evaluate returns the potentials
        at the targets alone."""
        if not periodic.supported(kernel, mask):
            raise NotImplementedError("unsupported kernel/periodicity")
        self.kernel, self.mask, self.p, self.s = kernel, mask, p, s
        self.k = kdim(kernel)
        self.L = float(box_length)
        pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
        self.n_src = pts.shape[0]
        self.n_trg = 0
        self.separate = targets is not None
        if self.separate:
            trg = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
            self.n_trg = trg.shape[0]
            pts = np.concatenate([pts, trg])
        self.u = otree.wrap(pts / self.L, mask)
        self.tree = otree.build_tree(self.u, s)
        self.lists = otree.build_lists(self.tree, mask, near_layers)
        self.ops = operators(kernel, mask, p, rel_threshold, near_layers)
        self.sorted_pts = self.u[self.tree.perm]

    # -- W/X lists: the cheaper of the surface operator and the direct sum
    def direct_source(self, a) -> bool:
        """A W-list box whose points are fewer than its surface points acts directly."""
        t = self.tree
        return t.is_leaf(a) and (t.end[a] - t.begin[a]) <= self.ops.n

    def direct_target(self, b) -> bool:
        """A leaf with fewer points than surface points takes its X list directly."""
        t = self.tree
        return t.is_leaf(b) and (t.end[b] - t.begin[b]) <= self.ops.n

    # -- geometry helpers
    def _pts(self, b, shift=(0, 0, 0)):
        t = self.tree
        return self.sorted_pts[t.begin[b]:t.end[b]] + np.asarray(shift, dtype=np.float64)

    def _surf(self, b, factor, shift=(0, 0, 0)):
        t = self.tree
        return t.centre(b) + np.asarray(shift, dtype=np.float64) + 0.5 * factor * t.edge(b) * unit_surface(self.p)

    # -- the two surface-form interactions of the adaptive lists (Section 2.2: a W-list box acts
    #    through its upward equivalent density, an X-list leaf's points act on the target box's
    #    downward check surface)
    def m2t(self, x, a, p, phi_u, pot):
        """W list: box a's upward equivalent density, on its inner (equivalent) surface moved by
        the image shift p, evaluated at the points x (added to pot)."""
        direct(self.kernel, x, self._surf(a, INNER, p), phi_u[a], pot)

    def s2l(self, b, a, p, ds, q):
        """X list: the points of leaf a moved by the image shift p, evaluated on box b's inner
        (downward check) surface (added to q)."""
        t = self.tree
        direct(self.kernel, self._surf(b, INNER), self._pts(a, p), ds[t.begin[a]:t.end[a]], q)

    def tp_laplace_background(self, ds, phi_root) -> float:
        """The part of the triply periodic Laplace far field that the root's equivalent density
        cannot carry (0 for every other kernel and periodicity).

        The Ewald kernel with its k = 0 mode removed (the zero-mean sum, which includes the
        uniform neutralising background of Section 5's one-component-plasma remark) satisfies
        laplacian G = 1/V away from the lattice points.  So, as a function of the source
        position y near the box, the far kernel is a harmonic function plus |y - c|^2 / 6
        (V = 1, c the box centre).  The equivalent density reproduces the sources' action on
        harmonic functions (Section 2.2) but not on |y - c|^2, the one moment that a harmonic
        field never sees; the far field M_root phi^{B0,u} therefore misses the constant
        (sum_s q_s |y_s - c|^2 - sum_j phi_j |y_j - c|^2) / 6, added here to every target.
        Its form does not depend on c for neutral densities (the sums of q and phi, and their
        dipoles, agree)."""
        if self.kernel != LAPLACE or self.mask != 7:
            return 0.0
        c = np.full(3, 0.5)
        ys = self.sorted_pts
        yj = self.tree.centre(0) + 0.5 * INNER * self.tree.edge(0) * unit_surface(self.p)
        m_src = float(np.sum(ds[:, 0] * np.sum((ys - c) ** 2, axis=1)))
        m_eq = float(np.sum(phi_root * np.sum((yj - c) ** 2, axis=1)))
        return (m_src - m_eq) / 6.0

    def upward(self, dens_sorted: np.ndarray) -> np.ndarray:
        """phi^{B,u} for every box (dens_sorted: [N, k] in Morton order), level by level."""
        t, ops, k = self.tree, self.ops, self.k
        kn = k * ops.n
        phi_u = np.zeros((t.nbox, kn))
        for lv in range(t.depth(), -1, -1):
            boxes = [b for b in range(t.nbox) if t.level[b] == lv]
            h = 0.5 ** lv
            Q = np.zeros((len(boxes), kn))
            for i, b in enumerate(boxes):
                if t.is_leaf(b):
                    direct(self.kernel, self._surf(b, OUTER), self._pts(b), dens_sorted[t.begin[b]:t.end[b]], Q[i])
            for o in range(8):
                rows = [i for i, b in enumerate(boxes) if t.children[b][o] >= 0]
                if rows:
                    ch = [t.children[boxes[i]][o] for i in rows]
                    Q[rows] += (ops.m2m[o] @ phi_u[ch].T).T / h
            phi_u[boxes] = h * ops.up.apply(Q.T).T
        return phi_u

    def evaluate(self, density: np.ndarray, target_leaves: Optional[Sequence[int]] = None,
                 return_sorted: bool = False, step_d: bool = False):
        """Potentials at all points (input order), or at the points of the given leaves.

        density: [N, k] (or [N] for Laplace) in input order, N the number of sources.
        With separate targets the result holds the targets' potentials, in target order.
        With target_leaves, returns {leaf: potentials [count, k] in Morton order} (every point of
        the leaf, sources included);
        only the downward pass along those leaves' ancestors is computed.

        The far field of the images beyond the first layer enters as the root's downward check
        potential M_root phi^{B0,u} (Section 3.3, Eqs. for q^{F} through the root's upward
        density).  By default it is added to the root's check potential and reaches the targets
        through L2L and each leaf's L2T.  With step_d, it is solved into its own downward
        equivalent density on the root's surface, phi^{B0,d} = T_M2L phi^{B0,u} (Section 3.4),
        which is evaluated at every target directly (Algorithm 2, step d); the tree's root
        then carries no far field.  The two agree to the FMM's truncation accuracy.
        """
        t, ops, k, L = self.tree, self.ops, self.k, self.L
        dens = np.asarray(density, dtype=np.float64).reshape(-1, k)
        if self.separate:
            dens = np.concatenate([dens, np.zeros((self.n_trg, k))])
        ds = np.ascontiguousarray(dens[t.perm])
        phi_u = self.upward(ds)
        kn = k * ops.n
        leaves = t.leaves() if target_leaves is None else list(target_leaves)
        need = set()
        for b in leaves:
            while b >= 0 and b not in need:
                need.add(b)
                b = t.parent[b]
        # V-list M2L (grouped by offset) and X-list S2L into downward check potentials
        qd = {b: np.zeros(kn) for b in need}
        groups: Dict[tuple, list] = {}
        for b in need:
            cb = np.array(t.coord[b])
            for (a, p) in self.lists.V.get(b, []):   # the root's: its image ring (near_layers > 1)
                delta = tuple(int(c) for c in np.array(t.coord[a]) + np.array(p) * (1 << t.level[b]) - cb)
                groups.setdefault(delta, []).append((b, a))
        for delta, pairs in groups.items():
            tb = [b for b, _ in pairs]
            src = [a for _, a in pairs]
            scale = np.array([1.0 / t.edge(b) for b in tb])
            contrib = (ops.m2l(delta) @ phi_u[src].T).T * scale[:, None]
            for i, b in enumerate(tb):
                qd[b] += contrib[i]
        for b in need:
            if self.direct_target(b):
                continue                     # its X-list sources go straight to its points below
            for (a, p) in self.lists.X[b]:
                self.s2l(b, a, p, ds, qd[b])
        # root far field (folded step c), L2L and downward solves
        phi_d = {}
        for b in sorted(need, key=lambda b: t.level[b]):
            h = t.edge(b)
            q = qd[b]
            if b == 0:
                if not step_d:
                    q = q + ops.mroot @ phi_u[0]
            else:
                par = t.parent[b]
                o = t.children[par].index(b)
                q = q + ops.l2l[o] @ phi_d[par] / t.edge(par)
            phi_d[b] = h * ops.down.apply(q)
        phi_far = t.edge(0) * ops.down.apply(ops.mroot @ phi_u[0]) if step_d else None
        background = self.tp_laplace_background(ds, phi_u[0])
        out = {}
        for b in leaves:
            x = self._pts(b)
            pot = np.zeros((x.shape[0], k))
            direct(self.kernel, x, self._surf(b, OUTER), phi_d[b], pot)
            if step_d:
                direct(self.kernel, x, self._surf(0, OUTER), phi_far, pot)
            for (a, p) in self.lists.W[b]:
                if self.direct_source(a):
                    direct(self.kernel, x, self._pts(a), ds[t.begin[a]:t.end[a]], pot, shift=p)
                else:
                    self.m2t(x, a, p, phi_u, pot)
            if self.direct_target(b):
                for (a, p) in self.lists.X[b]:
                    direct(self.kernel, x, self._pts(a), ds[t.begin[a]:t.end[a]], pot, shift=p)
            for (a, p) in self.lists.U[b]:
                direct(self.kernel, x, self._pts(a), ds[t.begin[a]:t.end[a]], pot, shift=p)
            out[b] = (pot + background) / L
        if target_leaves is not None:
            return out
        res = np.zeros((t.end[0], k))
        for b, pot in out.items():
            res[t.begin[b]:t.end[b]] = pot
        if return_sorted:
            return res
        full = np.zeros_like(res)
        full[t.perm] = res
        return full[self.n_src:] if self.separate else full


def evaluate(kernel: int, mask: int, p: int, s: int, points: np.ndarray, density: np.ndarray,
             rel_threshold: Optional[float] = None, step_d: bool = False) -> np.ndarray:
    """Convenience wrapper: [R, N, k] densities -> [R, N, k] potentials."""
    f = KIFMM(kernel, mask, p, s, points, rel_threshold)
    dens = np.asarray(density, dtype=np.float64)
    if dens.ndim == 2:
        dens = dens[None]
    return np.stack([f.evaluate(d, step_d=step_d) for d in dens])
