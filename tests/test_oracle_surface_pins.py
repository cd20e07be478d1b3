"""Pins of the oracle's surface-form W and X interactions and of its triply periodic Laplace sum.

The adaptive lists' W (a box acting on a leaf's points through its upward equivalent surface) and
X (a leaf's points acting on a box's downward check surface) take their surface form only when a
leaf holds more points than a surface (otherwise the exact direct form is cheaper and taken).  With
s above the surface size n(p) and strongly graded points, many W and X entries take the surface
form; the oracle is checked against the definitions (free-space direct sums, SP/DP lattice sums,
TP Ewald sums) at the KIFMM error of that p, and each plausible mistake in those two interactions
is planted in a subclass, on the CPU, to show that the same check fails."""
import numpy as np
import pytest

import workloads as W
from oracle import kifmm, kernels as K, periodic
from oracle._native import direct


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class _SwapW(kifmm.KIFMM):
    """Mistake: the W-list density on the box's outer surface instead of its inner one."""

    def m2t(self, x, a, p, phi_u, pot):
        direct(self.kernel, x, self._surf(a, K.OUTER, p), phi_u[a], pot)


class _SwapX(kifmm.KIFMM):
    """Mistake: the X-list sources evaluated on the outer surface instead of the inner one."""

    def s2l(self, b, a, p, ds, q):
        t = self.tree
        direct(self.kernel, self._surf(b, K.OUTER), self._pts(a, p), ds[t.begin[a]:t.end[a]], q)


class _ScaleW(kifmm.KIFMM):
    """Mistake: the W-list density divided by the box edge once more."""

    def m2t(self, x, a, p, phi_u, pot):
        direct(self.kernel, x, self._surf(a, K.INNER, p), phi_u[a] / self.tree.edge(a), pot)


class _ShiftX(kifmm.KIFMM):
    """Mistake: the X-list sources without their image shift."""

    def s2l(self, b, a, p, ds, q):
        t = self.tree
        direct(self.kernel, self._surf(b, K.INNER), self._pts(a), ds[t.begin[a]:t.end[a]], q)


def _graded(kernel, n, seed):
    """Points cubed toward one corner (a deep adaptive tree with W and X lists), densities with
    zero sum."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3)) ** 3
    d = rng.standard_normal((n, K.kdim(kernel)))
    d -= d.mean(0)
    return pts, d


def _surface_entries(f):
    t = f.tree
    nw = sum(1 for b in t.leaves() for (a, _) in f.lists.W[b] if not f.direct_source(a))
    nx = sum(1 for b in range(t.nbox) for (a, _) in f.lists.X.get(b, []) if not f.direct_target(b))
    return nw, nx


@pytest.mark.parametrize("kernel,p,s,n,tol", [(K.LAPLACE, 4, 120, 3000, 2e-4), (K.LAPLACE, 6, 200, 4000, 3e-6),
                                               (K.STOKES, 4, 120, 3000, 2e-3), (K.STOKES, 6, 200, 4000, 2e-4)])
def test_surface_w_and_x_free_space(kernel, p, s, n, tol):
    """Free space against the direct sum over every target; s > n(p) (56 at p = 4, 152 at p = 6)."""
    pts, d = _graded(kernel, n, 60)
    ref = np.zeros_like(d)
    direct(kernel, pts, pts, d, ref)
    f = kifmm.KIFMM(kernel, 0, p, s, pts)
    nw, nx = _surface_entries(f)
    assert nw > 20 and nx > 20, (nw, nx)
    assert _rel(f.evaluate(d), ref) < tol
    for wrong in (_SwapW, _SwapX, _ScaleW):
        assert _rel(wrong(kernel, 0, p, s, pts).evaluate(d), ref) > 20 * tol, wrong.__name__


@pytest.mark.parametrize("kernel,mask,tol", [(K.LAPLACE, 7, 1e-3), (K.STOKES, 7, 6e-3), (K.LAPLACE, 1, 1e-3),
                                             (K.STOKES, 3, 6e-3)])
def test_surface_w_and_x_periodic(kernel, mask, tol):
    """Triply, singly and doubly periodic sums at 60 sampled targets (p = 4, s = 120, graded
    points, many W/X entries through surfaces, many of them with an image shift): the oracle
    within the KIFMM error, each planted mistake (a swapped surface, a box-size factor, a lost
    image shift) at least 5 times beyond it."""
    n, p, s = 2000, 4, 120
    pts, d = _graded(kernel, n, 60)
    samp = np.random.default_rng(1).choice(n, 60, replace=False)
    ref = periodic.exact_potential(kernel, mask, pts[samp], pts, d)
    f = kifmm.KIFMM(kernel, mask, p, s, pts)
    nw, nx = _surface_entries(f)
    shifted = sum(1 for b in range(f.tree.nbox) for (a, sh) in f.lists.X.get(b, [])
                  if not f.direct_target(b) and any(sh))
    assert nw > 20 and nx > 20 and shifted > 20, (nw, nx, shifted)
    assert _rel(f.evaluate(d)[samp], ref) < tol
    for wrong in (_SwapW, _SwapX, _ScaleW, _ShiftX):
        assert _rel(wrong(kernel, mask, p, s, pts).evaluate(d)[samp], ref) > 5 * tol, wrong.__name__


class _NoBackground(kifmm.KIFMM):
    """The far field without the triply periodic Laplace background term."""

    def tp_laplace_background(self, ds, phi_root):
        return 0.0


def test_kifmm_tp_laplace_against_ewald():
    """Triply periodic Laplace KIFMM against the Ewald sum with its k = 0 mode removed: the error
    falls geometrically with p.  Without the background term (the constant that the root's
    equivalent density cannot carry) the result is off by a constant of a few per cent, the
    same at every p."""
    pb = W.laplace_sp_uniform(n=400, seed=11, s=20, mask=7)
    ex = periodic.exact_potential(K.LAPLACE, 7, pb.points, pb.points, pb.density[0])
    errs = [_rel(kifmm.KIFMM(K.LAPLACE, 7, p, 20, pb.points).evaluate(pb.density[0]), ex) for p in (4, 6, 8)]
    assert errs[0] < 2e-3 and errs[1] < 3e-5 and errs[2] < 1e-6, errs
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    off = _NoBackground(K.LAPLACE, 7, 8, 20, pb.points).evaluate(pb.density[0]) - ex
    assert _rel(off + ex, ex) > 1e-2
    assert np.std(off) < 1e-5 * np.abs(np.mean(off))       # a constant


@pytest.mark.parametrize("kernel,mask,tols", [(K.LAPLACE, 1, (2e-5, 5e-7)), (K.LAPLACE, 0, (1e-5, 2e-7)),
                                              (K.STOKES, 3, (6e-4, None))])
def test_separate_targets_against_the_periodic_sum(kernel, mask, tols):
    """T targets apart from S sources (Section 2's problem statement): the union tree's KIFMM at
    the targets against the periodic sum at the targets; the error falls with p."""
    rng = np.random.default_rng(70)
    src = rng.random((600, 3))
    trg = rng.random((300, 3)) ** 2            # denser near a corner than the sources
    d = rng.standard_normal((600, K.kdim(kernel)))
    d -= d.mean(0)
    ex = periodic.exact_potential(kernel, mask, trg, src, d)
    for p, tol in zip((6, 8), tols):
        if tol is None:
            continue
        f = kifmm.KIFMM(kernel, mask, p, 30, src, targets=trg)
        q = f.evaluate(d)
        assert q.shape == ex.shape
        assert _rel(q, ex) < tol, (p, _rel(q, ex))


def test_separate_targets_that_repeat_the_sources():
    """Targets placed exactly on the sources give the sources' own potentials (a coincident pair
    contributes nothing), to the KIFMM error of either tree; no targets give an empty result."""
    pb = W.stokes_tp_uniform(n=500, seed=71, p=6, s=40)
    same = kifmm.KIFMM(pb.kernel, 7, 6, 40, pb.points).evaluate(pb.density[0])
    sep = kifmm.KIFMM(pb.kernel, 7, 6, 40, pb.points, targets=pb.points.copy()).evaluate(pb.density[0])
    assert _rel(sep, same) < 2e-4
    none = kifmm.KIFMM(pb.kernel, 7, 6, 40, pb.points, targets=np.zeros((0, 3))).evaluate(pb.density[0])
    assert none.shape == (0, 3)


@pytest.mark.parametrize("kernel,mask,agree", [(K.STOKES, 7, 1e-10), (K.LAPLACE, 1, 1e-9), (K.LAPLACE, 7, 1e-12)])
def test_near_layer_option(kernel, mask, agree):
    """Section 3.6: a near field of l = 1, 2 or 3 layers of images (the root's image ring
    2 <= |p|_inf <= l as its V list, the far-field operator over |p|_inf > l) gives the same result
    to the FMM's accuracy (Table 4: "almost indistinguishable"); each against the periodic sum."""
    pb = (W.stokes_tp_uniform(n=300, seed=14, s=30, p=6) if kernel == K.STOKES
          else W.laplace_sp_uniform(n=400, seed=16, s=30, mask=mask))
    ex = periodic.exact_potential(kernel, mask, pb.points, pb.points, pb.density[0])
    res = {}
    for lay in (1, 2, 3):
        f = kifmm.KIFMM(kernel, mask, pb.p, 30, pb.points, near_layers=lay)
        ring = len(f.lists.V.get(0, []))
        assert ring == (0 if lay == 1 else ((2 * lay + 1) ** 3 - 27 if mask == 7 else 2 * (lay - 1)))
        res[lay] = f.evaluate(pb.density[0])
        assert _rel(res[lay], ex) < (5e-4 if kernel == K.STOKES else 1e-6)
    assert _rel(res[2], res[1]) < agree and _rel(res[3], res[1]) < agree
