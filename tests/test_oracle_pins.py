"""Pins of the oracle against what the paper and the mathematics fix (CPU only)."""
import itertools
import math

import numpy as np
import pytest

from conftest import golden
from oracle import kernels as K, periodic, kifmm, tree as otree
from oracle._native import direct
import workloads as W


# ------------------------------------------------------------------ kernels and surfaces

def test_kernel_closed_forms():
    rng = np.random.default_rng(0)
    r = rng.standard_normal((50, 3))
    rn = np.linalg.norm(r, axis=1)
    G = K.kernel_value(K.STOKES, r)
    # Stokeslet: symmetric, trace (1/8pi)(3/r + 1/r) = 1/(2 pi r), r is an eigenvector with eigenvalue 2/(8 pi r)
    assert np.allclose(G, G.transpose(0, 2, 1), rtol=0, atol=1e-15)
    assert np.allclose(np.trace(G, axis1=1, axis2=2), 4.0 / (8 * np.pi * rn), rtol=1e-14)
    assert np.allclose(np.einsum("nab,nb->na", G, r), (2.0 / (8 * np.pi * rn))[:, None] * r, rtol=1e-13)
    assert np.allclose(K.kernel_value(K.STOKES, -r), G, rtol=1e-15)
    assert np.allclose(K.kernel_value(K.LAPLACE, r), 1.0 / (4 * np.pi * rn), rtol=1e-15)
    # zero separation contributes nothing
    assert K.kernel_value(K.LAPLACE, np.zeros((1, 3)))[0] == 0.0
    assert np.all(K.kernel_value(K.STOKES, np.zeros((1, 3))) == 0.0)


def test_native_direct_matches_matrix():
    rng = np.random.default_rng(1)
    x, y = rng.random((40, 3)), rng.random((30, 3))
    y[3] = x[5]                                  # one coincident pair
    for kern in (K.LAPLACE, K.STOKES):
        k = K.kdim(kern)
        d = rng.standard_normal((30, k))
        out = np.zeros((40, k))
        sh = np.array([0.0, 1.0, -1.0])
        direct(kern, x, y, d, out, shift=sh)
        ref = K.kernel_matrix(kern, x, y + sh) @ d.reshape(-1)
        assert np.allclose(out.reshape(-1), ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 6, 8])
def test_surface_grid(p):
    u = K.unit_surface(p)
    assert u.shape == (6 * (p - 1) ** 2 + 2, 3)
    assert np.allclose(np.max(np.abs(u), axis=1), 1.0)
    assert len({tuple(r) for r in np.round(u, 12)}) == u.shape[0]
    # all 8 vertices present; lexicographic order starts at (-1,-1,-1)
    assert np.allclose(u[0], [-1, -1, -1]) and np.allclose(u[-1], [1, 1, 1])


@pytest.mark.parametrize("row", golden("table1_conditioning.txt"))
def test_table1_rank_and_condition(row):
    kern = K.STOKES if row[0] == "stokes" else K.LAPLACE
    p, kappa, rank, dim = int(row[1]), float(row[2]), int(row[3]), int(row[4])
    u = K.unit_surface(p)
    A = K.kernel_matrix(kern, 0.5 * K.INNER * u, 0.5 * K.OUTER * u)
    assert A.shape == (dim, dim)
    s = np.linalg.svd(A, compute_uv=False)
    r = int(np.sum(s >= np.finfo(float).eps * s[0] * dim))
    assert abs(r - rank) <= 2, (r, rank)
    assert abs(math.log10(s[0] / s[-1]) - math.log10(kappa)) < 0.1


def test_backward_stable_solver_stokes_p8():
    """Appendix B: (V S^+)(U^T b) is backward stable; the explicit pseudo-inverse is not."""
    u = K.unit_surface(8)
    A = K.kernel_matrix(K.STOKES, 0.5 * K.INNER * u, 0.5 * K.OUTER * u)
    f = kifmm.pinv_factors(A, rel_threshold=kifmm.EPS)     # Appendix B's cutoff, as in Table 7
    one = np.ones(A.shape[0])
    x = f.apply(one)
    err = np.max(np.abs(A @ x - one))
    explicit = (f.VS @ f.Ut) @ one
    err_explicit = np.max(np.abs(A @ explicit - one))
    assert err < 1e-12
    assert err_explicit > 100 * err


@pytest.mark.slow
def test_backward_stable_solver_stokes_p16():
    """Table 7 row at p = 16 (4056 x 4056): backward error in the 1e-14..1e-13 band."""
    rows = {r[1]: float(r[2]) for r in golden("svd_backward_error.txt")}
    u = K.unit_surface(16)
    A = K.kernel_matrix(K.STOKES, 0.5 * K.INNER * u, 0.5 * K.OUTER * u)
    f = kifmm.pinv_factors(A, rel_threshold=kifmm.EPS)     # Appendix B's cutoff, as in Table 7
    one = np.ones(A.shape[0])
    err = np.max(np.abs(A @ f.apply(one) - one))
    assert err < 10 * rows["SVDpvfmm"]
    err_explicit = np.max(np.abs(A @ ((f.VS @ f.Ut) @ one) - one))
    assert err_explicit > 100 * err



class _NoisySolve:
    """A check-to-equivalent solve whose input is perturbed by relative noise of 2^-53."""

    def __init__(self, base, rng):
        self.base, self.rng = base, rng

    def apply(self, q):
        return self.base.apply(q * (1.0 + 2.0 ** -53 * self.rng.standard_normal(q.shape)))


@pytest.mark.parametrize("kernel,p,lo,hi", [(K.STOKES, 8, 1e-13, 1.5e-12), (K.LAPLACE, 8, 0.0, 2e-13)])
def test_solve_amplification_of_rounding(kernel, p, lo, hi):
    """How far rounding-level changes of every check potential move the final potentials: the
    floor under FP64 agreement of two implementations that sum in different orders.  With the
    default cutoff (1e-11 s_max) Stokes p = 8 moves by ~4e-13 (with Table 1's rank criterion,
    which keeps singular values down to 2.18e-13 s_max, by ~3e-11); Laplace p = 8 is benign."""
    pb = (W.stokes_tp_uniform(n=4000, seed=21, p=p, s=300) if kernel == K.STOKES
          else W.laplace_sp_uniform(n=4000, seed=21, p=p, s=100))
    f = kifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
    a = f.evaluate(pb.density[0])
    up, dn = f.ops.up, f.ops.down
    rng = np.random.default_rng(1)
    try:
        f.ops.up, f.ops.down = _NoisySolve(up, rng), _NoisySolve(dn, rng)
        b = f.evaluate(pb.density[0])
    finally:
        f.ops.up, f.ops.down = up, dn
    x = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert lo < x < hi, x

# ------------------------------------------------------------------ singly periodic Laplace sums

@pytest.mark.parametrize("axis", [0, 2])
def test_madelung_exact(axis):
    val = {r[0]: float(r[1]) for r in golden("madelung_1d.txt")}
    pts, q = W.madelung_chain(axis)
    mask = 1 << axis
    pot = periodic.exact_potential(K.LAPLACE, mask, pts, pts, q)[:, 0]
    assert abs(pot[0] - val["kernel_1_over_4pi_r"]) < 1e-14
    assert abs(pot[2] - val["kernel_1_over_4pi_r"]) < 1e-14
    assert abs(pot[1] + val["kernel_1_over_4pi_r"]) < 1e-14
    assert abs(val["kernel_1_over_r"] / (4 * np.pi) - val["kernel_1_over_4pi_r"]) < 1e-15


@pytest.mark.parametrize("p", [6, 8, 10, 12])
def test_madelung_kifmm(p):
    """Algorithm 2 on the 1D crystal: the error falls with p (Section 3.2, Fig. 2).  Under the
    default solve cutoff (1e-11 s_max) the fall flattens past p = 10 (1.3e-10 at p = 10, 1.9e-11
    at p = 12); under Appendix B's bare cutoff (2^-52 s_max) p = 12 comes close to machine
    precision, as Fig. 2 shows for the converged far field."""
    val = float(golden("madelung_1d.txt")[1][1])
    pts, q = W.madelung_chain(2)
    f = kifmm.KIFMM(K.LAPLACE, 4, p, 10, pts)
    pot = f.evaluate(q[:, None])[:, 0]
    err = max(abs(pot[0] - val), abs(pot[2] - val))
    bound = {6: 2e-6, 8: 2e-8, 10: 3e-10, 12: 5e-11}[p]
    assert err < bound, err
    if p == 12:
        f = kifmm.KIFMM(K.LAPLACE, 4, p, 10, pts, rel_threshold=2.0 ** -52)
        pot = f.evaluate(q[:, None])[:, 0]
        assert max(abs(pot[0] - val), abs(pot[2] - val)) < 2e-12


def test_sp_tail_closed_form_matches_long_direct_sum():
    """The Legendre/Hurwitz tail equals the far images summed one by one."""
    rng = np.random.default_rng(3)
    r = rng.uniform(-1.0, 1.0, (40, 3))
    a = periodic.sp_laplace_sum(r, 0, kmin=2, n=8)
    b = periodic.sp_laplace_sum(r, 0, kmin=2, n=600)
    assert np.max(np.abs(a - b)) < 1e-14
    # the paper's own route: direct image sum to n, converging like 1/n^2 per pair after the
    # monopole subtraction; Richardson in n matches the closed form
    def direct_to(n):
        e = np.array([1.0, 0, 0])
        out = np.zeros(r.shape[0])
        for k in range(2, n + 1):
            for s in (1, -1):
                out += 1 / np.linalg.norm(r - s * k * e, axis=1) - 1.0 / k
        return out / (4 * np.pi)
    d1, d2 = direct_to(2000), direct_to(4000)
    rich = (4 * d2 - d1) / 3
    assert np.max(np.abs(rich - a)) < 1e-10
    assert np.max(np.abs(d2 - a)) > 1e-9       # the plain sum has not converged yet


def test_sp_periodicity_and_neutral_shift_invariance():
    rng = np.random.default_rng(4)
    src = rng.random((12, 3)); q = rng.uniform(-1, 1, 12); q -= q.mean()
    trg = rng.random((7, 3))
    a = periodic.exact_potential(K.LAPLACE, 1, trg, src, q)
    b = periodic.exact_potential(K.LAPLACE, 1, trg + [1.0, 0, 0], src, q)
    assert np.max(np.abs(a - b)) < 1e-13



def test_sp_stokes_tail_closed_form_and_relations():
    """SP Stokeslet sum: the closed-form tail (Legendre and index-3/2 Gegenbauer expansions)
    against a long direct image sum; the trace is four times the raw Laplace sum
    (tr(I/|x| + x x^T/|x|^3) = 4/|x|); periodic along the axis; far = full - near."""
    rng = np.random.default_rng(41)
    r = rng.uniform(-1.0, 1.0, (8, 3))
    r[0] = 0.0
    for axis in (0, 2):
        a = periodic.sp_stokes_sum(r, axis, n=64)
        b = periodic.sp_stokes_sum(r, axis, n=3000, mterms=3)
        assert np.max(np.abs(a - b)) < 1e-14
        lap = periodic.sp_laplace_sum(r, axis)
        assert np.max(np.abs(np.trace(a, axis1=1, axis2=2) - 2.0 * lap)) < 1e-14   # (4/8pi) = 2 (1/4pi)
        e = np.zeros(3); e[axis] = 1.0
        c = periodic.sp_stokes_sum(r + 2.0 * e, axis)
        assert np.max(np.abs(c[1:] - a[1:])) < 1e-14
        # the tree sums the images |k| <= 1 unregularised: full = near + far - 2 S(e)
        near = sum(K.kernel_value(K.STOKES, r[1:] - k * e) for k in (-1, 0, 1))
        far = periodic.sp_stokes_sum(r[1:], axis, kmin=2)
        two_s_e = 2.0 * K.kernel_value(K.STOKES, e[None, :])[0]
        assert np.max(np.abs(a[1:] - (near + far - two_s_e))) < 1e-14


@pytest.mark.parametrize("p,tol", [(6, 5e-4), (8, 5e-5)])
def test_kifmm_sp_stokes_against_lattice_sum(p, tol):
    """Singly periodic Stokes (axis x): the periodic KIFMM against the regularised image sum."""
    pb = W.stokes_tp_uniform(n=300, seed=42, p=p, s=25, mask=1)
    ex = periodic.exact_potential(K.STOKES, 1, pb.points, pb.points, pb.density[0])
    q = kifmm.KIFMM(K.STOKES, 1, p, 25, pb.points).evaluate(pb.density[0])
    assert np.linalg.norm(q - ex) / np.linalg.norm(ex) < tol

# ------------------------------------------------------------------ triply periodic Ewald sums

def test_tp_stokes_xi_independence():
    rng = np.random.default_rng(5)
    r = rng.uniform(-1.05, 1.05, (60, 3))
    r[0] = 0.0
    vals = [periodic.tp_stokes_sum(r, xi=xi) for xi in (3.0, 4.0, 5.5)]
    scale = np.max(np.abs(vals[0]))
    for v in vals[1:]:
        assert np.max(np.abs(v - vals[0])) < 1e-13 * scale
    far = [periodic.tp_stokes_sum(r, xi=xi, far_only=True) for xi in (3.0, 5.5)]
    assert np.max(np.abs(far[1] - far[0])) < 1e-13 * np.max(np.abs(far[0]))


def test_tp_stokes_far_equals_full_minus_near():
    rng = np.random.default_rng(6)
    r = rng.uniform(-0.9, 0.9, (30, 3))
    full = periodic.tp_stokes_sum(r)
    far = periodic.tp_stokes_sum(r, far_only=True)
    near = sum(K.kernel_value(K.STOKES, r - np.array(p)) for p in itertools.product((-1, 0, 1), repeat=3))
    assert np.max(np.abs(full - near - far)) < 1e-13


def test_tp_stokes_periodic_and_zero_flux():
    """u is periodic and the flux through each face vanishes (Section 3.3, TP tests)."""
    pts, f = W.one_point_force()
    n = 48
    g = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(g, g, indexing="ij")
    for axis in range(3):
        plane = np.zeros((n * n, 3))
        others = [a for a in range(3) if a != axis]
        plane[:, others[0]] = X.ravel(); plane[:, others[1]] = Y.ravel()
        u = periodic.exact_potential(K.STOKES, 7, plane, pts, f)
        flux = np.mean(u[:, axis])                  # periodic trapezoid rule, spectrally accurate
        assert abs(flux) < 1e-12
        shifted = plane.copy(); shifted[:, axis] += 1.0
        u2 = periodic.exact_potential(K.STOKES, 7, shifted[:50], pts, f)
        assert np.max(np.abs(u2 - u[:50])) < 1e-13


def test_tp_stokes_affine_difference_from_cubic_lattice_sum():
    """A cubic truncation of the force-free lattice sum differs from Ewald by an affine field."""
    pts, f = W.two_point_forces()
    rng = np.random.default_rng(7)
    trg = rng.random((30, 3))
    ew = periodic.exact_potential(K.STOKES, 7, trg, pts, f)
    resid = []
    for P in (8, 16):
        u = np.zeros((30, 3))
        for p in itertools.product(range(-P, P + 1), repeat=3):
            direct(K.STOKES, trg, pts, f, u, shift=np.array(p, dtype=float))
        diff = u - ew
        A = np.column_stack([np.ones(30), trg])
        coef, *_ = np.linalg.lstsq(A, diff, rcond=None)
        resid.append(np.max(np.abs(diff - A @ coef)))
    assert resid[1] < resid[0] / 3          # truncation error of the cubic sum falls with P
    assert resid[1] < 2e-4


def test_tp_laplace_nacl_madelung():
    """Rock-salt Madelung constant 1.747564594633... from the TP Laplace Ewald sum."""
    base = np.array(list(itertools.product((0, 0.5), repeat=3)))
    q = np.array([(-1.0) ** int(round(2 * sum(b))) for b in base])
    pts = base + 0.25
    pot = periodic.exact_potential(K.LAPLACE, 7, pts[:1], pts, q)[0, 0]
    # potential at a +1 ion = -M / (4 pi d), d = 0.5 nearest-neighbour distance
    M = -pot * 4 * np.pi * 0.5
    assert abs(M - 1.7475645946331822) < 1e-12
    a = periodic.tp_laplace_sum(np.array([[0.1, 0.2, 0.3], [0.0, 0.0, 0.0]]), xi=3.0)
    b = periodic.tp_laplace_sum(np.array([[0.1, 0.2, 0.3], [0.0, 0.0, 0.0]]), xi=5.0)
    assert np.max(np.abs(a - b)) < 1e-13



# ------------------------------------------------------------------ doubly periodic Ewald sums

def _dp(kernel):
    return periodic.dp_stokes_sum if kernel == K.STOKES else periodic.dp_laplace_sum


def _regularised_lattice_sum(kernel, r, R):
    """G(r) + sum_{0 < |p|_inf <= R} [G(r - p) - G(p)] over the in-plane lattice (x, y)."""
    a = np.arange(-R, R + 1)
    P = np.array([(x, y, 0.0) for x in a for y in a if (x, y) != (0, 0)])
    s = np.sum(K.kernel_value(kernel, r[None, :] - P) - K.kernel_value(kernel, P), axis=0)
    return s + K.kernel_value(kernel, r[None, :])[0]


@pytest.mark.parametrize("kernel", [K.STOKES, K.LAPLACE])
def test_dp_xi_independence(kernel):
    rng = np.random.default_rng(31)
    r = rng.uniform(-1.05, 1.05, (40, 3))
    r[0] = 0.0
    vals = [_dp(kernel)(r, 3, xi=xi) for xi in (3.0, 4.0, 5.5)]
    scale = np.max(np.abs(vals[0]))
    for v in vals[1:]:
        assert np.max(np.abs(v - vals[0])) < 1e-13 * scale
    far = [_dp(kernel)(r, 3, xi=xi, far_only=True) for xi in (3.0, 5.5)]
    assert np.max(np.abs(far[1] - far[0])) < 1e-13 * np.max(np.abs(far[0]))


@pytest.mark.parametrize("kernel", [K.STOKES, K.LAPLACE])
def test_dp_against_regularised_lattice_sum(kernel):
    """The DP sum is the limit of symmetric square image sums, each image regularised by
    its value at the lattice point; the partial sums converge like 1/R, so five of them
    (R = 16 .. 256) are Richardson-extrapolated in 1/R."""
    rng = np.random.default_rng(32)
    r = np.vstack([np.zeros(3), rng.uniform(-1.0, 1.0, (3, 3))])
    ew = _dp(kernel)(r, 3)
    for i, rv in enumerate(r):
        T = [_regularised_lattice_sum(kernel, rv, R) for R in (16, 32, 64, 128, 256)]
        for lvl in range(1, len(T)):
            T = [(2 ** lvl * T[j + 1] - T[j]) / (2 ** lvl - 1) for j in range(len(T) - 1)]
        assert np.max(np.abs(T[0] - ew[i])) < 2e-10 * max(1.0, np.max(np.abs(ew[i]))), i


@pytest.mark.parametrize("kernel", [K.STOKES, K.LAPLACE])
def test_dp_far_equals_full_minus_near_and_frames(kernel):
    rng = np.random.default_rng(33)
    r = rng.uniform(-0.9, 0.9, (20, 3))
    f = _dp(kernel)
    near = sum(K.kernel_value(kernel, r - np.array([a, b, 0.0])) for a in (-1, 0, 1) for b in (-1, 0, 1))
    assert np.max(np.abs(f(r, 3) - near - f(r, 3, far_only=True))) < 1e-13
    # periodic in x and y, even in r
    assert np.max(np.abs(f(r + [1.0, -2.0, 0.0], 3) - f(r, 3))) < 1e-13
    assert np.max(np.abs(f(-r, 3) - f(r, 3))) < 1e-13
    # the free axis may be any of the three: periodic in (y, z) is (x, y) with axes relabelled
    order = [1, 2, 0]                   # mask 6: periodic y, z then free x
    rr = np.empty_like(r)
    rr[:, order] = r                    # rr[:, order[i]] = r[:, i]
    a = f(rr, 6)
    b = f(r, 3)
    if kernel == K.STOKES:
        a = a[:, order][:, :, order]
    assert np.max(np.abs(a - b)) < 1e-13


def test_dp_stokes_zero_flux_and_shear_at_infinity():
    """Net-force-free forces in a slab: no net flux of u_z through any plane z = const
    (the k_par = 0 mode of u_z vanishes), and far from the slab the flow tends to a
    uniform stream, u_par(+-inf) = +-(1/2) sum_s z_s f_s,par (with K = S/(8 pi), mu = 1:
    a plane force density f gives a jump -f in du/dz)."""
    rng = np.random.default_rng(34)
    n = 7
    src = np.column_stack([rng.random((n, 2)), rng.uniform(0.3, 0.7, n)])
    f = rng.standard_normal((n, 3)); f -= f.mean(0)
    m = 40
    g = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(g, g, indexing="ij")
    for z0 in (0.95, 0.05):
        plane = np.column_stack([X.ravel(), Y.ravel(), np.full(m * m, z0)])
        u = periodic.exact_potential(K.STOKES, 3, plane, src, f)
        assert abs(np.mean(u[:, 2])) < 1e-12 * np.max(np.abs(u))
    mom = 0.5 * (src[:, 2:3] * f).sum(0)
    for zs, sign in ((6.0, 1.0), (-5.0, -1.0)):
        trg = np.column_stack([rng.random((5, 2)), np.full(5, zs)])
        u = periodic.exact_potential(K.STOKES, 3, trg, src, f)
        assert np.max(np.abs(u[:, :2] - sign * mom[:2])) < 1e-12
        assert np.max(np.abs(u[:, 2])) < 1e-12


def test_dp_laplace_dipole_layer_potential_jump():
    """Neutral charges in a slab: far above and below, the potential tends to
    +-(1/2) sum_s z_s q_s (the potential step of a dipole layer, 1/(4 pi r) units)."""
    rng = np.random.default_rng(35)
    src = np.column_stack([rng.random((6, 2)), rng.uniform(0.2, 0.8, 6)])
    q = rng.uniform(-1, 1, 6); q -= q.mean()
    mom = 0.5 * np.sum(src[:, 2] * q)
    for zs, sign in ((6.0, 1.0), (-5.0, -1.0)):
        trg = np.column_stack([rng.random((4, 2)), np.full(4, zs)])
        u = periodic.exact_potential(K.LAPLACE, 3, trg, src, q[:, None])
        assert np.max(np.abs(u[:, 0] - sign * mom)) < 1e-12

# ------------------------------------------------------------------ tree and lists

def _coverage_counts(t, lists, mask):
    """Count how many times each (target leaf, source leaf, shift) is covered by U, W, X, V."""
    per = [(-1, 0, 1) if mask & (1 << a) else (0,) for a in range(3)]
    shifts = list(itertools.product(*per))
    leaves = t.leaves()

    def anc(b):
        out = []
        while b >= 0:
            out.append(b)
            b = t.parent[b]
        return out
    count = {(tl, sl, p): 0 for tl in leaves for sl in leaves for p in shifts}
    for tl in leaves:
        for (a, p) in lists.U[tl]:
            count[(tl, a, p)] += 1
        for (a, p) in lists.W[tl]:
            for sl in leaves:
                if a in anc(sl):
                    count[(tl, sl, p)] += 1
        for b in anc(tl):
            for (a, p) in lists.X.get(b, []):
                count[(tl, a, p)] += 1
            for (a, p) in lists.V.get(b, []):
                for sl in leaves:
                    if a in anc(sl):
                        count[(tl, sl, p)] += 1
    return count


@pytest.mark.parametrize("mask,n,s,seed", [(0, 300, 8, 1), (1, 300, 8, 2), (7, 200, 6, 3), (3, 250, 10, 4), (7, 3, 1, 5)])
def test_lists_cover_every_pair_exactly_once(mask, n, s, seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3)) ** 2            # graded density -> adaptive tree
    u = otree.wrap(pts, mask)
    t = otree.build_tree(u, s)
    lists = otree.build_lists(t, mask)
    counts = _coverage_counts(t, lists, mask)
    bad = [k for k, c in counts.items() if c != 1]
    assert not bad, bad[:5]
    assert t.depth() >= 2 or n < 10


@pytest.mark.parametrize("mask,n,s,seed", [(0, 400, 6, 41), (7, 400, 6, 42), (3, 300, 5, 43), (1, 300, 5, 44)])
def test_direct_pair_separations_fit_twice_the_larger_edge(mask, n, s, seed):
    """The float32 near field forms every separation of a direct pair (U, and the W/X pairs
    taken through points) as an integer in units of 2^-29 H, H the larger of the two boxes'
    edges, and relies on |d| <= 2H per component (so |d| <= 2^30 units) and on the centre
    difference |c_B - c_A - p| <= 1.25 H.  Both hold for every U, W and X entry of adaptive
    trees (graded and clustered points, every periodicity)."""
    rng = np.random.default_rng(seed)
    pts = np.concatenate([rng.random((n // 2, 3)) ** 3,
                          np.mod(0.3 + 0.01 * rng.standard_normal((n - n // 2, 3)), 1.0)])
    u = otree.wrap(pts, mask)
    t = otree.build_tree(u, s)
    lists = otree.build_lists(t, mask)
    assert t.depth() >= 4
    worst_d = worst_c = 0.0
    for name in ("U", "W", "X"):
        for b, entries in getattr(lists, name).items():
            for (a, p) in entries:
                H = max(t.edge(a), t.edge(b))
                dc = np.abs(t.centre(b) - t.centre(a) - np.array(p, dtype=float))
                dmax = dc + 0.5 * (t.edge(a) + t.edge(b))
                worst_d = max(worst_d, float(np.max(dmax)) / H)
                worst_c = max(worst_c, float(np.max(dc)) / H)
    assert worst_d <= 2.0 and worst_c <= 1.25, (worst_d, worst_c)


def test_root_leaf_lists():
    t = otree.build_tree(np.array([[0.1, 0.2, 0.3], [0.6, 0.7, 0.8]]), 5)
    lists = otree.build_lists(t, 7)
    assert t.nbox == 1 and len(lists.U[0]) == 27
    lists1 = otree.build_lists(t, 1)
    assert sorted(p for _, p in lists1.U[0]) == [(-1, 0, 0), (0, 0, 0), (1, 0, 0)]


def test_tree_quantisation_edges():
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [1 - 2 ** -53, 0.5, -0.0], [0.999999, 1.0, 0.25]])
    u = otree.wrap(pts, 1)           # x periodic: 1.0 -> 0.0; y, z closed [0, 1]
    assert u[1, 0] == 0.0 and u[1, 1] == 1.0
    q = otree.quantise(u)
    assert q[1, 1] == (1 << 21) - 1 and q[2, 0] == (1 << 21) - 1 and q[2, 2] == 0
    with pytest.raises(otree.OutOfBox):
        otree.wrap(np.array([[0.5, 1.0 + 1e-12, 0.5]]), 1)
    w = otree.wrap(np.array([[-1e-300, 0.5, 0.5], [-0.25, 0.5, 0.5], [3.5, 0.5, 0.5]]), 1)
    assert list(w[:, 0]) == [0.0, 0.75, 0.5]


def test_tree_split_rule_and_order():
    rng = np.random.default_rng(9)
    u = rng.random((500, 3))
    t = otree.build_tree(u, 20)
    for b in range(t.nbox):
        cnt = t.end[b] - t.begin[b]
        assert cnt > 0
        assert t.is_leaf(b) == (cnt <= 20)
    assert all(t.level[i] <= t.level[i + 1] for i in range(t.nbox - 1))
    assert np.all(np.diff(t.keys.astype(np.float64)) >= 0)
    # stable: equal keys keep input order
    u2 = np.repeat(u[:5], 3, axis=0)
    t2 = otree.build_tree(u2, 100)
    for i in range(len(t2.perm) - 1):
        if t2.keys[i] == t2.keys[i + 1]:
            assert t2.perm[i] < t2.perm[i + 1]


# ------------------------------------------------------------------ KIFMM against the definitions

def test_kifmm_free_space_converges_to_direct_sum():
    rng = np.random.default_rng(10)
    pts = rng.random((1500, 3))
    for kern in (K.LAPLACE, K.STOKES):
        k = K.kdim(kern)
        d = rng.standard_normal((1500, k))
        ref = np.zeros((1500, k))
        direct(kern, pts, pts, d, ref)
        errs = []
        for p in (4, 6, 8, 10):
            q = kifmm.KIFMM(kern, 0, p, 40, pts).evaluate(d)
            errs.append(np.linalg.norm(q - ref) / np.linalg.norm(ref))
        assert all(errs[i] > 1.5 * errs[i + 1] for i in range(3)), errs
        if kern == K.LAPLACE:
            assert errs[0] > 10 * errs[1] > 100 * errs[2] and errs[2] < 1e-7, errs
        else:
            # the Stokeslet's surface representation converges more slowly with p
            assert errs[2] < 5e-6 and errs[3] < 1e-7, errs


def test_kifmm_sp_laplace_against_lattice_sum():
    pb = W.laplace_sp_uniform(n=400, seed=11, s=20)
    ex = periodic.exact_potential(K.LAPLACE, 1, pb.points, pb.points, pb.density[0])
    q = kifmm.KIFMM(K.LAPLACE, 1, 8, 20, pb.points).evaluate(pb.density[0])
    assert np.linalg.norm(q - ex) / np.linalg.norm(ex) < 1e-6


@pytest.mark.parametrize("pts_f", ["two", "one"])
def test_kifmm_tp_stokes_point_forces(pts_f):
    """Section 3.3 point-force tests: net force allowed in TP."""
    pts, f = W.two_point_forces() if pts_f == "two" else W.one_point_force()
    rng = np.random.default_rng(12)
    trg = rng.random((60, 3))
    allp = np.concatenate([pts, trg])
    dens = np.concatenate([f, np.zeros((60, 3))])
    ex = periodic.exact_potential(K.STOKES, 7, allp, pts, f)
    # KIFMM accuracy for the Stokeslet: ~1e-4 at p = 6, ~1e-6 at p = 8
    for p, tol in ((6, 5e-4), (8, 2e-5)):
        q = kifmm.KIFMM(K.STOKES, 7, p, 8, allp).evaluate(dens)
        assert np.max(np.abs(q - ex)) / np.max(np.abs(ex)) < tol


def test_kifmm_tp_stokes_random_against_ewald():
    pb = W.stokes_tp_uniform(n=300, seed=13, s=25, p=8)
    ex = periodic.exact_potential(K.STOKES, 7, pb.points, pb.points, pb.density[0])
    errs = []
    for p in (6, 8):
        q = kifmm.KIFMM(K.STOKES, 7, p, 25, pb.points).evaluate(pb.density[0])
        errs.append(np.linalg.norm(q - ex) / np.linalg.norm(ex))
    assert errs[1] < errs[0] / 10 and errs[1] < 5e-5, errs



@pytest.mark.parametrize("kernel,p,tol", [(K.STOKES, 6, 5e-4), (K.STOKES, 8, 5e-5), (K.LAPLACE, 8, 1e-6)])
def test_kifmm_dp_against_ewald(kernel, p, tol):
    """Doubly periodic slab (z ~ N(0.5, 0.1), clipped): the periodic KIFMM against the
    pairwise DP sum."""
    rng = np.random.default_rng(21)
    n = 300
    pts = np.column_stack([rng.random((n, 2)), np.clip(rng.normal(0.5, 0.1, n), 0, 1)])
    k = 3 if kernel == K.STOKES else 1
    d = rng.standard_normal((n, k)); d -= d.mean(0)
    ex = periodic.exact_potential(kernel, 3, pts, pts, d)
    q = kifmm.KIFMM(kernel, 3, p, 25, pts).evaluate(d)
    assert np.linalg.norm(q - ex) / np.linalg.norm(ex) < tol

def test_near_layer_independence():
    """Changing the near/far split layer l leaves the result unchanged to KIFMM accuracy
    (Section 3.4).  Near field: direct sum over |p|_inf <= l; far field: K^{P,F}_l applied
    to the root's upward density, its downward solve and an explicit L2T (step d)."""
    pb = W.stokes_tp_uniform(n=200, seed=14, s=30, p=8)
    f = kifmm.KIFMM(K.STOKES, 7, 8, 30, pb.points)
    ex = periodic.exact_potential(K.STOKES, 7, pb.points, pb.points, pb.density[0])
    ops = f.ops
    d = pb.density[0]
    phi_u = f.upward(d[f.tree.perm])[0]
    X = ops.inner + 0.5
    res = {}
    for lay in (1, 2, 3):
        near = np.zeros_like(d)
        for p in itertools.product(range(-lay, lay + 1), repeat=3):
            direct(K.STOKES, pb.points, pb.points, d, near, shift=np.array(p, dtype=float))
        kpf = periodic.far_kernel_matrix(K.STOKES, 7, X, X, near_layers=lay)
        phi_d = ops.down.apply(kpf @ phi_u)
        far = (K.kernel_matrix(K.STOKES, f.u, ops.outer + 0.5) @ phi_d).reshape(-1, 3)
        res[lay] = near + far
    err = {lay: np.linalg.norm(res[lay] - ex) / np.linalg.norm(ex) for lay in res}
    # every split reaches the exact sum to the accuracy of order-8 surfaces (measured under the
    # default solve cutoff: 2.4e-6, 7.0e-7 and 1.2e-6 for l = 1, 2, 3), and two splits agree
    # with each other to that accuracy
    assert max(err.values()) < 4e-6, err
    assert np.linalg.norm(res[2] - res[3]) / np.linalg.norm(ex) < 1e-6
    q1 = f.evaluate(d)
    assert np.linalg.norm(q1 - res[2]) / np.linalg.norm(ex) < 5e-6


def test_step_d_far_field():
    """Algorithm 2's step d (the far field solved into the root's own downward equivalent
    density, phi^{B0,d} = T_M2L phi^{B0,u} of Section 3.4, and evaluated at every target) against
    the Ewald sums, and against the default placement that hands the same check potential down
    the tree.  The two differ only by the truncation of the downward translations, far below the
    FMM's own error; a wrong surface, a lost box-size factor or a far field counted twice would
    each show at the 1e-3 level or above."""
    cases = [(K.STOKES, 7, W.stokes_tp_uniform(n=300, seed=14, s=30, p=8), 2e-5, 1e-6),
             (K.LAPLACE, 1, W.laplace_sp_uniform(n=400, seed=16, s=30), 1e-6, 2e-8)]
    for kern, mask, pb, tol, tol_d in cases:
        f = kifmm.KIFMM(kern, mask, 8, 30, pb.points)
        d = pb.density[0]
        ex = periodic.exact_potential(kern, mask, pb.points, pb.points, d)
        a = f.evaluate(d)
        b = f.evaluate(d, step_d=True)
        nx = np.linalg.norm(ex)
        assert np.linalg.norm(b - ex) / nx < tol
        assert 0 < np.linalg.norm(a - b) / nx < tol_d
        # the step-d term by itself is the images beyond the first layer, to the same accuracy
        ops = f.ops
        phi_u = f.upward(np.ascontiguousarray(d.reshape(len(d), -1)[f.tree.perm]))[0]
        far = (K.kernel_matrix(kern, f.u, ops.outer + 0.5) @ ops.down.apply(ops.mroot @ phi_u))
        near = np.zeros_like(ex)
        axes = [np.arange(-1, 2) if mask >> i & 1 else np.zeros(1, int) for i in range(3)]
        for p in itertools.product(*axes):
            direct(kern, pb.points, pb.points, d, near, shift=np.array(p, dtype=float))
        assert np.linalg.norm(far.reshape(ex.shape) - (ex - near)) / nx < tol


def test_kifmm_linearity_and_periodic_relabel():
    pb = W.stokes_tp_uniform(n=250, seed=15, s=30, p=6, n_rhs=2)
    f = kifmm.KIFMM(K.STOKES, 7, 6, 30, pb.points)
    a = f.evaluate(pb.density[0]); b = f.evaluate(pb.density[1])
    c = f.evaluate(2.0 * pb.density[0] - 0.5 * pb.density[1])
    assert np.max(np.abs(c - (2 * a - 0.5 * b))) < 1e-10 * np.max(np.abs(c))
    # shifting every point by a whole period leaves the wrapped problem unchanged
    # (the shifted coordinates round differently in their last bits, so the match is to rounding)
    g = kifmm.KIFMM(K.STOKES, 7, 6, 30, pb.points + np.array([1.0, -1.0, 2.0]))
    assert np.array_equal(g.tree.perm, f.tree.perm)
    assert np.max(np.abs(g.evaluate(pb.density[0]) - a)) < 1e-10 * np.max(np.abs(a))
    # a non-dyadic translation changes the tree but not the physics (to KIFMM accuracy)
    h = kifmm.KIFMM(K.STOKES, 7, 6, 30, pb.points + 0.3141)
    assert np.linalg.norm(h.evaluate(pb.density[0]) - a) / np.linalg.norm(a) < 2e-3


def test_kifmm_target_subset_matches_full():
    pb = W.laplace_sp_uniform(n=1500, seed=16, s=40)
    f = kifmm.KIFMM(K.LAPLACE, 1, 6, 40, pb.points)
    full = f.evaluate(pb.density[0], return_sorted=True)
    leaves = f.tree.leaves()[::5]
    sub = f.evaluate(pb.density[0], target_leaves=leaves)
    for b in leaves:
        assert np.allclose(sub[b], full[f.tree.begin[b]:f.tree.end[b]], rtol=0, atol=1e-14)


def test_solver_threshold_and_spread_stokes_p8():
    """The solve cutoff.  Two backward-stable SVD drivers (LAPACK gesdd, gesvd) agree on the
    Stokes p = 8 potentials to ~1e-12 with the default cutoff (singular values <= 1e-11 s_max
    dropped: rank 847 of 888), to ~5e-11 with Table 1's rank criterion eps * s_max * dim(A)
    (rank 881), and only to the 1e-9 level under Appendix B's bare eps * s_max, which keeps
    directions at the rounding level of A (condition number 1.26e13, Table 1).  The dropped
    directions also cost accuracy against the exact periodic sum: the default is the most
    accurate of the three."""
    import scipy.linalg as sl
    pb = W.stokes_tp_uniform(n=4000, seed=21, p=8, s=300)
    samp = np.random.default_rng(0).choice(pb.n, 60, replace=False)
    ex = periodic.exact_potential(pb.kernel, pb.periodic_mask, pb.points[samp], pb.points, pb.density[0])

    def solve(thr, driver):
        f = kifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
        ops = f.ops
        keep_up, keep_dn = ops.up, ops.down

        def pinv(A):
            U, s, Vt = sl.svd(A, lapack_driver=driver)
            keep = s > thr * s[0]
            return kifmm.Pinv(Ut=U[:, keep].T.copy(), VS=(Vt[keep].T / s[keep][None, :]).copy())
        try:
            ops.up = pinv(K.kernel_matrix(K.STOKES, ops.outer, ops.inner))
            ops.down = pinv(K.kernel_matrix(K.STOKES, ops.inner, ops.outer))
            return f.evaluate(pb.density[0])
        finally:
            ops.up, ops.down = keep_up, keep_dn
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    f0 = kifmm.KIFMM(pb.kernel, pb.periodic_mask, pb.p, pb.s, pb.points)
    assert f0.ops.up.Ut.shape[0] == 847 and f0.ops.down.Ut.shape[0] == 847
    default = f0.evaluate(pb.density[0])
    cut = [solve(kifmm.DEFAULT_CUTOFF, d) for d in ("gesdd", "gesvd")]
    table1 = [solve(kifmm.EPS * 888, d) for d in ("gesdd", "gesvd")]
    bare = [solve(kifmm.EPS, d) for d in ("gesdd", "gesvd")]
    assert rel(cut[0], default) < 1e-12 and rel(cut[1], cut[0]) < 3e-12
    assert 1e-11 < rel(table1[1], table1[0]) < 3e-10
    assert 1e-9 < rel(bare[1], bare[0]) < 2e-8
    e_cut, e_t1, e_bare = (rel(x[0][samp], ex) for x in (cut, table1, bare))
    assert e_cut < 0.6 * e_t1 and e_cut < 0.25 * e_bare, (e_cut, e_t1, e_bare)
