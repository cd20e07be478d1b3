"""Seeded synthetic workloads for the periodic KIFMM evaluation pass.

This module only draws random numbers: point clouds and densities with the
shapes and distributions of the evaluated configurations.  It holds none of the
method's arithmetic and is shared by the oracle, the tests and the benchmark so
that every side sees the same inputs.

All draws use ``numpy.random.default_rng(seed)`` (PCG64) in float64 and in the
order written below; changing the order changes the workload.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

LAPLACE = 1
STOKES = 2
PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4
SP_X = PERIODIC_X
DP_XY = PERIODIC_X | PERIODIC_Y
TP = PERIODIC_X | PERIODIC_Y | PERIODIC_Z


@dataclasses.dataclass
class Problem:
    """One periodic sum problem: points (sources = targets) and densities."""
    name: str
    kernel: int            # LAPLACE (k=1) or STOKES (k=3)
    periodic_mask: int     # bit 0: x, bit 1: y, bit 2: z
    p: int                 # surface points per cube edge
    s: int                 # maximum points per leaf
    points: np.ndarray     # [N, 3] float64 in the unit box
    density: np.ndarray    # [R, N, k] float64

    @property
    def k(self) -> int:
        return 1 if self.kernel == LAPLACE else 3

    @property
    def n(self) -> int:
        return self.points.shape[0]


def laplace_sp_uniform(n: int = 2000, seed: int = 1, p: int = 8, s: int = 50,
                       n_rhs: int = 1, mask: int = SP_X) -> Problem:
    """Uniform points in the unit cube, charges uniform in [-1, 1] made neutral.

    With the defaults this is the small Laplace singly periodic workload
    (N=2000, p=8, at most 50 points per leaf).
    """
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, (n_rhs, n))
    q -= q.mean(axis=1, keepdims=True)
    return Problem(f"laplace_mask{mask}_n{n}", LAPLACE, mask, p, s, pts, q[:, :, None].copy())


def stokes_tp_uniform(n: int = 1_000_000, seed: int = 2, p: int = 8, s: int = 2000,
                      n_rhs: int = 1, mask: int = TP) -> Problem:
    """Uniform points, i.i.d. N(0,1) force components made force-free.

    With the defaults this is the Stokes triply periodic workload at N=1M,
    p=8, at most 2000 points per leaf.
    """
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    f = rng.standard_normal((n_rhs, n, 3))
    f -= f.mean(axis=1, keepdims=True)
    return Problem(f"stokes_mask{mask}_n{n}", STOKES, mask, p, s, pts, f)


def stokes_dp_slab(n: int = 4_000_000, seed: int = 3, p: int = 10, s: int = 2000,
                   n_rhs: int = 1) -> Problem:
    """x, y uniform; z ~ N(0.5, 0.1) clipped to [0, 1]; force-free Gaussian forces."""
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    z = np.clip(rng.normal(0.5, 0.1, n), 0.0, 1.0)
    pts = np.column_stack([xy, z])
    f = rng.standard_normal((n_rhs, n, 3))
    f -= f.mean(axis=1, keepdims=True)
    return Problem(f"stokes_dp_n{n}", STOKES, DP_XY, p, s, pts, f)


def laplace_sp_batch(n_problems: int = 64, n_rhs: int = 16, p: int = 8, s: int = 2000,
                     base_seed: int = 4000, lo: float = 4.0, hi: float = 6.0) -> List[Problem]:
    """Independent Laplace singly periodic problems, N log-uniform in [10^lo, 10^hi]."""
    out = []
    for i in range(n_problems):
        rng = np.random.default_rng(base_seed + i)
        n = int(round(10.0 ** rng.uniform(lo, hi)))
        pts = rng.random((n, 3))
        q = rng.uniform(-1.0, 1.0, (n_rhs, n))
        q -= q.mean(axis=1, keepdims=True)
        out.append(Problem(f"laplace_batch{i}_n{n}", LAPLACE, SP_X, p, s, pts, q[:, :, None].copy()))
    return out


def stokes_tp_clustered(n: int = 16_000_000, seed: int = 5, p: int = 12, s: int = 2000,
                        n_rhs: int = 4, n_centres: int = 200, sigma: float = 0.02) -> Problem:
    """200 Gaussian clusters (80 % of points, wrapped) plus 20 % uniform background."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_centres, 3))
    n_cl = int(round(0.8 * n))
    pick = rng.integers(0, n_centres, n_cl)
    cl = np.mod(centres[pick] + rng.normal(0.0, sigma, (n_cl, 3)), 1.0)
    cl[cl >= 1.0] = 0.0
    bg = rng.random((n - n_cl, 3))
    pts = np.concatenate([cl, bg], axis=0)
    f = rng.standard_normal((n_rhs, n, 3))
    f -= f.mean(axis=1, keepdims=True)
    return Problem(f"stokes_tp_clustered_n{n}", STOKES, TP, p, s, pts, f)


def clenshaw_curtis_nodes(m: int = 97) -> np.ndarray:
    """The m Clenshaw-Curtis (Chebyshev extreme) nodes mapped to [0, 1], endpoints included."""
    return 0.5 * (1.0 - np.cos(np.pi * np.arange(m) / (m - 1)))


def stokes_paper_points(kind: str, mask: int = TP, p: int = 8, s: int = 1000, m: int = 97) -> Problem:
    """The timing workloads of Section 3.5: m^3 = 912673 points for m = 97,
    sources = targets, one force per point with components uniform in [-0.5, 0.5), made
    force-free (mean subtracted) for singly and doubly periodic sums; at most 1000 points per
    leaf.

    kind = "chebyshev": the tensor grid of Clenshaw-Curtis nodes, the paper's uniform set
    (forces seed 6).
    kind = "lognormal": each coordinate drawn from numpy's lognormal(mean=0.2, sigma=0.5) and
    taken modulo 1 into the unit box, the paper's non-uniform set (how its lognormal samples
    are placed in the box is not stated; seed 7, points first, then forces).
    """
    n = m ** 3
    if kind == "chebyshev":
        rng = np.random.default_rng(6)
        c = clenshaw_curtis_nodes(m)
        pts = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(n, 3)
    elif kind == "lognormal":
        rng = np.random.default_rng(7)
        pts = np.mod(rng.lognormal(0.2, 0.5, (n, 3)), 1.0)
    else:
        raise ValueError(kind)
    f = rng.uniform(-0.5, 0.5, (1, n, 3))
    naxes = bin(mask).count("1")
    if naxes in (1, 2):
        f -= f.mean(axis=1, keepdims=True)
    return Problem(f"stokes_paper_{kind}_mask{mask}_n{n}", STOKES, mask, p, s, np.ascontiguousarray(pts), f)


def madelung_chain(axis: int = 0):
    """Four alternating unit charges on a line along ``axis`` at 1/8, 3/8, 5/8, 7/8."""
    pts = np.full((4, 3), 0.5)
    pts[:, axis] = [0.125, 0.375, 0.625, 0.875]
    q = np.array([1.0, -1.0, 1.0, -1.0])
    return pts, q


def two_point_forces():
    """Two opposite point forces: x1=(0.7,0.6,0.5), f1=(1,2,3)/sqrt(14); x2=(0.2,0.8,0.7), f2=-f1."""
    f1 = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    pts = np.array([[0.7, 0.6, 0.5], [0.2, 0.8, 0.7]])
    f = np.stack([f1, -f1])
    return pts, f


def one_point_force():
    """A single point force at (0.7,0.6,0.4) with f=(1,2,3)/sqrt(14) (net force is not zero)."""
    return np.array([[0.7, 0.6, 0.4]]), (np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0))[None, :]
