"""Free-space kernels and surface grids, written out in plain numpy (FP64).

Kernels (Section 2, the example kernels): Laplace 1/|r| scaled to 1/(4 pi |r|),
and the Stokes velocity kernel (1/(8 pi)) (I/|r| + r r^T/|r|^3) with unit
viscosity.  A zero separation contributes nothing.

Surfaces (Section 2, the choice of check and equivalent surfaces): a regular
grid on the six faces of a cube, p points per edge including both vertices,
6(p-1)^2+2 points in total.  The order is lexicographic over the integer grid
(i, j, k) in [0, p)^3 restricted to points with some index equal to 0 or p-1.
"""
from __future__ import annotations

import numpy as np

LAPLACE = 1
STOKES = 2
INNER = 1.05   # edge of the upward-equivalent / downward-check cube, in box edges
OUTER = 2.95   # edge of the upward-check / downward-equivalent cube, in box edges


def kdim(kernel: int) -> int:
    return 1 if kernel == LAPLACE else 3


def unit_surface(p: int) -> np.ndarray:
    """Grid points on the surface of [-1, 1]^3 with p points per edge."""
    if p < 2:
        raise ValueError("p must be at least 2")
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if i in (0, p - 1) or j in (0, p - 1) or k in (0, p - 1):
                    pts.append((-1.0 + 2.0 * i / (p - 1), -1.0 + 2.0 * j / (p - 1), -1.0 + 2.0 * k / (p - 1)))
    out = np.array(pts, dtype=np.float64)
    assert out.shape[0] == 6 * (p - 1) ** 2 + 2
    return out


def box_surface(p: int, centre, edge: float, factor: float) -> np.ndarray:
    """Surface of the cube with the given centre and edge factor*edge."""
    return np.asarray(centre, dtype=np.float64)[None, :] + 0.5 * factor * edge * unit_surface(p)


def kernel_matrix(kernel: int, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Dense matrix of K(x_i - y_j): shape [k*m, k*n], row 3i+a, column 3j+b."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = X[:, None, :] - Y[None, :, :]
    r2 = np.einsum("ijc,ijc->ij", d, d)
    zero = r2 == 0.0
    r = np.sqrt(np.where(zero, 1.0, r2))
    inv = np.where(zero, 0.0, 1.0 / r)
    if kernel == LAPLACE:
        return inv / (4.0 * np.pi)
    m, n = r2.shape
    inv3 = inv ** 3
    G = np.empty((m, 3, n, 3))
    for a in range(3):
        for b in range(3):
            G[:, a, :, b] = (inv * (a == b) + d[:, :, a] * d[:, :, b] * inv3) / (8.0 * np.pi)
    return G.reshape(3 * m, 3 * n)


def kernel_value(kernel: int, r: np.ndarray) -> np.ndarray:
    """K(r) for an array of separations r [..., 3]: [...] (Laplace) or [..., 3, 3] (Stokes)."""
    r = np.asarray(r, dtype=np.float64)
    r2 = np.sum(r * r, axis=-1)
    zero = r2 == 0.0
    rn = np.sqrt(np.where(zero, 1.0, r2))
    inv = np.where(zero, 0.0, 1.0 / rn)
    if kernel == LAPLACE:
        return inv / (4.0 * np.pi)
    eye = np.eye(3)
    return (inv[..., None, None] * eye + r[..., :, None] * r[..., None, :] * (inv ** 3)[..., None, None]) / (8.0 * np.pi)
