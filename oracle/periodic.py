"""Periodic kernel sums in plain numpy/scipy (oracle, FP64).

What is computed (Section 2, the problem statement and the near/far split):
  K^P(r)   = sum over the lattice P of K(r - p)
  K^{P,F}  = K^P minus the near images; here the near images are |p|_inf <= 1
             (the tree covers exactly those), so K^{P,F} sums |p|_inf >= 2.

Conventions that the paper leaves to the cited Ewald literature:
  * singly periodic (SP) Laplace: the image sum diverges like log n for one
    pair, so each image term is regularised by its monopole value,
    K(r - k e) - K(k e); for a neutral system the subtracted terms cancel.
    The paper's own route for this geometry is a direct image sum that
    converges like 1/n^2 under neutrality (Section 3, the 1D Madelung
    example); the tail beyond |k| = n is added in closed form from the
    Legendre expansion of 1/|k e -+ r|, using the Hurwitz zeta function;
  * triply periodic (TP) Stokes: Hasimoto's split of the Stokeslet with the
    k = 0 Fourier mode removed (zero mean flow, Section 3, the triply
    periodic Stokes test).  With S(r) = I/|r| + r r^T/|r|^3 (so K = S/(8 pi)):
        S^R(r) = [erfc(xi r)/r - c e^{-xi^2 r^2}] I + [erfc(xi r)/r + c e^{-xi^2 r^2}] rr^T/r^2
        S^F(r) = S(r) - S^R(r),    c = 2 xi / sqrt(pi),   S^F(0) = 2c I
        K^P(r) = sum_p S^R(r - p)/(8 pi) + sum_{k != 0} (I - k k^T/k^2) / k^2 (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)} cos(k.r)
    with k in 2 pi Z^3 (unit cell, unit viscosity);
  * triply periodic Laplace: standard Ewald with the k = 0 mode removed.
A coincident pair contributes nothing from its own singular term, but every
other image of it is kept.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import erfc, erf, zeta, eval_legendre

from .kernels import LAPLACE, STOKES, kernel_value

FOUR_PI = 4.0 * np.pi
EIGHT_PI = 8.0 * np.pi


# ---------------------------------------------------------------- singly periodic

def sp_laplace_sum(r: np.ndarray, axis: int, kmin: int = 0, n: int = 64, mterms: int = 10) -> np.ndarray:
    """Regularised singly periodic Laplace sum over images |k| >= kmin.

    Returns (1/4pi) * ( [kmin == 0] K0(r) + sum_{|k|>=max(kmin,1)} (1/|r - k e| - 1/|k|) ),
    with K0(r) = 1/|r| (0 at r = 0).  Terms with |k| <= n are summed
    directly; the rest in closed form,
        sum_{k>n} 1/|r-ke| + 1/|r+ke| - 2/k = 2 sum_m P_2m(cos t) |r|^2m zeta(2m+1, n+1).
    Requires |r| < n + 1.
    """
    r = np.asarray(r, dtype=np.float64)
    e = np.zeros(3); e[axis] = 1.0
    out = np.zeros(r.shape[:-1])
    if kmin == 0:
        r2 = np.sum(r * r, axis=-1)
        out += np.where(r2 == 0.0, 0.0, 1.0 / np.sqrt(np.where(r2 == 0.0, 1.0, r2)))
    for k in range(max(kmin, 1), n + 1):
        for sgn in (1.0, -1.0):
            d = r - sgn * k * e
            out += 1.0 / np.sqrt(np.sum(d * d, axis=-1)) - 1.0 / k
    rn = np.sqrt(np.sum(r * r, axis=-1))
    assert np.all(rn < n + 1)
    cos_t = np.where(rn == 0.0, 0.0, (r @ e) / np.where(rn == 0.0, 1.0, rn))
    for m in range(1, mterms + 1):
        out += 2.0 * eval_legendre(2 * m, cos_t) * rn ** (2 * m) * zeta(2 * m + 1, n + 1)
    return out / FOUR_PI


# ---------------------------------------------------------------- triply periodic Stokes

def _hasimoto_real(r: np.ndarray, xi: float) -> np.ndarray:
    """S^R(r) [..., 3, 3] (without the 1/(8 pi)); caller excludes r = 0."""
    rn = np.sqrt(np.sum(r * r, axis=-1))
    c = 2.0 * xi / math.sqrt(math.pi)
    g = c * np.exp(-(xi * rn) ** 2)
    ec = erfc(xi * rn) / rn
    eye = np.eye(3)
    rr = r[..., :, None] * r[..., None, :] / (rn ** 2)[..., None, None]
    return (ec - g)[..., None, None] * eye + (ec + g)[..., None, None] * rr


def _hasimoto_smooth(r: np.ndarray, xi: float) -> np.ndarray:
    """S^F(r) = S(r) - S^R(r) [..., 3, 3], smooth, with S^F(0) = (4 xi/sqrt(pi)) I."""
    rn = np.sqrt(np.sum(r * r, axis=-1))
    c = 2.0 * xi / math.sqrt(math.pi)
    small = rn < 1e-3
    rs = np.where(small, 1.0, rn)
    g = c * np.exp(-(xi * rn) ** 2)
    ef = erf(xi * rs) / rs
    # series for small r: erf(xi r)/r = c (1 - (xi r)^2/3 + (xi r)^4/10 - (xi r)^6/42 + ...)
    x2 = (xi * rn) ** 2
    ef_small = c * (1.0 - x2 / 3.0 + x2 ** 2 / 10.0 - x2 ** 3 / 42.0 + x2 ** 4 / 216.0)
    ef = np.where(small, ef_small, ef)
    # (ef - g)/r^2 for the rr term; series: c xi^2 (2/3 - 2 x2 /5 + x2^2 /7 - x2^3/27 ...)
    a_rr = np.where(small, c * xi ** 2 * (2.0 / 3.0 - 0.4 * x2 + x2 ** 2 / 7.0 - x2 ** 3 / 27.0),
                    (ef - g) / np.where(small, 1.0, rn ** 2))
    eye = np.eye(3)
    rr = r[..., :, None] * r[..., None, :]
    return (ef + g)[..., None, None] * eye + a_rr[..., None, None] * rr


def _kvectors(kmax_int: int):
    """Half of the nonzero integer vectors m with |m| <= kmax_int (one of each +-m pair)."""
    rng = np.arange(-kmax_int, kmax_int + 1)
    m = np.array(list(itertools.product(rng, rng, rng)), dtype=np.float64)
    m = m[np.sum(m * m, axis=1) <= kmax_int ** 2]
    nz = np.any(m != 0, axis=1)
    m = m[nz]
    first = np.where(m[:, 0] != 0, m[:, 0], np.where(m[:, 1] != 0, m[:, 1], m[:, 2]))
    return m[first > 0]


def _ewald_params(xi: float, tol: float = 1e-17):
    # real space: erfc(xi rho) < tol for rho > rc ; Fourier: exp(-k^2/(4 xi^2)) (1 + k^2/4xi^2) < tol
    rc = 6.2 / xi
    kc = 2.0 * xi * 6.6
    return rc, int(math.ceil(kc / (2.0 * math.pi)))


def tp_stokes_sum(r: np.ndarray, xi: float = 4.0, far_only: bool = False, exclude_self: bool = True,
                  near_layers: int = 1) -> np.ndarray:
    """Triply periodic Stokeslet (k=0 removed) at separations r [M, 3]: [M, 3, 3].

    far_only: return K^{P,F} (images |p|_inf <= near_layers removed analytically).
    exclude_self: when r == 0 exactly and not far_only, drop the singular term.
    """
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    M = r.shape[0]
    rc, kint = _ewald_params(xi)
    out = np.zeros((M, 3, 3))
    rmax = np.max(np.abs(r)) if M else 0.0
    P = int(math.ceil(rmax + rc)) + 1
    for p in itertools.product(range(-P, P + 1), repeat=3):
        p = np.array(p, dtype=np.float64)
        near = np.max(np.abs(p)) <= near_layers
        d = r - p
        dn = np.sqrt(np.sum(d * d, axis=1))
        if far_only and near:
            out -= _hasimoto_smooth(d, xi) / EIGHT_PI
            continue
        mask = dn < rc + 1e-12
        if not np.any(mask):
            continue
        zero = dn == 0.0
        sel = mask & ~zero
        if np.any(sel):
            out[sel] += _hasimoto_real(d[sel], xi) / EIGHT_PI
        if np.any(zero) and exclude_self:
            out[zero] -= _hasimoto_smooth(d[zero], xi) / EIGHT_PI
    # Fourier part over k = 2 pi m, m != 0 (pairs +-m folded into 2 cos)
    m = _kvectors(kint)
    kv = 2.0 * np.pi * m
    k2 = np.sum(kv * kv, axis=1)
    w = 2.0 * (1.0 + k2 / (4 * xi * xi)) * np.exp(-k2 / (4 * xi * xi)) / k2
    khat = kv / np.sqrt(k2)[:, None]
    cols = [w] + [w * khat[:, a] * khat[:, b] for a in range(3) for b in range(3)]
    Wm = np.stack(cols, axis=1)                 # [K, 10]
    chunk = max(1, 4_000_000 // max(1, kv.shape[0]))
    for i0 in range(0, M, chunk):
        c = np.cos(r[i0:i0 + chunk] @ kv.T)      # [m, K]
        s = c @ Wm                               # [m, 10]
        blk = -s[:, 1:].reshape(-1, 3, 3)
        blk[:, 0, 0] += s[:, 0]; blk[:, 1, 1] += s[:, 0]; blk[:, 2, 2] += s[:, 0]
        out[i0:i0 + chunk] += blk
    return out


def tp_laplace_sum(r: np.ndarray, xi: float = 4.0, far_only: bool = False, exclude_self: bool = True,
                   near_layers: int = 1) -> np.ndarray:
    """Triply periodic 1/(4 pi r) with the k = 0 mode removed: [M]."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    M = r.shape[0]
    rc, kint = _ewald_params(xi)
    out = np.full(M, -1.0 / (4.0 * xi * xi))
    rmax = np.max(np.abs(r)) if M else 0.0
    P = int(math.ceil(rmax + rc)) + 1
    c0 = 2.0 * xi / math.sqrt(math.pi)
    for p in itertools.product(range(-P, P + 1), repeat=3):
        p = np.array(p, dtype=np.float64)
        near = np.max(np.abs(p)) <= near_layers
        d = r - p
        dn = np.sqrt(np.sum(d * d, axis=1))
        zero = dn == 0.0
        ds = np.where(zero, 1.0, dn)
        smooth = np.where(zero, c0, erf(xi * ds) / ds) / FOUR_PI    # (1/r - erfc/r)/(4 pi)
        if far_only and near:
            out -= smooth
            continue
        mask = (dn < rc + 1e-12) & ~zero
        out[mask] += erfc(xi * dn[mask]) / dn[mask] / FOUR_PI
        if exclude_self:
            out[zero] -= smooth[zero]
    m = _kvectors(kint)
    kv = 2.0 * np.pi * m
    k2 = np.sum(kv * kv, axis=1)
    w = 2.0 * np.exp(-k2 / (4 * xi * xi)) / k2
    chunk = max(1, 4_000_000 // max(1, kv.shape[0]))
    for i0 in range(0, M, chunk):
        out[i0:i0 + chunk] += np.cos(r[i0:i0 + chunk] @ kv.T) @ w
    return out


# ---------------------------------------------------------------- dispatch

def periodic_axes(mask: int):
    return [a for a in range(3) if mask & (1 << a)]


def supported(kernel: int, mask: int) -> bool:
    n = len(periodic_axes(mask))
    if n == 0:
        return True
    if n == 1 and kernel == LAPLACE:
        return True
    if n == 3:
        return True
    return False


def far_kernel_matrix(kernel: int, mask: int, X: np.ndarray, Y: np.ndarray, near_layers: int = 1) -> np.ndarray:
    """Dense K^{P,F}(x_i, y_j) over images |p|_inf > near_layers: [k m, k n]."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    m, n = X.shape[0], Y.shape[0]
    r = (X[:, None, :] - Y[None, :, :]).reshape(-1, 3)
    axes = periodic_axes(mask)
    if len(axes) == 0:
        k = 1 if kernel == LAPLACE else 3
        return np.zeros((k * m, k * n))
    if kernel == LAPLACE and len(axes) == 1:
        return sp_laplace_sum(r, axes[0], kmin=near_layers + 1).reshape(m, n)
    if kernel == LAPLACE and len(axes) == 3:
        return tp_laplace_sum(r, far_only=True, near_layers=near_layers).reshape(m, n)
    if kernel == STOKES and len(axes) == 3:
        G = tp_stokes_sum(r, far_only=True, near_layers=near_layers).reshape(m, n, 3, 3)
        return G.transpose(0, 2, 1, 3).reshape(3 * m, 3 * n)
    raise NotImplementedError(f"no far-field operator for kernel {kernel}, mask {mask}")


def exact_potential(kernel: int, mask: int, targets: np.ndarray, sources: np.ndarray,
                    density: np.ndarray) -> np.ndarray:
    """The periodic sum itself at the targets (small inputs only): [T, k]."""
    targets = np.asarray(targets, dtype=np.float64)
    sources = np.asarray(sources, dtype=np.float64)
    k = 1 if kernel == LAPLACE else 3
    dens = np.asarray(density, dtype=np.float64).reshape(sources.shape[0], k)
    r = (targets[:, None, :] - sources[None, :, :]).reshape(-1, 3)
    T, S = targets.shape[0], sources.shape[0]
    axes = periodic_axes(mask)
    if len(axes) == 0:
        K = kernel_value(kernel, r)
    elif kernel == LAPLACE and len(axes) == 1:
        K = sp_laplace_sum(r, axes[0], kmin=0, n=max(64, int(np.max(np.abs(r))) + 2))
    elif kernel == LAPLACE and len(axes) == 3:
        K = tp_laplace_sum(r)
    elif kernel == STOKES and len(axes) == 3:
        K = tp_stokes_sum(r)
    else:
        raise NotImplementedError
    if kernel == LAPLACE:
        return (K.reshape(T, S) @ dens[:, 0])[:, None]
    K = K.reshape(T, S, 3, 3)
    return np.einsum("tsab,sb->ta", K, dens)
