"""Periodic kernel sums in plain numpy/scipy (oracle, FP64).

What is computed (Section 2, the problem statement and the near/far split):
  K^P(r)   = sum over the lattice P of K(r - p)
  K^{P,F}  = K^P minus the near images; here the near images are |p|_inf <= 1
             (the tree covers exactly those), so K^{P,F} sums |p|_inf >= 2.

Conventions that the paper leaves to the cited Ewald literature:
  * singly periodic (SP) Laplace and Stokes: the image sum diverges like log n for one
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
  * triply periodic Laplace: standard Ewald with the k = 0 mode removed;
  * doubly periodic (DP) Stokes and Laplace: the same real-space splits summed
    over the in-plane lattice, and the Fourier part over in-plane wave vectors
    k != 0 with the k_z integral done in closed form (below).  The k = 0 mode
    and the additive constant follow the definition of the sum itself: the
    limit of symmetric in-plane image sums, each image regularised by its
    value at the lattice point, G(r) + sum_{p != 0} [G(r - p) - G(p)]; for a
    net-force-free (or neutral) set of sources the subtracted terms cancel.
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



def sp_stokes_sum(r: np.ndarray, axis: int, kmin: int = 0, n: int = 64, mterms: int = 10) -> np.ndarray:
    """Regularised singly periodic Stokeslet sum over images |k| >= kmin: [M, 3, 3].

    Returns (1/8pi) * ( [kmin == 0] S(r) + sum_{|k|>=max(kmin,1)} (S(r - k e) - S(k e)) ) with
    S(x) = I/|x| + x x^T/|x|^3 (S(0) = 0): the limit of symmetric image sums, each image term
    regularised by its value at the lattice point; for a net-force-free set of sources the
    subtracted terms cancel.  Images with |k| <= n are summed directly.  Beyond, with
    x = k e -+ r, 1/|x| = sum_l P_l(u) rho^l / k^(l+1) and 1/|x|^3 = sum_l C_l(u) rho^l / k^(l+3)
    (Legendre P, Gegenbauer C of index 3/2; rho = |r|, u = r.e/rho), so that
        S(ke - r) + S(ke + r) - 2 S(ke) = sum_{m even >= 2} 2 k^-(m+1) Q_m(r),
        Q_m = I P_m rho^m + e e^T C_m rho^m - (e r^T + r e^T) C_{m-1} rho^(m-1) + r r^T C_{m-2} rho^(m-2),
    and the tail is sum_m 2 Q_m(r) zeta(m+1, n+1).  Requires |r| < n + 1."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    M = r.shape[0]
    e = np.zeros(3); e[axis] = 1.0
    out = np.zeros((M, 3, 3))
    if kmin == 0:
        out += kernel_value(STOKES, r) * EIGHT_PI
    for k in range(max(kmin, 1), n + 1):
        ke = k * e
        g0 = kernel_value(STOKES, ke[None, :])[0] * EIGHT_PI
        for sgn in (1.0, -1.0):
            out += kernel_value(STOKES, r - sgn * ke) * EIGHT_PI - g0
    rho = np.sqrt(np.sum(r * r, axis=1))
    assert np.all(rho < n + 1)
    u = np.where(rho > 0, (r @ e) / np.where(rho > 0, rho, 1.0), 0.0)
    L = 2 * mterms + 1
    P = [np.ones(M), u.copy()]
    C = [np.ones(M), 3.0 * u]
    for l in range(1, L):
        P.append(((2 * l + 1) * u * P[l] - l * P[l - 1]) / (l + 1))
        C.append((2.0 * u * (l + 1.5) * C[l] - (l + 2) * C[l - 1]) / (l + 1))
    ee = np.outer(e, e)
    er = e[None, :, None] * r[:, None, :] + r[:, :, None] * e[None, None, :]
    rr = r[:, :, None] * r[:, None, :]
    for mm in range(1, mterms + 1):
        m = 2 * mm
        q = (P[m] * rho ** m)[:, None, None] * np.eye(3) + (C[m] * rho ** m)[:, None, None] * ee \
            - (C[m - 1] * rho ** (m - 1))[:, None, None] * er + (C[m - 2] * rho ** (m - 2))[:, None, None] * rr
        out += 2.0 * q * zeta(m + 1, n + 1)
    return out / EIGHT_PI

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


# ---------------------------------------------------------------- doubly periodic
#
# Frame: the two periodic axes first, the free axis last (z).  For an
# in-plane wave vector k with kappa = |k| > 0 define, with
# u+- = kappa/(2 xi) +- xi z,
#     E = e^{kappa z} erfc(u+) + e^{-kappa z} erfc(u-),   D = e^{kappa z} erfc(u+) - e^{-kappa z} erfc(u-),
#     g = exp(-kappa^2/(4 xi^2) - xi^2 z^2).
# Then (1/2pi) int dk_z cos(k_z z) e^{-|k|^2/4xi^2}/|k|^2 = E/(4 kappa)           (the 2D Ewald kernel),
#      A = (1/2pi) int cos(k_z z) H/|k|^2 = E/(4 kappa) + g/(4 xi sqrt(pi)),
#      B = (1/2pi) int cos(k_z z) H/|k|^4 = -dA_0/d(kappa^2)
#        = E/(8 kappa^3) - z D/(8 kappa^2) + g/(4 xi sqrt(pi) kappa^2),      dB/dz = -z E/(8 kappa),
# with H = (1 + |k|^2/(4 xi^2)) e^{-|k|^2/(4 xi^2)} Hasimoto's screening.  The
# Stokeslet's Fourier transform 8 pi (I/|k|^2 - k k^T/|k|^4) then gives, per k,
# in-plane block 8 pi cos(k.r)(delta A - k_i k_j B), zz 8 pi cos(k.r) kappa^2 B,
# and iz, zi -8 pi sin(k.r) k_i dB/dz.  The k = 0 mode (in-plane diagonal only;
# its zz part vanishes) is T0(z) = -4 pi z erf(xi z) - (2 sqrt(pi)/xi)(e^{-xi^2 z^2} - 1)
# for Stokes and -2 pi z erf(xi z) - (2 sqrt(pi)/xi)(e^{-xi^2 z^2} - 1) for
# Laplace, i.e. the mode's divergent z-independent part removed.

def _dp_frame(mask: int):
    axes = periodic_axes(mask)
    assert len(axes) == 2
    free = [a for a in range(3) if a not in axes][0]
    return axes + [free]                       # frame index i is original axis order[i]


def _dp_kvectors(xi: float) -> np.ndarray:
    """All in-plane k = 2 pi (m1, m2) != 0 with |k| <= 2 xi * 6.7 (both signs)."""
    kmax = 2.0 * xi * 6.7
    M = int(math.ceil(kmax / (2.0 * math.pi)))
    m = np.array([(a, b) for a in range(-M, M + 1) for b in range(-M, M + 1) if (a, b) != (0, 0)], dtype=np.float64)
    kv = 2.0 * np.pi * m
    return kv[np.sqrt(np.sum(kv * kv, axis=1)) <= kmax]


def _dp_fourier(r: np.ndarray, xi: float, stokes: bool) -> np.ndarray:
    """Sum over in-plane k != 0 at separations r [M, 3] (frame order): [M, 3, 3] or [M]."""
    kv = _dp_kvectors(xi)
    kx, ky = kv[:, 0], kv[:, 1]
    kap = np.sqrt(kx * kx + ky * ky)
    M = r.shape[0]
    assert M == 0 or np.max(np.abs(r[:, 2])) * np.max(kap) < 650.0
    out = np.zeros((M, 3, 3)) if stokes else np.zeros(M)
    sp = math.sqrt(math.pi)
    chunk = max(1, 2_000_000 // max(1, kv.shape[0]))
    for i0 in range(0, M, chunk):
        rr = r[i0:i0 + chunk]
        th = rr[:, :2] @ kv.T                                   # [m, K]
        z = rr[:, 2:3]
        ep = np.exp(kap * z) * erfc(kap / (2 * xi) + xi * z)
        em = np.exp(-kap * z) * erfc(kap / (2 * xi) - xi * z)
        E = ep + em
        c = np.cos(th)
        if not stokes:
            out[i0:i0 + chunk] = FOUR_PI * np.sum(c * E / (4.0 * kap), axis=1)
            continue
        D = ep - em
        g = np.exp(-kap ** 2 / (4 * xi * xi) - (xi * z) ** 2)
        A = E / (4.0 * kap) + g / (4.0 * xi * sp)
        B = E / (8.0 * kap ** 3) - z * D / (8.0 * kap ** 2) + g / (4.0 * xi * sp * kap ** 2)
        dB = -z * E / (8.0 * kap)
        s = np.sin(th)
        o = out[i0:i0 + chunk]
        o[:, 0, 0] = EIGHT_PI * np.sum(c * (A - kx * kx * B), axis=1)
        o[:, 1, 1] = EIGHT_PI * np.sum(c * (A - ky * ky * B), axis=1)
        o[:, 0, 1] = o[:, 1, 0] = -EIGHT_PI * np.sum(c * kx * ky * B, axis=1)
        o[:, 2, 2] = EIGHT_PI * np.sum(c * kap * kap * B, axis=1)
        o[:, 0, 2] = o[:, 2, 0] = -EIGHT_PI * np.sum(s * kx * dB, axis=1)
        o[:, 1, 2] = o[:, 2, 1] = -EIGHT_PI * np.sum(s * ky * dB, axis=1)
    return out


def _dp_zero_mode(z: np.ndarray, xi: float, stokes: bool) -> np.ndarray:
    lin = (EIGHT_PI if stokes else FOUR_PI) / 2.0
    return -lin * z * erf(xi * z) - (2.0 * math.sqrt(math.pi) / xi) * (np.exp(-(xi * z) ** 2) - 1.0)


def _dp_constant(xi: float, stokes: bool):
    """C such that Ewald + C -> 0 as r -> 0 once the singular term G(r) is dropped,
    which is the value of the per-image regularised symmetric sum at r = 0."""
    rc, _ = _ewald_params(xi)
    P = int(math.ceil(rc)) + 1
    ps = np.array([(a, b, 0.0) for a in range(-P, P + 1) for b in range(-P, P + 1)
                   if (a, b) != (0, 0) and a * a + b * b < rc * rc], dtype=np.float64)
    c0 = 2.0 * xi / math.sqrt(math.pi)
    zero = np.zeros((1, 3))
    if stokes:
        return 2.0 * c0 * np.eye(3) - np.sum(_hasimoto_real(ps, xi), axis=0) - _dp_fourier(zero, xi, True)[0]
    pn = np.sqrt(np.sum(ps * ps, axis=1))
    return c0 - np.sum(erfc(xi * pn) / pn) - _dp_fourier(zero, xi, False)[0]


def _dp_sum(r: np.ndarray, mask: int, xi: float, far_only: bool, exclude_self: bool, near_layers: int,
            stokes: bool) -> np.ndarray:
    order = _dp_frame(mask)
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    rf = r[:, order]
    M = rf.shape[0]
    rc, _ = _ewald_params(xi)
    c0 = 2.0 * xi / math.sqrt(math.pi)
    out = np.zeros((M, 3, 3)) if stokes else np.zeros(M)
    P = int(math.ceil((np.max(np.abs(rf[:, :2])) if M else 0.0) + rc)) + 1
    for px, py in itertools.product(range(-P, P + 1), repeat=2):
        p = np.array([px, py, 0.0])
        near = max(abs(px), abs(py)) <= near_layers
        d = rf - p
        dn = np.sqrt(np.sum(d * d, axis=1))
        zero = dn == 0.0
        if stokes:
            if far_only and near:
                out -= _hasimoto_smooth(d, xi)
                continue
            sel = (dn < rc + 1e-12) & ~zero
            if np.any(sel):
                out[sel] += _hasimoto_real(d[sel], xi)
            if np.any(zero) and exclude_self:
                out[zero] -= _hasimoto_smooth(d[zero], xi)
        else:
            ds = np.where(zero, 1.0, dn)
            smooth = np.where(zero, c0, erf(xi * ds) / ds)
            if far_only and near:
                out -= smooth
                continue
            sel = (dn < rc + 1e-12) & ~zero
            out[sel] += erfc(xi * dn[sel]) / dn[sel]
            if exclude_self:
                out[zero] -= smooth[zero]
    out += _dp_fourier(rf, xi, stokes)
    t0 = _dp_zero_mode(rf[:, 2], xi, stokes)
    C = _dp_constant(xi, stokes)
    if stokes:
        out[:, 0, 0] += t0
        out[:, 1, 1] += t0
        out += C
        back = np.empty_like(out)
        back[:, np.array(order)[:, None], np.array(order)[None, :]] = out
        return back / EIGHT_PI
    return (out + t0 + C) / FOUR_PI


def dp_stokes_sum(r: np.ndarray, mask: int = 3, xi: float = 4.0, far_only: bool = False,
                  exclude_self: bool = True, near_layers: int = 1) -> np.ndarray:
    """Doubly periodic Stokeslet (per-image regularised, see above) at separations r: [M, 3, 3].

    mask names the two periodic axes.  far_only: only in-plane images with
    |p|_inf > near_layers (the near ones removed analytically through the smooth
    part of the split).  exclude_self: r == 0 drops its own singular term."""
    return _dp_sum(r, mask, xi, far_only, exclude_self, near_layers, True)


def dp_laplace_sum(r: np.ndarray, mask: int = 3, xi: float = 4.0, far_only: bool = False,
                   exclude_self: bool = True, near_layers: int = 1) -> np.ndarray:
    """Doubly periodic 1/(4 pi r), per-image regularised: [M]."""
    return _dp_sum(r, mask, xi, far_only, exclude_self, near_layers, False)


# ---------------------------------------------------------------- dispatch

def periodic_axes(mask: int):
    return [a for a in range(3) if mask & (1 << a)]


def supported(kernel: int, mask: int) -> bool:
    """Every kernel with free space or one, two or three periodic axes has a far-field sum."""
    return kernel in (LAPLACE, STOKES) and 0 <= mask <= 7


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
    if kernel == STOKES and len(axes) == 1:
        G = sp_stokes_sum(r, axes[0], kmin=near_layers + 1).reshape(m, n, 3, 3)
        return G.transpose(0, 2, 1, 3).reshape(3 * m, 3 * n)
    if kernel == LAPLACE and len(axes) == 3:
        return tp_laplace_sum(r, far_only=True, near_layers=near_layers).reshape(m, n)
    if kernel == STOKES and len(axes) == 3:
        G = tp_stokes_sum(r, far_only=True, near_layers=near_layers).reshape(m, n, 3, 3)
        return G.transpose(0, 2, 1, 3).reshape(3 * m, 3 * n)
    if kernel == LAPLACE and len(axes) == 2:
        return dp_laplace_sum(r, mask, far_only=True, near_layers=near_layers).reshape(m, n)
    if kernel == STOKES and len(axes) == 2:
        G = dp_stokes_sum(r, mask, far_only=True, near_layers=near_layers).reshape(m, n, 3, 3)
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
    elif kernel == STOKES and len(axes) == 1:
        K = sp_stokes_sum(r, axes[0], kmin=0, n=max(64, int(np.max(np.abs(r))) + 2))
    elif kernel == LAPLACE and len(axes) == 3:
        K = tp_laplace_sum(r)
    elif kernel == STOKES and len(axes) == 3:
        K = tp_stokes_sum(r)
    elif kernel == LAPLACE and len(axes) == 2:
        K = dp_laplace_sum(r, mask)
    elif kernel == STOKES and len(axes) == 2:
        K = dp_stokes_sum(r, mask)
    else:
        raise NotImplementedError
    if kernel == LAPLACE:
        return (K.reshape(T, S) @ dens[:, 0])[:, None]
    K = K.reshape(T, S, 3, 3)
    return np.einsum("tsab,sb->ta", K, dens)
