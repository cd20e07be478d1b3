// Operator construction (Algorithm 2, Stage 1) in float64 on the device:
// kernel matrices between surface grids, the periodic far-field kernel
// K^{P,F} over images |p|_inf > l (l = 1 by default; 2 and 3 for singly and triply
// periodic sums, Section 3.6's near-field layer), and the split SVD factors of the
// check-to-equivalent solves.  Raw kernels throughout (1/|r| and
// I/|r| + r r^T/|r|^3); the 1/(4 pi), 1/(8 pi) factors are applied to the
// final potentials.
//
// Periodic far-field kernels (the paper leaves the periodic sums to the
// Ewald literature; the conventions used here):
//   * singly periodic Laplace and Stokes along axis e: each image term is regularised by
//     its value at the lattice point, sum_{|k|>=2} K(r - k e) - K(k e); images up to
//     |k| = kNear are summed directly and the rest in closed form from the
//     Legendre (and for Stokes also Gegenbauer) expansions with Hurwitz zeta sums;
//   * triply periodic Stokes: Hasimoto's split with the k = 0 mode removed;
//     real-space part S^R over the far images, Fourier part over k != 0, and
//     the near images |p|_inf <= 1 removed analytically by subtracting the
//     smooth part S^F = S - S^R (finite at r = 0, where it equals 4 xi/sqrt(pi) I);
//   * triply periodic Laplace: Ewald with the k = 0 mode removed, near images
//     removed the same way;
//   * doubly periodic Stokes and Laplace: the same splits over the in-plane
//     lattice; each in-plane Fourier mode k != 0 has its k_z integral in closed
//     form (erfc terms), the k = 0 mode keeps its z-dependent part, and a
//     constant makes the sum equal the limit of symmetric image sums
//     regularised per image by the kernel's value at the lattice point.
#include <cmath>
#include <vector>

#include "launch.h"

namespace pk {

namespace {

constexpr int kNear = 40;       // SP: images |k| <= kNear summed directly
constexpr int kLegendre = 12;   // SP: tail terms
constexpr double kXi = 3.5;     // TP Ewald splitting parameter

__global__ void k_kmat(int kernel, const double* __restrict__ X, int m, const double* __restrict__ Y, int n,
                       double* __restrict__ out, int64_t ld) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;   // target point
    int j = blockIdx.y;                               // source point
    if (i >= m) return;
    double dx = X[3 * i] - Y[3 * j], dy = X[3 * i + 1] - Y[3 * j + 1], dz = X[3 * i + 2] - Y[3 * j + 2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double ri = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    if (kernel == PKIFMM_LAPLACE) {
        out[i + (int64_t)j * ld] = ri;
        return;
    }
    double d[3] = {dx, dy, dz};
    double ri3 = ri * ri * ri;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            out[(3 * i + a) + (int64_t)(3 * j + b) * ld] = (a == b ? ri : 0.0) + d[a] * d[b] * ri3;
}

// ---- singly periodic Laplace
__global__ void k_far_sp_laplace(int axis, const double* __restrict__ X, int m, const double* __restrict__ Y, int n,
                                 double* __restrict__ out, int64_t ld, const double* __restrict__ zeta, int near) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= m) return;
    double r[3] = {X[3 * i] - Y[3 * j], X[3 * i + 1] - Y[3 * j + 1], X[3 * i + 2] - Y[3 * j + 2]};
    double acc = 0.0;
    for (int k = kNear; k >= near + 1; --k) {   // small terms first
        double rp[3] = {r[0], r[1], r[2]}, rm[3] = {r[0], r[1], r[2]};
        rp[axis] -= k;
        rm[axis] += k;
        double a = 1.0 / sqrt(rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]);
        double b = 1.0 / sqrt(rm[0] * rm[0] + rm[1] * rm[1] + rm[2] * rm[2]);
        acc += (a - 1.0 / k) + (b - 1.0 / k);
    }
    double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = sqrt(rr);
    double ct = rn > 0.0 ? r[axis] / rn : 0.0;
    // Legendre recurrence up to order 2*kLegendre
    double pm1 = 1.0, p0 = ct, tail = 0.0, rpow = 1.0;
    for (int l = 1; l < 2 * kLegendre; ++l) {
        double pn = ((2 * l + 1) * ct * p0 - l * pm1) / (l + 1);
        pm1 = p0;
        p0 = pn;
        if ((l + 1) % 2 == 0) {
            int mm = (l + 1) / 2;
            rpow *= rr;
            tail += 2.0 * pn * rpow * zeta[mm - 1];
        }
    }
    out[i + (int64_t)j * ld] = acc + tail;
}

// ---- singly periodic Stokes, same regularisation; tail from the Legendre (1/|x|) and index-3/2
// Gegenbauer (1/|x|^3) expansions: for x = k e -+ r,
//   S(ke - r) + S(ke + r) - 2 S(ke) = sum_{m even >= 2} 2 k^-(m+1) Q_m(r),
//   Q_m = I P_m rho^m + e e^T C_m rho^m - (e r^T + r e^T) C_{m-1} rho^(m-1) + r r^T C_{m-2} rho^(m-2)
// (rho = |r|, u = r.e/rho), summed against zeta(m+1, kNear+1).
__global__ void k_far_sp_stokes(int axis, const double* __restrict__ X, int m, const double* __restrict__ Y, int n,
                                double* __restrict__ out, int64_t ld, const double* __restrict__ zeta, int near) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= m) return;
    const double r[3] = {X[3 * i] - Y[3 * j], X[3 * i + 1] - Y[3 * j + 1], X[3 * i + 2] - Y[3 * j + 2]};
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = kNear; k >= near + 1; --k) {   // small terms first
        for (int sg = -1; sg <= 1; sg += 2) {
            double d[3] = {r[0], r[1], r[2]};
            d[axis] -= sg * k;
            const double ri = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double ri3 = ri * ri * ri;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    // S(d) - S(k e): S(k e) = (I + e e^T) / k
                    const double s0 = ((p == q ? 1.0 : 0.0) + (p == axis && q == axis ? 1.0 : 0.0)) / k;
                    A[p][q] += ((p == q ? ri : 0.0) + d[p] * d[q] * ri3) - s0;
                }
        }
    }
    const double rho2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double rho = sqrt(rho2);
    const double u = rho > 0.0 ? r[axis] / rho : 0.0;
    // P_l and C_l (index 3/2) by their three-term recurrences, with the powers of rho folded in:
    // pl[l] = P_l(u) rho^l, cl[l] = C_l(u) rho^l
    double pl[2 * kLegendre + 1], cl[2 * kLegendre + 1];
    pl[0] = 1.0; pl[1] = u * rho;
    cl[0] = 1.0; cl[1] = 3.0 * u * rho;
    for (int l = 1; l < 2 * kLegendre; ++l) {
        pl[l + 1] = ((2 * l + 1) * u * rho * pl[l] - l * rho2 * pl[l - 1]) / (l + 1);
        cl[l + 1] = (2.0 * u * rho * (l + 1.5) * cl[l] - (l + 2) * rho2 * cl[l - 1]) / (l + 1);
    }
    for (int mm = 1; mm <= kLegendre; ++mm) {
        const int mo = 2 * mm;
        const double z = 2.0 * zeta[mm - 1];
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                const double e_p = p == axis ? 1.0 : 0.0, e_q = q == axis ? 1.0 : 0.0;
                double qv = (p == q ? pl[mo] : 0.0) + e_p * e_q * cl[mo] - (e_p * r[q] + r[p] * e_q) * cl[mo - 1] +
                            r[p] * r[q] * cl[mo - 2];
                A[p][q] += z * qv;
            }
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) out[(3 * i + p) + (int64_t)(3 * j + q) * ld] = A[p][q];
}

// ---- triply periodic Stokes (Hasimoto)
__device__ void hasimoto_real(const double d[3], double rn, double xi, double S[3][3]) {
    const double c = 2.0 * xi / sqrt(M_PI);
    double g = c * exp(-xi * xi * rn * rn);
    double ec = erfc(xi * rn) / rn;
    double a = ec - g, b = (ec + g) / (rn * rn);
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) S[p][q] = (p == q ? a : 0.0) + b * d[p] * d[q];
}

__device__ void hasimoto_smooth(const double d[3], double rn, double xi, double S[3][3]) {
    const double c = 2.0 * xi / sqrt(M_PI);
    double x2 = xi * xi * rn * rn;
    double g = c * exp(-x2);
    double ef, arr;
    if (rn < 1e-3) {
        ef = c * (1.0 - x2 / 3.0 + x2 * x2 / 10.0 - x2 * x2 * x2 / 42.0);
        arr = c * xi * xi * (2.0 / 3.0 - 0.4 * x2 + x2 * x2 / 7.0);
    } else {
        ef = erf(xi * rn) / rn;
        arr = (ef - g) / (rn * rn);
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) S[p][q] = (p == q ? ef + g : 0.0) + arr * d[p] * d[q];
}

__global__ void k_far_tp_stokes(const double* __restrict__ X, int m, const double* __restrict__ Y, int n,
                                double* __restrict__ out, int64_t ld, const double4* __restrict__ kv, int nk,
                                double rc, int P, int near) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= m) return;
    const double xi = kXi;
    double r[3] = {X[3 * i] - Y[3 * j], X[3 * i + 1] - Y[3 * j + 1], X[3 * i + 2] - Y[3 * j + 2]};
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double S[3][3];
    for (int px = -P; px <= P; ++px)
        for (int py = -P; py <= P; ++py)
            for (int pz = -P; pz <= P; ++pz) {
                double d[3] = {r[0] - px, r[1] - py, r[2] - pz};
                double rn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                int pin = max(abs(px), max(abs(py), abs(pz)));
                if (pin <= near) {
                    hasimoto_smooth(d, rn, xi, S);
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) A[p][q] -= S[p][q];
                } else if (rn < rc) {
                    hasimoto_real(d, rn, xi, S);
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) A[p][q] += S[p][q];
                }
            }
    // Fourier part: kv = (kx, ky, kz, weight) over half the lattice, weight includes the pair
    double f0 = 0.0, f[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int t = nk - 1; t >= 0; --t) {    // small terms first
        double4 k = kv[t];
        double cw = k.w * cos(k.x * r[0] + k.y * r[1] + k.z * r[2]);
        double kk = k.x * k.x + k.y * k.y + k.z * k.z;
        double kh[3] = {k.x, k.y, k.z};
        f0 += cw;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) f[p][q] += cw * kh[p] * kh[q] / kk;
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double v = A[p][q] + (p == q ? f0 : 0.0) - f[p][q];
            out[(3 * i + p) + (int64_t)(3 * j + q) * ld] = v;
        }
}

// ---- triply periodic Laplace
__global__ void k_far_tp_laplace(const double* __restrict__ X, int m, const double* __restrict__ Y, int n,
                                 double* __restrict__ out, int64_t ld, const double4* __restrict__ kv, int nk,
                                 double rc, int P, int near) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= m) return;
    const double xi = kXi;
    const double c = 2.0 * xi / sqrt(M_PI);
    double r[3] = {X[3 * i] - Y[3 * j], X[3 * i + 1] - Y[3 * j + 1], X[3 * i + 2] - Y[3 * j + 2]};
    double acc = -M_PI / (xi * xi);
    for (int px = -P; px <= P; ++px)
        for (int py = -P; py <= P; ++py)
            for (int pz = -P; pz <= P; ++pz) {
                double d[3] = {r[0] - px, r[1] - py, r[2] - pz};
                double rn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                int pin = max(abs(px), max(abs(py), abs(pz)));
                if (pin <= near) acc -= rn > 0.0 ? erf(xi * rn) / rn : c;
                else if (rn < rc) acc += erfc(xi * rn) / rn;
            }
    double fs = 0.0;
    for (int t = nk - 1; t >= 0; --t) {
        double4 k = kv[t];
        fs += k.w * cos(k.x * r[0] + k.y * r[1] + k.z * r[2]);
    }
    out[i + (int64_t)j * ld] = acc + fs;
}

// ---- doubly periodic.  Frame: periodic axes f0, f1, free axis f2.  For an in-plane
// wave vector of length kap and u+- = kap/(2 xi) +- xi z:
//   E = e^{kap z} erfc(u+) + e^{-kap z} erfc(u-),   D = e^{kap z} erfc(u+) - e^{-kap z} erfc(u-),
//   g = exp(-kap^2/(4 xi^2) - xi^2 z^2),
//   A = E/(4 kap) + g/(4 xi sqrt(pi)),  B = E/(8 kap^3) - z D/(8 kap^2) + g/(4 xi sqrt(pi) kap^2),
//   dB/dz = -z E/(8 kap).
// Stokes per mode: in-plane 8 pi cos(k.r)(delta_ij A - k_i k_j B), zz 8 pi cos(k.r) kap^2 B,
// iz and zi -8 pi sin(k.r) k_i dB/dz.  Laplace per mode: 4 pi cos(k.r) E/(4 kap).
// k = 0 mode on the in-plane diagonal (Stokes) or the scalar (Laplace):
//   -c z erf(xi z) - (2 sqrt(pi)/xi)(e^{-xi^2 z^2} - 1),  c = 4 pi (Stokes), 2 pi (Laplace).
__global__ void k_far_dp(int stokes, int f0, int f1, int f2, const double* __restrict__ X, int m,
                         const double* __restrict__ Y, int n, double* __restrict__ out, int64_t ld,
                         const double2* __restrict__ kv, int nk, double rc, int P, double c_par, double c_z) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= m) return;
    const double xi = kXi;
    const double sp = sqrt(M_PI);
    const double c0 = 2.0 * xi / sp;
    const int fr[3] = {f0, f1, f2};
    double r[3];
    for (int a = 0; a < 3; ++a) r[a] = X[3 * i + fr[a]] - Y[3 * j + fr[a]];
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double acc = 0.0;                  // Laplace
    double S[3][3];
    for (int px = -P; px <= P; ++px)
        for (int py = -P; py <= P; ++py) {
            double d[3] = {r[0] - px, r[1] - py, r[2]};
            double rn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const bool near = max(abs(px), abs(py)) <= 1;
            if (stokes) {
                if (near) {
                    hasimoto_smooth(d, rn, xi, S);
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) A[p][q] -= S[p][q];
                } else if (rn < rc) {
                    hasimoto_real(d, rn, xi, S);
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) A[p][q] += S[p][q];
                }
            } else {
                if (near) acc -= rn > 0.0 ? erf(xi * rn) / rn : c0;
                else if (rn < rc) acc += erfc(xi * rn) / rn;
            }
        }
    // Fourier part: kv holds one of each +-k pair; both members contribute the same
    const double z = r[2];
    double fxx = 0, fyy = 0, fxy = 0, fzz = 0, fxz = 0, fyz = 0, fl = 0;
    for (int t = nk - 1; t >= 0; --t) {      // small terms first
        const double kx = kv[t].x, ky = kv[t].y;
        const double kap = sqrt(kx * kx + ky * ky);
        double sn, cs;
        sincos(kx * r[0] + ky * r[1], &sn, &cs);
        const double ep = exp(kap * z) * erfc(kap / (2.0 * xi) + xi * z);
        const double em = exp(-kap * z) * erfc(kap / (2.0 * xi) - xi * z);
        const double E = ep + em;
        if (!stokes) {
            fl += cs * E / kap;
            continue;
        }
        const double D = ep - em;
        const double g = exp(-kap * kap / (4.0 * xi * xi) - xi * xi * z * z);
        const double Av = E / (4.0 * kap) + g / (4.0 * xi * sp);
        const double Bv = E / (8.0 * kap * kap * kap) - z * D / (8.0 * kap * kap) + g / (4.0 * xi * sp * kap * kap);
        const double dB = -z * E / (8.0 * kap);
        fxx += cs * (Av - kx * kx * Bv);
        fyy += cs * (Av - ky * ky * Bv);
        fxy -= cs * kx * ky * Bv;
        fzz += cs * kap * kap * Bv;
        fxz -= sn * kx * dB;
        fyz -= sn * ky * dB;
    }
    const double t0 = -(stokes ? 4.0 : 2.0) * M_PI * z * erf(xi * z) - (2.0 * sp / xi) * (exp(-xi * xi * z * z) - 1.0);
    if (!stokes) {
        out[i + (int64_t)j * ld] = acc + 2.0 * M_PI * fl + t0 + c_par;   // 2 x (4 pi / 4) per +-k pair
        return;
    }
    const double w = 2.0 * 8.0 * M_PI;
    const double F[3][3] = {{w * fxx + t0 + c_par, w * fxy, w * fxz},
                            {w * fxy, w * fyy + t0 + c_par, w * fyz},
                            {w * fxz, w * fyz, w * fzz + c_z}};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
            out[(3 * i + fr[p]) + (int64_t)(3 * j + fr[q]) * ld] = A[p][q] + F[p][q];
}

__global__ void k_pinv_factors(const double* __restrict__ U, const double* __restrict__ Vt,
                               const double* __restrict__ S, int kn, int r, double* __restrict__ Ut_r,
                               double* __restrict__ VS) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;   // 0..kn-1
    int i = blockIdx.y;                               // 0..r-1
    if (j >= kn) return;
    Ut_r[i + (int64_t)j * r] = U[j + (int64_t)i * kn];
    VS[j + (int64_t)i * kn] = Vt[i + (int64_t)j * kn] / S[i];
}

// Hurwitz zeta(s, a) = sum_{k>=0} (k + a)^-s for a > 1, s > 1: ten terms summed
// directly, the rest by Euler-Maclaurin with Bernoulli numbers B2..B12.
double hurwitz_zeta(double s, double a) {
    double sum = 0.0;
    const int M = 10;
    for (int k = M - 1; k >= 0; --k) sum += std::pow(a + k, -s);
    double b = a + M;
    sum += std::pow(b, 1.0 - s) / (s - 1.0) + 0.5 * std::pow(b, -s);
    const double B[6] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730};
    double fact = 1.0, rising = s;   // (2j)! and s(s+1)...(s+2j-2)
    double term_pow = std::pow(b, -s - 1.0);
    for (int j = 1; j <= 6; ++j) {
        fact *= (2.0 * j - 1.0) * (2.0 * j);
        sum += B[j - 1] / fact * rising * term_pow;
        rising *= (s + 2.0 * j - 1.0) * (s + 2.0 * j);
        term_pow /= b * b;
    }
    return sum;
}

// half of the nonzero k = 2 pi m with |k| <= kmax, weights for the Fourier sums
std::vector<double> kvectors(double kmax, bool stokes) {
    std::vector<double> out;
    int M = (int)std::ceil(kmax / (2.0 * M_PI));
    const double xi2 = kXi * kXi;
    for (int a = -M; a <= M; ++a)
        for (int b = -M; b <= M; ++b)
            for (int c = -M; c <= M; ++c) {
                int first = a != 0 ? a : (b != 0 ? b : c);
                if (first <= 0) continue;
                double kx = 2 * M_PI * a, ky = 2 * M_PI * b, kz = 2 * M_PI * c;
                double k2 = kx * kx + ky * ky + kz * kz;
                if (k2 > kmax * kmax) continue;
                double e = std::exp(-k2 / (4 * xi2));
                // two of each +-k pair; 8 pi (Stokes) or 4 pi (Laplace) undoes the kernel factor
                double w = stokes ? 2.0 * 8.0 * M_PI * (1.0 + k2 / (4 * xi2)) * e / k2 : 2.0 * 4.0 * M_PI * e / k2;
                out.insert(out.end(), {kx, ky, kz, w});
            }
    return out;
}

// in-plane k = 2 pi (a, b), one of each +-k pair, |k| <= kmax
std::vector<double> kvectors_2d(double kmax) {
    std::vector<double> out;
    int M = (int)std::ceil(kmax / (2.0 * M_PI));
    for (int a = -M; a <= M; ++a)
        for (int b = -M; b <= M; ++b) {
            int first = a != 0 ? a : b;
            if (first <= 0) continue;
            double kx = 2 * M_PI * a, ky = 2 * M_PI * b;
            if (kx * kx + ky * ky > kmax * kmax) continue;
            out.insert(out.end(), {kx, ky});
        }
    return out;
}

// Constant of the doubly periodic sum (frame diagonal: in-plane c_par, free axis c_z):
// the Ewald form plus this constant vanishes at r -> 0 once the singular term is dropped,
// as the per-image regularised symmetric sum does there.
void dp_constant(bool stokes, double rc, const std::vector<double>& kv, double& c_par, double& c_z) {
    const double xi = kXi, sp = std::sqrt(M_PI), c0 = 2.0 * xi / sp;
    double rs_par = 0.0, rs_z = 0.0;     // sum over in-plane p != 0 of the real-space split
    int P = (int)std::ceil(rc) + 1;
    for (int a = -P; a <= P; ++a)
        for (int b = -P; b <= P; ++b) {
            if ((a == 0 && b == 0) || a * a + b * b >= rc * rc) continue;
            double rn = std::sqrt((double)(a * a + b * b));
            double ec = std::erfc(xi * rn) / rn;
            if (!stokes) { rs_par += ec; continue; }
            double g = c0 * std::exp(-xi * xi * rn * rn);
            rs_par += (ec - g) + (ec + g) * (double)(a * a) / (rn * rn);
            rs_z += ec - g;
        }
    double f_par = 0.0, f_z = 0.0;       // Fourier part at r = 0 (both members of each pair)
    for (size_t t = 0; t < kv.size() / 2; ++t) {
        double kx = kv[2 * t], ky = kv[2 * t + 1];
        double kap = std::sqrt(kx * kx + ky * ky);
        double E = 2.0 * std::erfc(kap / (2.0 * xi));
        if (!stokes) { f_par += 2.0 * M_PI * E / kap; continue; }
        double g = std::exp(-kap * kap / (4.0 * xi * xi));
        double Av = E / (4.0 * kap) + g / (4.0 * xi * sp);
        double Bv = E / (8.0 * kap * kap * kap) + g / (4.0 * xi * sp * kap * kap);
        f_par += 2.0 * 8.0 * M_PI * (Av - kx * kx * Bv);
        f_z += 2.0 * 8.0 * M_PI * kap * kap * Bv;
    }
    if (!stokes) {
        c_par = c0 - rs_par - f_par;
        c_z = 0.0;
        return;
    }
    c_par = 2.0 * c0 - rs_par - f_par;
    c_z = 2.0 * c0 - rs_z - f_z;
}

}  // namespace

void launch_kmat(int kernel, const double* X, int m, const double* Y, int n, double* out, int64_t ld,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_kmat, dim3((m + 127) / 128, n), dim3(128), 0, s, kernel, X, m, Y, n, out, ld);
    PK_HIP(hipGetLastError());
}

void launch_far_kmat(int kernel, unsigned mask, const double* X, int m, const double* Y, int n, double* out,
                     int64_t ld, int near, hipStream_t s) {
    int naxes = __builtin_popcount(mask & 7u);
    dim3 grid((m + 127) / 128, n);
    if (naxes == 1) {
        int axis = mask & 1u ? 0 : (mask & 2u ? 1 : 2);
        std::vector<double> z(kLegendre);
        for (int mm = 1; mm <= kLegendre; ++mm) z[mm - 1] = hurwitz_zeta(2.0 * mm + 1.0, kNear + 1.0);
        DBuf<double> dz;
        dz.upload(z, s);
        if (kernel == PKIFMM_LAPLACE)
            hipLaunchKernelGGL(k_far_sp_laplace, grid, dim3(128), 0, s, axis, X, m, Y, n, out, ld, dz.p, near);
        else
            hipLaunchKernelGGL(k_far_sp_stokes, grid, dim3(128), 0, s, axis, X, m, Y, n, out, ld, dz.p, near);
        PK_HIP(hipGetLastError());
        PK_HIP(hipStreamSynchronize(s));
        return;
    }
    if (naxes == 3) {
        // real space: erfc(xi rho) < 1e-18 beyond rc; Fourier: (1+k^2/4xi^2) e^{-k^2/4xi^2} < 1e-18 beyond kmax
        const double rc = 6.3 / kXi;
        const double kmax = 2.0 * kXi * 6.7;
        double rmax = 0.0;
        std::vector<double> hx(3 * (size_t)m), hy(3 * (size_t)n);
        PK_HIP(hipMemcpyAsync(hx.data(), X, hx.size() * 8, hipMemcpyDeviceToHost, s));
        PK_HIP(hipMemcpyAsync(hy.data(), Y, hy.size() * 8, hipMemcpyDeviceToHost, s));
        PK_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < 3; ++c) {
            double xlo = 1e300, xhi = -1e300, ylo = 1e300, yhi = -1e300;
            for (int i = 0; i < m; ++i) { xlo = std::min(xlo, hx[3 * i + c]); xhi = std::max(xhi, hx[3 * i + c]); }
            for (int j = 0; j < n; ++j) { ylo = std::min(ylo, hy[3 * j + c]); yhi = std::max(yhi, hy[3 * j + c]); }
            rmax = std::max(rmax, std::max(std::fabs(xhi - ylo), std::fabs(xlo - yhi)));
        }
        int P = std::max((int)std::ceil(rmax + rc) + 1, near);
        std::vector<double> kv = kvectors(kmax, kernel == PKIFMM_STOKES);
        DBuf<double> dk;
        dk.upload(kv, s);
        int nk = (int)(kv.size() / 4);
        if (kernel == PKIFMM_STOKES)
            hipLaunchKernelGGL(k_far_tp_stokes, grid, dim3(128), 0, s, X, m, Y, n, out, ld, (const double4*)dk.p, nk,
                               rc, P, near);
        else
            hipLaunchKernelGGL(k_far_tp_laplace, grid, dim3(128), 0, s, X, m, Y, n, out, ld, (const double4*)dk.p,
                               nk, rc, P, near);
        PK_HIP(hipGetLastError());
        PK_HIP(hipStreamSynchronize(s));
        return;
    }
    if (naxes == 2) {
        int fr[3], nf = 0;
        for (int a = 0; a < 3; ++a)
            if (mask & (1u << a)) fr[nf++] = a;
        for (int a = 0; a < 3; ++a)
            if (!(mask & (1u << a))) fr[2] = a;
        const double rc = 6.3 / kXi;
        const double kmax = 2.0 * kXi * 6.7;
        std::vector<double> hx(3 * (size_t)m), hy(3 * (size_t)n);
        PK_HIP(hipMemcpyAsync(hx.data(), X, hx.size() * 8, hipMemcpyDeviceToHost, s));
        PK_HIP(hipMemcpyAsync(hy.data(), Y, hy.size() * 8, hipMemcpyDeviceToHost, s));
        PK_HIP(hipStreamSynchronize(s));
        double rmax = 0.0;
        for (int c = 0; c < 2; ++c) {
            double xlo = 1e300, xhi = -1e300, ylo = 1e300, yhi = -1e300;
            for (int i = 0; i < m; ++i) { xlo = std::min(xlo, hx[3 * i + fr[c]]); xhi = std::max(xhi, hx[3 * i + fr[c]]); }
            for (int j = 0; j < n; ++j) { ylo = std::min(ylo, hy[3 * j + fr[c]]); yhi = std::max(yhi, hy[3 * j + fr[c]]); }
            rmax = std::max(rmax, std::max(std::fabs(xhi - ylo), std::fabs(xlo - yhi)));
        }
        const int P = (int)std::ceil(rmax + rc) + 1;
        std::vector<double> kv = kvectors_2d(kmax);
        double c_par, c_z;
        dp_constant(kernel == PKIFMM_STOKES, rc, kv, c_par, c_z);
        DBuf<double> dk;
        dk.upload(kv, s);
        hipLaunchKernelGGL(k_far_dp, grid, dim3(128), 0, s, kernel == PKIFMM_STOKES ? 1 : 0, fr[0], fr[1], fr[2], X, m,
                           Y, n, out, ld, (const double2*)dk.p, (int)(kv.size() / 2), rc, P, c_par, c_z);
        PK_HIP(hipGetLastError());
        PK_HIP(hipStreamSynchronize(s));
        return;
    }
    throw Error(PKIFMM_ERR_UNSUPPORTED, "no far-field operator for this kernel and periodicity");
}

void launch_pinv_factors(const double* U, const double* Vt, const double* S, int kn, int r, double* Ut_r, double* VS,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pinv_factors, dim3((kn + 127) / 128, r), dim3(128), 0, s, U, Vt, S, kn, r, Ut_r, VS);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
