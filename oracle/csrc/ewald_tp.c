/*
 * Triply periodic sums at a few targets from many sources (oracle; test infrastructure only).
 *
 * The definitions are those of oracle/periodic.py's pairwise Ewald sums (the k = 0 mode removed:
 * zero mean; Section 3, triply periodic Stokes uses the Hasimoto split): for a target x and
 * sources y_s with densities f_s,
 *   Stokes   u(x) = sum_s sum_p S^R(x - y_s - p) f_s / (8 pi)
 *                 + sum_{k != 0} (1 + k^2/4xi^2) e^{-k^2/4xi^2} / k^2 (I - k k^T/k^2) Re e^{ik.x} F(k)
 *   Laplace  u(x) = sum_s sum_p erfc(xi r)/(4 pi r) q_s - sum_s q_s / (4 xi^2)
 *                 + sum_{k != 0} e^{-k^2/4xi^2} / k^2 Re e^{ik.x} Q(k)
 * with k over 2 pi Z^3 (each +-k pair once, doubled), F(k) = sum_s f_s e^{-ik.y_s} (Q alike), the
 * real-space part taken over the nearest image only (the cutoff rc is at most half the period),
 * and a pair at exactly zero separation contributing nothing (its smooth part is subtracted).
 * The structure factors F(k) are summed once over all sources, so the cost is O(N K + T N)
 * rather than O(T N (images + K)).  Separable exponentials e^{-i 2 pi m y} are built by
 * repeated multiplication along each axis.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    double re, im;
} cplx;

static int build_modes(int kint, int** mx, int** my, int** mz) {
    int cap = (2 * kint + 1) * (2 * kint + 1) * (2 * kint + 1), n = 0;
    *mx = (int*)malloc(sizeof(int) * cap);
    *my = (int*)malloc(sizeof(int) * cap);
    *mz = (int*)malloc(sizeof(int) * cap);
    for (int a = -kint; a <= kint; ++a)
        for (int b = -kint; b <= kint; ++b)
            for (int c = -kint; c <= kint; ++c) {
                if (a * a + b * b + c * c > kint * kint) continue;
                const int first = a != 0 ? a : (b != 0 ? b : c);   /* one of each +-m pair */
                if (first <= 0) continue;
                (*mx)[n] = a; (*my)[n] = b; (*mz)[n] = c;
                ++n;
            }
    return n;
}

/* e^{-i 2 pi m v} for m = -kint .. kint, into e[m + kint] */
static void axis_phases(double v, int kint, cplx* e) {
    const double th = -2.0 * M_PI * v;
    const cplx w = {cos(th), sin(th)};
    e[kint].re = 1.0; e[kint].im = 0.0;
    for (int m = 1; m <= kint; ++m) {
        const cplx p = e[kint + m - 1];
        e[kint + m].re = p.re * w.re - p.im * w.im;
        e[kint + m].im = p.re * w.im + p.im * w.re;
        e[kint - m].re = e[kint + m].re;            /* conjugate */
        e[kint - m].im = -e[kint + m].im;
    }
}

/*
 * kernel: 1 Laplace (k = 1), 2 Stokes (k = 3).  xt [T][3], ys [N][3] in the unit box (any
 * period representative), dens [R][N][k] (R right-hand sides); out [R][T][k] overwritten.
 * xi: Ewald splitting; rc <= 0.5: real-space cutoff; kint: Fourier cutoff |m| <= kint.
 */
void tp_ewald_targets(int kernel, int R, int64_t T, const double* xt, int64_t N, const double* ys,
                      const double* dens_rnk, double xi, double rc, int kint, double* out) {
    const int kd = (kernel == 1 ? 1 : 3) * R;     /* values per source: every right-hand side */
    const int kk = kernel == 1 ? 1 : 3;
    /* the densities as [N][R][k], so that one source's values are adjacent */
    double* dens = (double*)malloc(sizeof(double) * (size_t)N * kd);
    for (int r = 0; r < R; ++r)
        for (int64_t s = 0; s < N; ++s)
            for (int q = 0; q < kk; ++q) dens[s * kd + r * kk + q] = dens_rnk[((int64_t)r * N + s) * kk + q];
    int *mx, *my, *mz;
    const int K = build_modes(kint, &mx, &my, &mz);
    const int L = 2 * kint + 1;
    double* F = (double*)calloc((size_t)K * kd * 2, sizeof(double));      /* [K][kd][re, im] */
#pragma omp parallel
    {
        double* Fl = (double*)calloc((size_t)K * kd * 2, sizeof(double));
        cplx* ex = (cplx*)malloc(sizeof(cplx) * 3 * L);
        cplx *ey = ex + L, *ez = ex + 2 * L;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < N; ++s) {
            axis_phases(ys[3 * s], kint, ex);
            axis_phases(ys[3 * s + 1], kint, ey);
            axis_phases(ys[3 * s + 2], kint, ez);
            for (int j = 0; j < K; ++j) {
                const cplx a = ex[mx[j] + kint], b = ey[my[j] + kint], c = ez[mz[j] + kint];
                const double abr = a.re * b.re - a.im * b.im, abi = a.re * b.im + a.im * b.re;
                const double vr = abr * c.re - abi * c.im, vi = abr * c.im + abi * c.re;
                for (int q = 0; q < kd; ++q) {
                    Fl[(j * kd + q) * 2] += dens[s * kd + q] * vr;
                    Fl[(j * kd + q) * 2 + 1] += dens[s * kd + q] * vi;
                }
            }
        }
#pragma omp critical
        for (size_t i = 0; i < (size_t)K * kd * 2; ++i) F[i] += Fl[i];
        free(Fl);
        free(ex);
    }
    double qsum[16] = {0.0};
    if (kk == 1)
        for (int64_t s = 0; s < N; ++s)
            for (int r = 0; r < R; ++r) qsum[r] += dens[s * kd + r];
    const double c0 = 2.0 * xi / sqrt(M_PI);
#pragma omp parallel
    {
        cplx* ex = (cplx*)malloc(sizeof(cplx) * 3 * L);
        cplx *ey = ex + L, *ez = ex + 2 * L;
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < T; ++t) {
            double acc[64];
            for (int q = 0; q < kd; ++q) acc[q] = 0.0;
            const double x = xt[3 * t], y = xt[3 * t + 1], z = xt[3 * t + 2];
            /* real space, nearest image */
            for (int64_t s = 0; s < N; ++s) {
                double d[3] = {x - ys[3 * s], y - ys[3 * s + 1], z - ys[3 * s + 2]};
                for (int a = 0; a < 3; ++a) d[a] -= nearbyint(d[a]);
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 >= rc * rc) continue;
                if (r2 == 0.0) {      /* coincident: drop the singular term, i.e. remove the smooth part */
                    for (int q = 0; q < kd; ++q)
                        acc[q] -= (kk == 1 ? c0 / (4.0 * M_PI) : 2.0 * c0 / (8.0 * M_PI)) * dens[s * kd + q];
                    continue;
                }
                const double r = sqrt(r2);
                const double ec = erfc(xi * r) / r;
                if (kk == 1) {
                    for (int q = 0; q < kd; ++q) acc[q] += ec / (4.0 * M_PI) * dens[s * kd + q];
                } else {
                    const double g = c0 * exp(-xi * xi * r2);
                    for (int rr = 0; rr < R; ++rr) {
                        const double* f = dens + s * kd + 3 * rr;
                        const double fd = (f[0] * d[0] + f[1] * d[1] + f[2] * d[2]) / r2;
                        for (int a = 0; a < 3; ++a)
                            acc[3 * rr + a] += ((ec - g) * f[a] + (ec + g) * fd * d[a]) / (8.0 * M_PI);
                    }
                }
            }
            if (kk == 1)
                for (int r = 0; r < R; ++r) acc[r] -= qsum[r] / (4.0 * xi * xi);
            /* Fourier part */
            axis_phases(-x, kint, ex);
            axis_phases(-y, kint, ey);
            axis_phases(-z, kint, ez);
            for (int j = 0; j < K; ++j) {
                const double kx = 2.0 * M_PI * mx[j], ky = 2.0 * M_PI * my[j], kz = 2.0 * M_PI * mz[j];
                const double k2 = kx * kx + ky * ky + kz * kz, x4 = k2 / (4.0 * xi * xi);
                const cplx a = ex[mx[j] + kint], b = ey[my[j] + kint], c = ez[mz[j] + kint];
                const double abr = a.re * b.re - a.im * b.im, abi = a.re * b.im + a.im * b.re;
                const double er = abr * c.re - abi * c.im, ei = abr * c.im + abi * c.re;   /* e^{ik.x} */
                if (kk == 1) {
                    const double w = 2.0 * exp(-x4) / k2;
                    for (int q = 0; q < kd; ++q) acc[q] += w * (er * F[(j * kd + q) * 2] - ei * F[(j * kd + q) * 2 + 1]);
                } else {
                    const double w = 2.0 * (1.0 + x4) * exp(-x4) / k2;
                    for (int rr = 0; rr < R; ++rr) {
                        double v[3];
                        for (int q = 0; q < 3; ++q) {
                            const int c = j * kd + 3 * rr + q;
                            v[q] = er * F[2 * c] - ei * F[2 * c + 1];
                        }
                        const double kv = (kx * v[0] + ky * v[1] + kz * v[2]) / k2;
                        acc[3 * rr] += w * (v[0] - kx * kv);
                        acc[3 * rr + 1] += w * (v[1] - ky * kv);
                        acc[3 * rr + 2] += w * (v[2] - kz * kv);
                    }
                }
            }
            for (int r = 0; r < R; ++r)
                for (int q = 0; q < kk; ++q) out[((int64_t)r * T + t) * kk + q] = acc[r * kk + q];
        }
        free(ex);
    }
    free(F);
    free(dens);
    free(mx);
    free(my);
    free(mz);
}
