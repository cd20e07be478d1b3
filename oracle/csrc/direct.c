/*
 * Oracle direct sums (test infrastructure only; never part of the product).
 *
 * Plain, unblocked double-precision loops for
 *     out[t] += sum_s K(x_t - (y_s + shift)) dens[s]
 * with the free-space kernels of the paper's examples (Section 2, the
 * Laplace and Stokes-velocity kernels):
 *     Laplace  K(r) = 1 / (4 pi |r|)                                (k = 1)
 *     Stokes   K(r) = (1 / (8 pi)) (I / |r| + r r^T / |r|^3)        (k = 3)
 * A pair whose separation is exactly zero contributes nothing (the usual
 * self-interaction convention; the paper's Madelung example evaluates the
 * potential at a charge without its own singular term).
 *
 * Layout: points are [n][3] row-major, densities and outputs are [n][k].
 */
#include <math.h>
#include <stdint.h>

#define ORACLE_PI 3.14159265358979323846

void oracle_direct(int kernel, int64_t nt, const double *xt, int64_t ns,
                   const double *ys, const double *dens, const double *shift,
                   double *out)
{
    const double sx = shift ? shift[0] : 0.0;
    const double sy = shift ? shift[1] : 0.0;
    const double sz = shift ? shift[2] : 0.0;
    if (kernel == 1) {
        const double c = 1.0 / (4.0 * ORACLE_PI);
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < nt; ++t) {
            double acc = 0.0;
            for (int64_t s = 0; s < ns; ++s) {
                double dx = xt[3 * t + 0] - (ys[3 * s + 0] + sx);
                double dy = xt[3 * t + 1] - (ys[3 * s + 1] + sy);
                double dz = xt[3 * t + 2] - (ys[3 * s + 2] + sz);
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                acc += dens[s] / sqrt(r2);
            }
            out[t] += c * acc;
        }
    } else {
        const double c = 1.0 / (8.0 * ORACLE_PI);
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < nt; ++t) {
            double ux = 0.0, uy = 0.0, uz = 0.0;
            for (int64_t s = 0; s < ns; ++s) {
                double dx = xt[3 * t + 0] - (ys[3 * s + 0] + sx);
                double dy = xt[3 * t + 1] - (ys[3 * s + 1] + sy);
                double dz = xt[3 * t + 2] - (ys[3 * s + 2] + sz);
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double fx = dens[3 * s + 0], fy = dens[3 * s + 1], fz = dens[3 * s + 2];
                double fr = (fx * dx + fy * dy + fz * dz) / (r2 * r);
                ux += fx / r + dx * fr;
                uy += fy / r + dy * fr;
                uz += fz / r + dz * fr;
            }
            out[3 * t + 0] += c * ux;
            out[3 * t + 1] += c * uy;
            out[3 * t + 2] += c * uz;
        }
    }
}
