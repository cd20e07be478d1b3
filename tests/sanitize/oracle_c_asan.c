/* The oracle's C helpers under AddressSanitizer and UndefinedBehaviorSanitizer (built by
 * tests/test_sanitize_host.py with gcc): the direct sums with and without a shift and with a
 * coincident pair, and the triply periodic Ewald sums at targets, for both kernels and several
 * right-hand sides.  Checks Laplace direct against a hand-written double loop. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_direct(int kernel, int64_t nt, const double *xt, int64_t ns, const double *ys, const double *dens,
                   const double *shift, double *out);
void tp_ewald_targets(int kernel, int R, int64_t T, const double *xt, int64_t N, const double *ys,
                      const double *dens_rnk, double xi, double rc, int kint, double *out);

static double rnd(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) / 16777216.0; }

int main(void) {
    unsigned seed = 7;
    enum { NT = 37, NS = 53, R = 3 };
    double *xt = malloc(sizeof(double) * 3 * NT), *ys = malloc(sizeof(double) * 3 * NS);
    double *d = malloc(sizeof(double) * 3 * NS * R), *out = malloc(sizeof(double) * 3 * NT * R);
    for (int i = 0; i < 3 * NT; ++i) xt[i] = rnd(&seed);
    for (int i = 0; i < 3 * NS; ++i) ys[i] = rnd(&seed);
    for (int i = 0; i < 3 * NS * R; ++i) d[i] = rnd(&seed) - 0.5;
    for (int a = 0; a < 3; ++a) ys[3 * 5 + a] = xt[3 * 2 + a];          /* a coincident pair */
    int fails = 0;
    const double shift[3] = {1.0, 0.0, -1.0};
    for (int kernel = 1; kernel <= 2; ++kernel)
        for (int sh = 0; sh < 2; ++sh) {
            const int k = kernel == 1 ? 1 : 3;
            for (int i = 0; i < NT * k; ++i) out[i] = 0.0;
            oracle_direct(kernel, NT, xt, NS, ys, d, sh ? shift : NULL, out);
            if (kernel == 1) {
                for (int t = 0; t < NT; ++t) {
                    double ref = 0.0;
                    for (int s = 0; s < NS; ++s) {
                        double dx = xt[3 * t] - ys[3 * s] - (sh ? shift[0] : 0), dy = xt[3 * t + 1] - ys[3 * s + 1] - (sh ? shift[1] : 0),
                               dz = xt[3 * t + 2] - ys[3 * s + 2] - (sh ? shift[2] : 0);
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r > 0) ref += d[s] / (4.0 * 3.14159265358979323846 * r);
                    }
                    if (fabs(out[t] - ref) > 1e-12 * (1.0 + fabs(ref))) ++fails;
                }
            }
            for (int i = 0; i < NT * k; ++i) if (!isfinite(out[i])) ++fails;
        }
    for (int kernel = 1; kernel <= 2; ++kernel) {
        const int k = kernel == 1 ? 1 : 3;
        /* zero net density per right-hand side (the triply periodic sums need it) */
        for (int r = 0; r < R; ++r)
            for (int c = 0; c < k; ++c) {
                double m = 0.0;
                for (int s = 0; s < NS; ++s) m += d[(r * NS + s) * k + c];
                for (int s = 0; s < NS; ++s) d[(r * NS + s) * k + c] -= m / NS;
            }
        tp_ewald_targets(kernel, R, NT, xt, NS, ys, d, 6.0, 0.5, 6, out);
        for (int i = 0; i < NT * k * R; ++i) if (!isfinite(out[i])) ++fails;
    }
    free(xt); free(ys); free(d); free(out);
    printf("oracle C under the sanitizers: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
