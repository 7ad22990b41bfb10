/*
 * Host check of the oracle's C routines, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitize.py.
 *
 * Solves small problems with seeded coefficients, checks the relative
 * residual, that the residual routine agrees (zero field: r = b; the
 * solution: r ~ 0), that the assembled band is finite and that the timing
 * routine factors a prefix.  The point is memory and arithmetic safety of
 * the routines; their numerical pins live in the Python tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_solve(int N, const double* kappa, const double* f, int sweeps, double* u_full, double* relres);
void oracle_residual(int N, const double* kappa, const double* f, const double* u_full, double* r_full);
void oracle_band(int N, const double* kappa, double* band_out);
double oracle_factor_prefix_seconds(int N, const double* kappa, int64_t ncols);

static uint64_t st = 88172645463325252ull;
static double urand(void) {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (double)(st >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    int fails = 0;
    const int sizes[] = {1, 2, 3, 7, 15, 31};
    for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
        const int N = sizes[k], nc = N + 1;
        double* kap = malloc(sizeof(double) * nc * nc * 2);
        double* f = malloc(sizeof(double) * (N + 2) * (N + 2));
        double* u = malloc(sizeof(double) * (N + 2) * (N + 2));
        double* z = calloc((size_t)(N + 2) * (N + 2), sizeof(double));
        double* r = malloc(sizeof(double) * (N + 2) * (N + 2));
        double* band = malloc(sizeof(double) * (size_t)N * N * (N + 1));
        for (int e = 0; e < nc * nc * 2; ++e) kap[e] = exp(2.0 * urand() - 1.0);
        for (int e = 0; e < (N + 2) * (N + 2); ++e) f[e] = urand();
        double rel = -1.0;
        const int64_t info = oracle_solve(N, kap, f, 1, u, &rel);
        if (info != 0 || !(rel < 1e-14)) {
            fprintf(stderr, "N=%d: info %lld relres %g\n", N, (long long)info, rel);
            ++fails;
        }
        oracle_residual(N, kap, f, u, r);
        double rmax = 0.0;
        for (int e = 0; e < (N + 2) * (N + 2); ++e) rmax = fmax(rmax, fabs(r[e]));
        oracle_residual(N, kap, f, z, r);
        double bmax = 0.0;
        for (int e = 0; e < (N + 2) * (N + 2); ++e) bmax = fmax(bmax, fabs(r[e]));
        if (!(bmax > 0.0) || !(rmax <= 1e-13 * bmax)) {
            fprintf(stderr, "N=%d: residual %g of %g\n", N, rmax, bmax);
            ++fails;
        }
        oracle_band(N, kap, band);
        for (int e = 0; e < N * N * (N + 1); ++e)
            if (!isfinite(band[e])) {
                fprintf(stderr, "N=%d: band entry %d not finite\n", N, e);
                ++fails;
                break;
            }
        if (!(oracle_factor_prefix_seconds(N, kap, (N * N + 1) / 2) >= 0.0)) {
            fprintf(stderr, "N=%d: prefix factorization failed\n", N);
            ++fails;
        }
        free(kap); free(f); free(u); free(z); free(r); free(band);
    }
    printf("oracle checks: %d failures\n", fails);
    return fails ? 1 : 0;
}
