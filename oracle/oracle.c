/*
 * oracle.c -- plain, slow, obviously correct FP64 reference for the HDD path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU library.
 *
 * What it computes.  The paper states that, up to the hierarchical-matrix
 * approximation (not used here), the HDD result is exactly the finite element
 * solution of the global problem (abstract; Root-to-Leaves remark that the
 * interface values together form the solution of the initial problem).  So the
 * oracle is that definition written out: assemble the P1 system A u = b for
 * -div(kappa grad u) = f, u = 0 on the boundary of the unit square (problem
 * statement, eq. elliptic), and solve it directly.
 *
 *  - Mesh: N interior nodes per side, Nc = N+1 cells, h = 1/Nc.  Cell (i,j)
 *    is split along its SW-NE diagonal into T- = {(i,j),(i+1,j),(i+1,j+1)}
 *    and T+ = {(i,j),(i+1,j+1),(i,j+1)}; kappa is constant per triangle,
 *    kappa[(j*Nc+i)*2 + 0] for T-, [... + 1] for T+.
 *  - Stiffness (eq. coefA, A_ij = int kappa grad b_i . grad b_j): on a right
 *    isosceles triangle with legs h the P1 element matrix is
 *    kappa/2 * [[1,-1,0],[-1,2,-1],[0,-1,1]] with the right-angle vertex in
 *    the middle, so a leg couples its endpoints by -kappa/2 and the hypotenuse
 *    by 0.  Each mesh edge is a leg of exactly the triangles beside it, which
 *    gives the closed-form 5-point operator used below (not an element loop):
 *      horizontal edge (i,j)-(i+1,j): c = (kappa-(i,j) + kappa+(i,j-1)) / 2
 *      vertical   edge (i,j)-(i,j+1): c = (kappa+(i,j) + kappa-(i-1,j)) / 2
 *      A_pp = sum of c over the four edges at p, A_pq = -c.
 *  - Load (eq. coefc, vertex rule c_i = |t| f(x_i) / 3 per triangle): an
 *    interior node lies in 6 triangles of area h^2/2, so b_p = 6 (h^2/2) f_p / 3.
 *  - Solve: banded Cholesky (bandwidth N, lexicographic DOF order
 *    p = (j-1) N + (i-1)), forward and backward substitution, then sweeps of
 *    iterative refinement whose residual b - A u is accumulated in x87
 *    extended precision (long double), so that the result is accurate to
 *    about the FP64 unit roundoff rather than cond(A) times it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef long double ld_t;

static double kap_minus(const double* kappa, int nc, int i, int j) {
    if (i < 0 || j < 0 || i >= nc || j >= nc) return 0.0;
    return kappa[((size_t)j * nc + i) * 2 + 0];
}
static double kap_plus(const double* kappa, int nc, int i, int j) {
    if (i < 0 || j < 0 || i >= nc || j >= nc) return 0.0;
    return kappa[((size_t)j * nc + i) * 2 + 1];
}
/* coupling of the horizontal edge (i,j)-(i+1,j) */
static double c_horiz(const double* kappa, int nc, int i, int j) {
    return 0.5 * (kap_minus(kappa, nc, i, j) + kap_plus(kappa, nc, i, j - 1));
}
/* coupling of the vertical edge (i,j)-(i,j+1) */
static double c_vert(const double* kappa, int nc, int i, int j) {
    return 0.5 * (kap_plus(kappa, nc, i, j) + kap_minus(kappa, nc, i - 1, j));
}

/* Lower band in column-major band storage: band[p*(N+1) + d] = A[p+d][p].
 * Only columns [0, ncols) are written. */
static void assemble_band(int N, const double* kappa, double* band, int64_t ncols) {
    const int nc = N + 1;
    const int64_t n = (int64_t)N * N;
    if (ncols > n) ncols = n;
    memset(band, 0, sizeof(double) * (size_t)ncols * (size_t)(N + 1));
    for (int64_t p = 0; p < ncols; ++p) {
        const int i = (int)(p % N) + 1, j = (int)(p / N) + 1;
        double* col = band + (size_t)p * (N + 1);
        col[0] = c_horiz(kappa, nc, i - 1, j) + c_horiz(kappa, nc, i, j) +
                 c_vert(kappa, nc, i, j - 1) + c_vert(kappa, nc, i, j);
        if (i + 1 <= N) col[1] = -c_horiz(kappa, nc, i, j);
        if (j + 1 <= N) col[N] = -c_vert(kappa, nc, i, j);
    }
}

/* Right-looking banded Cholesky of columns [c0, c1).  Returns 0, or 1 + the
 * column whose pivot is not positive. */
static int64_t band_factor(double* band, int bw, int64_t n, int64_t c0, int64_t c1) {
    for (int64_t j = c0; j < c1; ++j) {
        double* cj = band + (size_t)j * (bw + 1);
        if (!(cj[0] > 0.0)) return j + 1;
        const double d = sqrt(cj[0]);
        cj[0] = d;
        const int64_t m = (bw < n - 1 - j) ? bw : n - 1 - j;
        for (int64_t k = 1; k <= m; ++k) cj[k] /= d;
        for (int64_t k = 1; k <= m; ++k) {
            double* ck = band + (size_t)(j + k) * (bw + 1);
            const double l = cj[k];
            for (int64_t t = 0; t <= m - k; ++t) ck[t] -= cj[k + t] * l;
        }
    }
    return 0;
}

/* x <- (L L^T)^{-1} x with the factor in band storage. */
static void band_solve(const double* band, int bw, int64_t n, double* x) {
    for (int64_t j = 0; j < n; ++j) {
        const double* cj = band + (size_t)j * (bw + 1);
        x[j] /= cj[0];
        const int64_t m = (bw < n - 1 - j) ? bw : n - 1 - j;
        for (int64_t k = 1; k <= m; ++k) x[j + k] -= cj[k] * x[j];
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        const double* cj = band + (size_t)j * (bw + 1);
        const int64_t m = (bw < n - 1 - j) ? bw : n - 1 - j;
        double s = x[j];
        for (int64_t k = 1; k <= m; ++k) s -= cj[k] * x[j + k];
        x[j] = s / cj[0];
    }
}

static double load_at(int N, const double* f, int i, int j) {
    const double h = 1.0 / (N + 1);
    const double area = 0.5 * h * h;
    return 6.0 * area * f[(size_t)j * (N + 2) + i] / 3.0;
}

/* r = b - A u in extended precision, u given on DOFs (lexicographic). */
static void residual_ext(int N, const double* kappa, const double* f, const double* u, ld_t* r) {
    const int nc = N + 1;
    for (int j = 1; j <= N; ++j) {
        for (int i = 1; i <= N; ++i) {
            const int64_t p = (int64_t)(j - 1) * N + (i - 1);
            const ld_t cw = c_horiz(kappa, nc, i - 1, j), ce = c_horiz(kappa, nc, i, j);
            const ld_t cs = c_vert(kappa, nc, i, j - 1), cn = c_vert(kappa, nc, i, j);
            ld_t au = (cw + ce + cs + cn) * (ld_t)u[p];
            if (i > 1) au -= cw * (ld_t)u[p - 1];
            if (i < N) au -= ce * (ld_t)u[p + 1];
            if (j > 1) au -= cs * (ld_t)u[p - N];
            if (j < N) au -= cn * (ld_t)u[p + N];
            r[p] = (ld_t)load_at(N, f, i, j) - au;
        }
    }
}

/*
 * Full solve.  kappa: [Nc][Nc][2]; f: [N+2][N+2] nodal (boundary ignored);
 * u_full: [N+2][N+2] output, zero on the boundary.  relres (may be NULL)
 * receives ||b - A u||_2 / ||b||_2 evaluated in extended precision.
 * Returns 0, -1 on allocation failure, or 1 + the failing pivot column.
 */
int64_t oracle_solve(int N, const double* kappa, const double* f, int sweeps,
                     double* u_full, double* relres) {
    const int64_t n = (int64_t)N * N;
    double* band = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(N + 1));
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    ld_t* r = (ld_t*)malloc(sizeof(ld_t) * (size_t)n);
    if (!band || !x || !d || !r) {
        free(band); free(x); free(d); free(r);
        return -1;
    }
    assemble_band(N, kappa, band, n);
    int64_t info = band_factor(band, N, n, 0, n);
    if (info) {
        free(band); free(x); free(d); free(r);
        return info;
    }
    for (int j = 1; j <= N; ++j)
        for (int i = 1; i <= N; ++i) x[(int64_t)(j - 1) * N + (i - 1)] = load_at(N, f, i, j);
    band_solve(band, N, n, x);
    for (int s = 0; s < sweeps; ++s) {
        residual_ext(N, kappa, f, x, r);
        for (int64_t p = 0; p < n; ++p) d[p] = (double)r[p];
        band_solve(band, N, n, d);
        for (int64_t p = 0; p < n; ++p) x[p] = (double)((ld_t)x[p] + (ld_t)d[p]);
    }
    if (relres) {
        residual_ext(N, kappa, f, x, r);
        ld_t rr = 0, bb = 0;
        for (int j = 1; j <= N; ++j)
            for (int i = 1; i <= N; ++i) {
                const int64_t p = (int64_t)(j - 1) * N + (i - 1);
                const ld_t b = load_at(N, f, i, j);
                rr += r[p] * r[p];
                bb += b * b;
            }
        *relres = (double)(bb > 0 ? sqrtl(rr / bb) : sqrtl(rr));
    }
    memset(u_full, 0, sizeof(double) * (size_t)(N + 2) * (N + 2));
    for (int j = 1; j <= N; ++j)
        for (int i = 1; i <= N; ++i) u_full[(size_t)j * (N + 2) + i] = x[(int64_t)(j - 1) * N + (i - 1)];
    free(band); free(x); free(d); free(r);
    return 0;
}

/*
 * Residual of an arbitrary nodal field: r_full[j][i] = (b - A u)_p at interior
 * nodes (extended-precision accumulation, rounded), 0 on the boundary.  Used
 * to check solutions at sizes the direct solve cannot reach in a test.
 */
void oracle_residual(int N, const double* kappa, const double* f, const double* u_full,
                     double* r_full) {
    const int64_t n = (int64_t)N * N;
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    ld_t* r = (ld_t*)malloc(sizeof(ld_t) * (size_t)n);
    for (int j = 1; j <= N; ++j)
        for (int i = 1; i <= N; ++i) x[(int64_t)(j - 1) * N + (i - 1)] = u_full[(size_t)j * (N + 2) + i];
    residual_ext(N, kappa, f, x, r);
    memset(r_full, 0, sizeof(double) * (size_t)(N + 2) * (N + 2));
    for (int j = 1; j <= N; ++j)
        for (int i = 1; i <= N; ++i) r_full[(size_t)j * (N + 2) + i] = (double)r[(int64_t)(j - 1) * N + (i - 1)];
    free(x); free(r);
}

/* The assembled band (for tests that compare it with an element loop). */
void oracle_band(int N, const double* kappa, double* band_out) {
    assemble_band(N, kappa, band_out, (int64_t)N * N);
}

/*
 * Timing sample for the CPU baseline: assemble the columns the first `ncols`
 * factorization steps touch and factor those `ncols` columns with the same
 * routine as oracle_solve.  Every column of the banded factorization away
 * from the end costs the same (bandwidth^2 multiply-adds), so the full
 * factorization time is this time scaled by n / ncols.  Returns seconds of the
 * factorization alone, or a negative value on failure.
 */
double oracle_factor_prefix_seconds(int N, const double* kappa, int64_t ncols) {
    const int64_t n = (int64_t)N * N;
    if (ncols > n) ncols = n;
    int64_t cols = ncols + N + 1;
    if (cols > n) cols = n;
    double* band = (double*)malloc(sizeof(double) * (size_t)cols * (size_t)(N + 1));
    if (!band) return -1.0;
    assemble_band(N, kappa, band, cols);
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int64_t info = band_factor(band, N, cols, 0, ncols);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    free(band);
    if (info) return -2.0;
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
