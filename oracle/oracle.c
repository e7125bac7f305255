/*
 * oracle.c -- CPU oracle for the Jacobi pressure sweep. TEST INFRASTRUCTURE.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this file's library. The product path never does.
 * It shares no code, header or helper with the HIP library.
 *
 * What it computes. The paper's Himeno workload solves a Poisson equation by
 * Jacobi iteration (section 5.1.1). Its offload method keeps every array on
 * the device for the whole nest, transferring only at the outermost loop
 * (sections 3.2 and 3.3). The paper prints no stencil, so the operator below
 * is the reading this project fixes for it: a 19-point variable-coefficient
 * stencil on a grid of nx*ny*nz points (k contiguous), with a one-cell
 * Dirichlet shell that is never written.
 *
 * One Jacobi iteration, over interior cells (1 <= i <= nx-2, same for j, k),
 * every term using only p from before the iteration:
 *   s0 = a0 p(i+1,j,k) + a1 p(i,j+1,k) + a2 p(i,j,k+1)
 *      + b0 [p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k)]
 *      + b1 [p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1)]
 *      + b2 [p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1)]
 *      + c0 p(i-1,j,k) + c1 p(i,j-1,k) + c2 p(i,j,k-1) + wrk1
 *   ss   = (s0 a3 - p) bnd
 *   gosa = sum of ss^2 over the interior (FP64)
 *   wrk2 = p + omega ss
 * then p = wrk2 on the interior. Coefficients are taken at (i,j,k).
 *
 * Evaluation order: every sum above is accumulated left to right as written,
 * each bracket left to right before its multiply; then t = s0*a3, t = t - p,
 * ss = t*bnd, wrk2 = p + (omega*ss). Every operation rounds to nearest; this
 * file must be built with -ffp-contract=off and no fast-math.
 *
 * gosa is summed with Neumaier's compensated summation per i plane (cells in
 * j, k order) and the plane sums are combined, compensated, in i order, so the
 * value does not depend on the thread count.
 *
 * Field order of the 14 arrays: p a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1 wrk2,
 * each a dense C-order [nx][ny][nz] array of doubles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { P = 0, A0, A1, A2, A3, B0, B1, B2, C0, C1, C2, BND, WRK1, WRK2, NF };

typedef struct { double s, c; } kahan_t;

static inline void kadd(kahan_t* a, double x)
{
    /* Neumaier (1974): the larger magnitude operand absorbs the smaller. */
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

/* The residual term ss at cell (i,j,k). */
static inline double cell_ss(double* const f[NF], long sj, long si, long n)
{
    const double* p = f[P];
    double s0 = f[A0][n] * p[n + si];
    s0 = s0 + f[A1][n] * p[n + sj];
    s0 = s0 + f[A2][n] * p[n + 1];
    s0 = s0 + f[B0][n] * (((p[n + si + sj] - p[n + si - sj]) - p[n - si + sj]) + p[n - si - sj]);
    s0 = s0 + f[B1][n] * (((p[n + sj + 1] - p[n - sj + 1]) - p[n + sj - 1]) + p[n - sj - 1]);
    s0 = s0 + f[B2][n] * (((p[n + si + 1] - p[n - si + 1]) - p[n + si - 1]) + p[n - si - 1]);
    s0 = s0 + f[C0][n] * p[n - si];
    s0 = s0 + f[C1][n] * p[n - sj];
    s0 = s0 + f[C2][n] * p[n - 1];
    s0 = s0 + f[WRK1][n];
    double t = s0 * f[A3][n];
    t = t - p[n];
    return t * f[BND][n];
}

static int check(int nx, int ny, int nz, double* const f[NF])
{
    if (nx < 3 || ny < 3 || nz < 3) return -2;
    for (int q = 0; q < NF; ++q)
        if (!f[q]) return -1;
    return 0;
}

/* One pass over the interior. Writes wrk2 when `update`, returns gosa. */
static double pass(int nx, int ny, int nz, double* const f[NF], double omega, int update,
                   kahan_t* plane, int nthreads)
{
    const long sj = nz, si = (long)ny * nz;
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int i = 1; i < nx - 1; ++i) {
        kahan_t acc = {0.0, 0.0};
        for (int j = 1; j < ny - 1; ++j)
            for (int k = 1; k < nz - 1; ++k) {
                const long n = i * si + j * sj + k;
                const double ss = cell_ss(f, sj, si, n);
                kadd(&acc, ss * ss);
                if (update) f[WRK2][n] = f[P][n] + omega * ss;
            }
        plane[i] = acc;
    }
    kahan_t tot = {0.0, 0.0};
    for (int i = 1; i < nx - 1; ++i) kadd(&tot, plane[i].s + plane[i].c);
    return tot.s + tot.c;
}

/*
 * n_iter Jacobi iterations. On return p holds the field after the last
 * iteration, wrk2 the last iteration's output (equal to p on the interior;
 * its shell is left as the caller set it), gosa_hist[t] (if not NULL) the gosa
 * of iteration t, computed from the field before that iteration's update.
 * nthreads <= 0 means one thread. Returns 0, -1 (null array), -2 (shape),
 * -3 (n_iter < 0) or -4 (out of memory).
 */
int oracle_sweep(int nx, int ny, int nz, double* const f[NF], int n_iter, double omega,
                 double* gosa_hist, int nthreads)
{
    int rc = check(nx, ny, nz, f);
    if (rc) return rc;
    if (n_iter < 0) return -3;
    kahan_t* plane = (kahan_t*)calloc((size_t)nx, sizeof(kahan_t));
    if (!plane) return -4;
    const long sj = nz, si = (long)ny * nz;
    for (int t = 0; t < n_iter; ++t) {
        const double g = pass(nx, ny, nz, f, omega, 1, plane, nthreads);
        if (gosa_hist) gosa_hist[t] = g;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
        for (int i = 1; i < nx - 1; ++i)
            for (int j = 1; j < ny - 1; ++j)
                memcpy(&f[P][i * si + j * sj + 1], &f[WRK2][i * si + j * sj + 1],
                       sizeof(double) * (size_t)(nz - 2));
    }
    free(plane);
    return 0;
}

/* gosa of the current p without updating anything (-1.0 on bad arguments). */
double oracle_residual(int nx, int ny, int nz, double* const f[NF], int nthreads)
{
    if (check(nx, ny, nz, f)) return -1.0;
    kahan_t* plane = (kahan_t*)calloc((size_t)nx, sizeof(kahan_t));
    if (!plane) return -1.0;
    const double g = pass(nx, ny, nz, f, 0.0, 0, plane, nthreads);
    free(plane);
    return g;
}

/*
 * One iteration evaluated at selected interior cells only: for each dense
 * linear index idx[q], ss_out[q] = ss and wrk2_out[q] = p + omega*ss, from the
 * current p. Used to check single cells of grids too large to sweep on the
 * host. Returns 0, or -5 if an index is not an interior cell.
 */
int oracle_cells(int nx, int ny, int nz, double* const f[NF], double omega, long long n_cells,
                 const long long* idx, double* ss_out, double* wrk2_out)
{
    int rc = check(nx, ny, nz, f);
    if (rc) return rc;
    const long sj = nz, si = (long)ny * nz;
    for (long long q = 0; q < n_cells; ++q) {
        const long long n = idx[q];
        const long long i = n / si, j = (n / sj) % ny, k = n % nz;
        if (i < 1 || j < 1 || k < 1 || i > nx - 2 || j > ny - 2 || k > nz - 2) return -5;
        const double ss = cell_ss(f, sj, si, (long)n);
        if (ss_out) ss_out[q] = ss;
        if (wrk2_out) wrk2_out[q] = f[P][n] + omega * ss;
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
