/*
 * spx_oracle_omp.c -- all-core variants of the oracle's CSR product and CG.
 *
 * TEST INFRASTRUCTURE ONLY (the CPU baseline of the benchmark, and the
 * float64 reference solution of full-size tests). Same definitions as the
 * plain oracle in spx_oracle.c, with the loops over rows and vector entries
 * shared among OpenMP threads (static schedule):
 *  - the product sums each row sequentially in storage order, exactly as the
 *    plain oracle does, so y is bitwise the plain oracle's;
 *  - CG (Hestenes-Stiefel; Barrett et al., "Templates", 1994) takes the
 *    same steps as orc_cg with precond 0 (none) or 1 (scalar Jacobi) from
 *    x0 = 0; the dot products are summed per thread over a fixed block and
 *    the partials added in thread order (reproducible for a thread count), and
 *    the true residual that confirms convergence is summed in plain float64
 *    (orc_cg uses Dot2 there), so its iterates agree with orc_cg's to
 *    rounding.
 * Shares no code with the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

int orc_omp_threads(void) { return omp_get_max_threads(); }

void orc_csr_spmv_omp(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                      const double *x, double *y, double alpha, double beta)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s += val[p] * x[col[p]];
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* Thread t of T owns the entries [t*n/T, (t+1)*n/T). */
static int32_t block_lo(int32_t n, int t, int T) { return (int32_t)((int64_t)n * t / T); }

/* Partial sums, one per thread over its own block, are added in thread
 * order: the same bits on every run with the same thread count (an OpenMP
 * reduction clause combines the partials in an unspecified order). */
#define ORC_MAX_THREADS 1024

static double dot_omp(int32_t n, const double *a, const double *b)
{
    double part[ORC_MAX_THREADS];
    int nt = 1;
#pragma omp parallel num_threads(omp_get_max_threads() < ORC_MAX_THREADS ? omp_get_max_threads() : ORC_MAX_THREADS)
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
        double s = 0.0;
        for (int32_t i = block_lo(n, t, T); i < block_lo(n, t + 1, T); ++i) s += a[i] * b[i];
        part[t] = s;
        if (t == 0) nt = T;
    }
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += part[t];
    return s;
}

/* True residual r = b - A x (plain float64 row sums) and its 2-norm. */
static double residual_omp(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                           const double *b, const double *x, double *r)
{
    double part[ORC_MAX_THREADS];
    int nt = 1;
#pragma omp parallel num_threads(omp_get_max_threads() < ORC_MAX_THREADS ? omp_get_max_threads() : ORC_MAX_THREADS)
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
        double s2 = 0.0;
        for (int32_t i = block_lo(n, t, T); i < block_lo(n, t + 1, T); ++i) {
            double s = b[i];
            for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s -= val[p] * x[col[p]];
            r[i] = s;
            s2 += s * s;
        }
        part[t] = s2;
        if (t == 0) nt = T;
    }
    double s2 = 0.0;
    for (int t = 0; t < nt; ++t) s2 += part[t];
    return sqrt(s2);
}

typedef struct {
    int32_t status, iters, spmv_count, outer_iters;
    double relres_recursive, relres_true;
} orc_omp_info;

enum { OMP_OK = 0, OMP_NOT_CONVERGED = 1, OMP_BREAKDOWN = 2, OMP_NONFINITE = 3, OMP_ZERO_DIAG = 4,
       OMP_EARG = -1, OMP_ENOMEM = -4 };

int orc_cg_omp(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, const double *b,
               double *x, double tol, int32_t maxit, int32_t precond, orc_omp_info *info)
{
    memset(info, 0, sizeof(*info));
    if (precond != 0 && precond != 1) return info->status = OMP_EARG;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *diag = precond ? malloc(sizeof(double) * n) : NULL;
    if (!r || !z || !p || !q || (precond && !diag)) { info->status = OMP_ENOMEM; goto out; }
    if (precond) {
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int32_t i = 0; i < n; ++i) {
            double d = 0.0;
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i) d = val[k];
            if (d == 0.0 || !isfinite(d)) bad = 1;
            diag[i] = d;
        }
        if (bad) { info->status = OMP_ZERO_DIAG; goto out; }
    }
    /* x0 = 0, so r = b */
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    const double bn = sqrt(dot_omp(n, b, b));
    if (!isfinite(bn)) { info->status = OMP_NONFINITE; goto out; }
    if (bn == 0.0) { info->status = OMP_OK; goto out; }
    int restart = 1;
    double rho = 0.0;
    info->status = OMP_NOT_CONVERGED;
    while (info->status == OMP_NOT_CONVERGED) {
        if (restart) {
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) { z[i] = diag ? r[i] / diag[i] : r[i]; p[i] = z[i]; }
            rho = dot_omp(n, r, z);
            restart = 0;
        }
        if (info->iters >= maxit) break;
        orc_csr_spmv_omp(n, rowptr, col, val, p, q, 1.0, 0.0);
        info->iters += 1;
        info->spmv_count += 1;
        const double pq = dot_omp(n, p, q);
        if (!isfinite(pq)) { info->status = OMP_NONFINITE; break; }
        if (pq <= 0.0) { info->status = OMP_BREAKDOWN; break; }
        const double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        const double rn = sqrt(dot_omp(n, r, r));
        info->relres_recursive = rn / bn;
        if (!isfinite(rn)) { info->status = OMP_NONFINITE; break; }
        if (rn <= tol * bn) {
            const double tn = residual_omp(n, rowptr, col, val, b, x, r); /* r <- true residual */
            if (tn <= tol * bn) { info->status = OMP_OK; break; }
            restart = 1;
            continue;
        }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) z[i] = diag ? r[i] / diag[i] : r[i];
        const double rho_new = dot_omp(n, r, z);
        const double beta = rho_new / rho;
        rho = rho_new;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    info->relres_true = residual_omp(n, rowptr, col, val, b, x, q) / bn;
out:
    free(r); free(z); free(p); free(q); free(diag);
    return info->status;
}
