/*
 * CPU oracle for the CSR SpMV / Jacobi-PCG path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the bench's CPU-baseline leg may
 * load this library.  The product library never links, loads or calls it, and
 * it shares no source, header, table or helper with the HIP implementation.
 *
 * Plain, serial, slow and obviously correct.  Build with -O2 -ffp-contract=off
 * so that the compiler never fuses a multiply and an add on its own; the only
 * fused operations are the explicit fma() calls in the vector updates, where
 * the plain definition is "exact result, rounded once".
 *
 * Precision: sums are accumulated in long double (x87 80-bit, 64-bit
 * significand) and rounded to double once, so the oracle's own rounding error
 * is far below the GPU tolerance and the whole tolerance budget belongs to the
 * GPU side.
 *
 * What each function follows:
 *  - The matrix is CSR ("compressed sparse row", the MATAIJ type of the
 *    paper's Sec. 4, with 32-bit column indices and the per-nonzero byte
 *    count of Challenge A7 in Sec. 3).
 *  - The vector operations are the Vec operations of Sec. 5.1 (VecAXPY
 *    y <- alpha x + y) and the inner products / norms of Sec. 4 (Response F3,
 *    Response A1).
 *  - The solver is the conjugate gradient method with a pointwise Jacobi
 *    preconditioner (CG is named in Sec. 5.5, Jacobi in Sec. 5.3).  The paper
 *    prints no CG algorithm, so this is the textbook preconditioned CG
 *    (Hestenes & Stiefel 1952), with the readings listed at orc_pcg().
 *  - The multigrid functions (orc_mg_*) follow the geometric multigrid of
 *    Sec. 5.3 (Chebyshev-Jacobi smoothing, direct coarsest solve), with the
 *    aggregation reading of the grid transfers stated at orc_mg_coarse_shape().
 *
 * Every function is pinned by CPU tests against values fixed by mathematics
 * (closed-form eigenpairs, exact integer arithmetic, brute-force dense solves,
 * finite termination), not against itself.
 *
 * Parallel build (only for timing the oracle on all host cores): the same
 * file compiled with -fopenmp runs the row and vector loops of the SpMV, the
 * vector updates and the PCG with "omp parallel for" (static schedule), and
 * forms each inner product as fixed chunks of ORC_CHUNK entries summed in long
 * double, then the chunk sums in chunk order (the same bits for any thread
 * count).  The serial build ignores the pragmas and keeps one long double sum.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the loops run on: 1 in the serial build. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#ifdef _OPENMP
#define ORC_CHUNK 32768
/* sum_i x_i y_i over fixed chunks (parallel build only). */
static long double chunked_dot(int32_t n, const double *x, const double *y)
{
    const int32_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    long double *part = (long double *)malloc(sizeof(long double) * (size_t)(nc > 0 ? nc : 1));
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t e = (c + 1) * (int64_t)ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
        long double s = 0.0L;
        for (int32_t i = c * ORC_CHUNK; i < e; ++i) s += (long double)x[i] * (long double)y[i];
        part[c] = s;
    }
    long double s = 0.0L;
    for (int32_t c = 0; c < nc; ++c) s += part[c];
    free(part);
    return s;
}
#endif

/* y_i = sum_k val[k] * x[col[k]] over k in [rowptr[i], rowptr[i+1]). */
void orc_spmv(int32_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += (long double)val[k] * (long double)x[col[k]];
        y[i] = (double)s;
    }
}

/* Same product for FP32 values and FP32 x: the product of two floats is exact
 * in long double, the sum is accumulated in long double and rounded to float
 * once (the reference the FP32-value kernels are judged against). */
void orc_spmv_f32(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const float *val, const float *x, float *y)
{
    for (int32_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += (long double)val[k] * (long double)x[col[k]];
        y[i] = (float)s;
    }
}

/* sum_i |val| * |x| per row: the scale the per-entry SpMV tolerance uses. */
void orc_spmv_abs(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += fabsl((long double)val[k] * (long double)x[col[k]]);
        y[i] = (double)s;
    }
}

/* Selected rows only: y[j] = (A x)_{rows[j]} (for spot checks at full size). */
void orc_spmv_rows(int32_t nrows, const int32_t *rows, const int32_t *rowptr,
                   const int32_t *col, const double *val, const double *x,
                   double *y, double *yabs)
{
    for (int32_t j = 0; j < nrows; ++j) {
        int32_t i = rows[j];
        long double s = 0.0L, a = 0.0L;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            long double t = (long double)val[k] * (long double)x[col[k]];
            s += t;
            a += fabsl(t);
        }
        y[j] = (double)s;
        if (yabs) yabs[j] = (double)a;
    }
}

double orc_dot(int32_t n, const double *x, const double *y)
{
#ifdef _OPENMP
    return (double)chunked_dot(n, x, y);
#endif
    long double s = 0.0L;
    for (int32_t i = 0; i < n; ++i)
        s += (long double)x[i] * (long double)y[i];
    return (double)s;
}

double orc_nrm2(int32_t n, const double *x)
{
#ifdef _OPENMP
    return (double)sqrtl(chunked_dot(n, x, x));
#endif
    long double s = 0.0L;
    for (int32_t i = 0; i < n; ++i)
        s += (long double)x[i] * (long double)x[i];
    return (double)sqrtl(s);
}

/* y <- alpha x + y, exact product-plus-sum rounded once. */
void orc_axpy(int32_t n, double alpha, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        y[i] = fma(alpha, x[i], y[i]);
}

/* y <- x + beta y, exact product-plus-sum rounded once. */
void orc_aypx(int32_t n, double beta, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        y[i] = fma(beta, y[i], x[i]);
}

/* Jacobi preconditioner setup: dinv_i = 1 / a_ii.  Returns 0, or -4 if some
 * row has no stored diagonal or a zero diagonal. */
int orc_diag_inv(int32_t n, const int32_t *rowptr, const int32_t *col,
                 const double *val, double *dinv)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) d += val[k];
        if (d == 0.0) return ORC_EZERODIAG;
        dinv[i] = 1.0 / d;
    }
    return 0;
}

/* Jacobi PCApply: z_i = dinv_i * r_i. */
void orc_jacobi_apply(int32_t n, const double *dinv, const double *r, double *z)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
}

static int finite_d(double v) { return isfinite(v); }

/* The preconditioner of orc_pcg: the Jacobi PCApply with ctx = dinv. */
static int jacobi_pc(void *ctx, int32_t n, const double *r, double *z)
{
    orc_jacobi_apply(n, (const double *)ctx, r, z);
    return 0;
}

/*
 * Jacobi-preconditioned conjugate gradient, FP64.
 *
 * Readings (the paper prints no algorithm and no stopping rule):
 *  - x0 = 0 unless x0_nonzero; r = b - A x0.
 *  - Convergence on the unpreconditioned recursive residual:
 *    ||r_k||_2 <= max(rtol ||b||_2, atol).  Reason RTOL if ||r_k|| <= rtol ||b||,
 *    otherwise ATOL.  ||b|| = 0 returns x = 0, CONVERGED_ATOL, 0 iterations.
 *  - When the recursive test passes, the true residual b - A x is formed; if
 *    it fails the same test, CG restarts from the current x with the true
 *    residual (p = z); after 3 such restarts the solve stops with BREAKDOWN.
 *  - eta = p.Ap <= 0 -> INDEFINITE_MAT (x not updated); rho' = r.z < 0 ->
 *    INDEFINITE_PC; rho' = 0 -> BREAKDOWN; any non-finite scalar -> NANORINF.
 *  - k reaching maxit without convergence -> DIVERGED_ITS.
 * hist (if not NULL, hist_len entries) receives ||r_k|| for k = 0.. .
 */
int orc_pcg(int32_t n, const int32_t *rowptr, const int32_t *col,
            const double *val, const double *b, double *x, double rtol,
            double atol, int32_t maxit, int32_t x0_nonzero, double *hist,
            int32_t hist_len, orc_pcg_result *res)
{
    memset(res, 0, sizeof(*res));
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!dinv) return ORC_ENOMEM;
    int status = orc_diag_inv(n, rowptr, col, val, dinv);
    if (!status)
        status = orc_pcg_pc(n, rowptr, col, val, b, x, rtol, atol, maxit, x0_nonzero,
                            jacobi_pc, dinv, hist, hist_len, res);
    free(dinv);
    return status;
}

/* The same iteration with the preconditioner given as z = pc(r) (a
 * multigrid cycle, for instance); a non-zero return of pc ends the solve
 * with that status. */
int orc_pcg_pc(int32_t n, const int32_t *rowptr, const int32_t *col,
               const double *val, const double *b, double *x, double rtol,
               double atol, int32_t maxit, int32_t x0_nonzero, orc_pc_fn pc,
               void *pc_ctx, double *hist, int32_t hist_len, orc_pcg_result *res)
{
    memset(res, 0, sizeof(*res));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = 0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }

    double bnorm = orc_nrm2(n, b);
    res->bnorm = bnorm;
    double thresh = rtol * bnorm > atol ? rtol * bnorm : atol;
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        res->reason = ORC_CONVERGED_ATOL;
        if (hist && hist_len > 0) hist[0] = 0.0;
        goto done;
    }
    if (x0_nonzero) {
        orc_spmv(n, rowptr, col, val, x, q);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    } else {
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    }
    double rnorm = orc_nrm2(n, r);
    res->rnorm0 = rnorm;
    if (hist && hist_len > 0) hist[0] = rnorm;
    int32_t k = 0;
    int restarts = 0;
    double rho = 0.0;

    for (;;) { /* (re)start from the current x with a true residual in r */
        if (!finite_d(rnorm)) { res->reason = ORC_DIVERGED_NANORINF; break; }
        if (rnorm <= thresh) {
            res->reason = rnorm <= rtol * bnorm ? ORC_CONVERGED_RTOL : ORC_CONVERGED_ATOL;
            break;
        }
        if ((status = pc(pc_ctx, n, r, z)) != 0) goto done;
        rho = orc_dot(n, r, z);
        if (!finite_d(rho)) { res->reason = ORC_DIVERGED_NANORINF; break; }
        if (rho < 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_PC; break; }
        if (rho == 0.0) { res->reason = ORC_DIVERGED_BREAKDOWN; break; }
        memcpy(p, z, sizeof(double) * (size_t)n);

        int restart = 0;
        while (!res->reason && !restart) {
            if (k >= maxit) { res->reason = ORC_DIVERGED_ITS; break; }
            orc_spmv(n, rowptr, col, val, p, q);
            double eta = orc_dot(n, p, q);
            if (!finite_d(eta)) { res->reason = ORC_DIVERGED_NANORINF; break; }
            if (eta <= 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_MAT; break; }
            double alpha = rho / eta;
            orc_axpy(n, alpha, p, x);
            orc_axpy(n, -alpha, q, r);
            ++k;
            rnorm = orc_nrm2(n, r);
            if (hist && k < hist_len) hist[k] = rnorm;
            if (!finite_d(rnorm)) { res->reason = ORC_DIVERGED_NANORINF; break; }
            if (rnorm <= thresh) {
                /* recursive test passed: confirm with the true residual */
                orc_spmv(n, rowptr, col, val, x, q);
#pragma omp parallel for schedule(static)
                for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
                double tn = orc_nrm2(n, r);
                if (tn <= thresh) {
                    rnorm = tn;
                    res->reason = tn <= rtol * bnorm ? ORC_CONVERGED_RTOL : ORC_CONVERGED_ATOL;
                    break;
                }
                if (restarts == 3) { rnorm = tn; res->reason = ORC_DIVERGED_BREAKDOWN; break; }
                ++restarts;
                rnorm = tn;
                restart = 1;
                break;
            }
            if (k >= maxit) { res->reason = ORC_DIVERGED_ITS; break; }
            if ((status = pc(pc_ctx, n, r, z)) != 0) goto done;
            double rho_new = orc_dot(n, r, z);
            if (!finite_d(rho_new)) { res->reason = ORC_DIVERGED_NANORINF; break; }
            if (rho_new < 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_PC; break; }
            if (rho_new == 0.0) { res->reason = ORC_DIVERGED_BREAKDOWN; break; }
            double beta = rho_new / rho;
            orc_aypx(n, beta, z, p);
            rho = rho_new;
        }
        if (res->reason) break;
    }
    res->iterations = k;
    res->restarts = restarts;
    res->rnorm = rnorm;
    /* report the true relative residual from a fresh accurate product */
    orc_spmv(n, rowptr, col, val, x, q);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    res->true_rel_residual = orc_nrm2(n, r) / bnorm;

done:
    free(r); free(z); free(p); free(q);
    return status;
}

/* Dense SPD solve by Cholesky factorisation A = L L^T (brute-force check for
 * small systems).  A is n*n row-major and is overwritten by L; b is
 * overwritten by the solution.  Returns 0, or -1 if A is not positive
 * definite. */
/*
 * Single-reduction preconditioned CG (Chronopoulos & Gear, J. Comput. Appl.
 * Math. 25, 1989): the same Krylov iterates as orc_pcg in exact arithmetic,
 * but the two inner products of an iteration are formed together, from
 * u = D^-1 r and w = A u, so a parallel implementation needs one reduction
 * phase per iteration (Sec. 4, Challenge A1: synchronisation points).  The
 * recurrences (s = A p carried as a vector):
 *
 *   u = D^-1 r, w = A u, gamma = (r, u), delta = (w, u)
 *   first step:  beta = 0, alpha = gamma / delta
 *   later steps: beta = gamma / gamma_prev,
 *                alpha = gamma / (delta - beta gamma / alpha_prev)
 *   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
 *
 * Stopping rule, true-residual restarts (a restart starts a new "first
 * step"), breakdown reasons and results as in orc_pcg; a non-positive
 * alpha denominator is INDEFINITE_MAT.
 */
int orc_pcg_sr(int32_t n, const int32_t *rowptr, const int32_t *col,
               const double *val, const double *b, double *x, double rtol,
               double atol, int32_t maxit, int32_t x0_nonzero, double *hist,
               int32_t hist_len, orc_pcg_result *res)
{
    memset(res, 0, sizeof(*res));
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *dinv = (double *)malloc(bytes), *r = (double *)malloc(bytes), *u = (double *)malloc(bytes);
    double *w = (double *)malloc(bytes), *p = (double *)malloc(bytes), *s = (double *)malloc(bytes);
    double *t = (double *)malloc(bytes);
    int status = 0;
    if (!dinv || !r || !u || !w || !p || !s || !t) { status = ORC_ENOMEM; goto done; }
    status = orc_diag_inv(n, rowptr, col, val, dinv);
    if (status) goto done;

    double bnorm = orc_nrm2(n, b);
    res->bnorm = bnorm;
    double thresh = rtol * bnorm > atol ? rtol * bnorm : atol;
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        res->reason = ORC_CONVERGED_ATOL;
        if (hist && hist_len > 0) hist[0] = 0.0;
        goto done;
    }
    if (x0_nonzero) {
        orc_spmv(n, rowptr, col, val, x, t);
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    } else {
        for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    }
    double rnorm = orc_nrm2(n, r);
    res->rnorm0 = rnorm;
    if (hist && hist_len > 0) hist[0] = rnorm;
    int32_t k = 0;
    int restarts = 0;

    for (;;) { /* (re)start from the current x with a true residual in r */
        if (!finite_d(rnorm)) { res->reason = ORC_DIVERGED_NANORINF; break; }
        if (rnorm <= thresh) {
            res->reason = rnorm <= rtol * bnorm ? ORC_CONVERGED_RTOL : ORC_CONVERGED_ATOL;
            break;
        }
        orc_jacobi_apply(n, dinv, r, u);
        orc_spmv(n, rowptr, col, val, u, w);
        double gamma = orc_dot(n, r, u);
        double delta = orc_dot(n, w, u);
        if (!finite_d(gamma)) { res->reason = ORC_DIVERGED_NANORINF; break; }
        if (gamma < 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_PC; break; }
        if (gamma == 0.0) { res->reason = ORC_DIVERGED_BREAKDOWN; break; }
        int first = 1;
        double gamma_prev = 0.0, alpha_prev = 0.0;
        int restart = 0;
        while (!res->reason && !restart) {
            if (k >= maxit) { res->reason = ORC_DIVERGED_ITS; break; }
            double alpha, beta;
            if (first) {
                beta = 0.0;
                if (!finite_d(delta)) { res->reason = ORC_DIVERGED_NANORINF; break; }
                if (delta <= 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_MAT; break; }
                alpha = gamma / delta;
            } else {
                beta = gamma / gamma_prev;
                const double den = delta - beta * gamma / alpha_prev;
                if (!finite_d(den)) { res->reason = ORC_DIVERGED_NANORINF; break; }
                if (den <= 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_MAT; break; }
                alpha = gamma / den;
            }
            for (int32_t i = 0; i < n; ++i) {
                p[i] = first ? u[i] : u[i] + beta * p[i];
                s[i] = first ? w[i] : w[i] + beta * s[i];
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * s[i];
            }
            first = 0;
            ++k;
            rnorm = orc_nrm2(n, r);
            if (hist && k < hist_len) hist[k] = rnorm;
            if (!finite_d(rnorm)) { res->reason = ORC_DIVERGED_NANORINF; break; }
            if (rnorm <= thresh) {
                orc_spmv(n, rowptr, col, val, x, t);
                for (int32_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
                double tn = orc_nrm2(n, r);
                if (tn <= thresh) {
                    rnorm = tn;
                    res->reason = tn <= rtol * bnorm ? ORC_CONVERGED_RTOL : ORC_CONVERGED_ATOL;
                    break;
                }
                if (restarts == 3) { rnorm = tn; res->reason = ORC_DIVERGED_BREAKDOWN; break; }
                ++restarts;
                rnorm = tn;
                restart = 1;
                break;
            }
            if (k >= maxit) { res->reason = ORC_DIVERGED_ITS; break; }
            orc_jacobi_apply(n, dinv, r, u);
            orc_spmv(n, rowptr, col, val, u, w);
            gamma_prev = gamma;
            alpha_prev = alpha;
            gamma = orc_dot(n, r, u);
            delta = orc_dot(n, w, u);
            if (!finite_d(gamma)) { res->reason = ORC_DIVERGED_NANORINF; break; }
            if (gamma < 0.0) { res->reason = ORC_DIVERGED_INDEFINITE_PC; break; }
            if (gamma == 0.0) { res->reason = ORC_DIVERGED_BREAKDOWN; break; }
        }
        if (res->reason) break;
    }
    res->iterations = k;
    res->restarts = restarts;
    res->rnorm = rnorm;
    orc_spmv(n, rowptr, col, val, x, t);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    res->true_rel_residual = orc_nrm2(n, r) / bnorm;

done:
    free(dinv); free(r); free(u); free(w); free(p); free(s); free(t);
    return status;
}

/*
 * Chebyshev acceleration of the Jacobi iteration: the smoother that the
 * paper's geometric multigrid runs on every level but the coarsest (Sec. 5.3,
 * "Jacobi-preconditioned Chebyshev smoothers").  The paper gives no formulas;
 * this is the textbook three-term Chebyshev iteration for the preconditioned
 * system D^-1 A x = D^-1 b (D = diag(A)) on a spectral interval [emin, emax]
 * of D^-1 A (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
 * Sec. 12.3, Chebyshev acceleration):
 *
 *   theta = (emax + emin) / 2, delta = (emax - emin) / 2, sigma = theta / delta
 *   r_0 = b - A x_0,  rho_0 = 1 / sigma,  d_0 = D^-1 r_0 / theta
 *   for k = 0 .. steps-1:
 *       x_{k+1} = x_k + d_k
 *       r_{k+1} = r_k - A d_k
 *       rho_{k+1} = 1 / (2 sigma - rho_k)
 *       d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) D^-1 r_{k+1}
 *
 * The error after k steps is P_k(D^-1 A) e_0 with
 * P_k(t) = T_k((theta - t) / delta) / T_k(sigma), T_k the Chebyshev
 * polynomial of the first kind.  x (in: x_0 when x0_nonzero, else ignored and
 * taken as 0; out: x_steps); r_out (optional) receives r_steps.
 * Returns 0, ORC_EZERODIAG, ORC_ENOMEM, or -1 for emin/emax outside
 * 0 < emin < emax.
 */
int orc_chebyshev(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, const double *b, double *x, double *r_out,
                  int32_t steps, double emin, double emax, int32_t x0_nonzero)
{
    if (!(emin > 0.0) || !(emax > emin)) return -1;
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *dinv = (double *)malloc(bytes);
    double *r = (double *)malloc(bytes);
    double *d = (double *)malloc(bytes);
    double *ad = (double *)malloc(bytes);
    if (!dinv || !r || !d || !ad) {
        free(dinv); free(r); free(d); free(ad);
        return ORC_ENOMEM;
    }
    int rc = orc_diag_inv(n, rowptr, col, val, dinv);
    if (rc) {
        free(dinv); free(r); free(d); free(ad);
        return rc;
    }
    const double theta = 0.5 * (emax + emin);
    const double delta = 0.5 * (emax - emin);
    const double sigma = theta / delta;
    if (x0_nonzero) {
        orc_spmv(n, rowptr, col, val, x, ad);
        for (int32_t i = 0; i < n; ++i) r[i] = b[i] - ad[i];
    } else {
        for (int32_t i = 0; i < n; ++i) {
            x[i] = 0.0;
            r[i] = b[i];
        }
    }
    double rho = 1.0 / sigma;
    for (int32_t i = 0; i < n; ++i) d[i] = dinv[i] * r[i] / theta;
    for (int32_t k = 0; k < steps; ++k) {
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + d[i];
        orc_spmv(n, rowptr, col, val, d, ad);
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - ad[i];
        const double rho_next = 1.0 / (2.0 * sigma - rho);
        const double c1 = rho_next * rho;
        const double c2 = 2.0 * rho_next / delta;
        for (int32_t i = 0; i < n; ++i) d[i] = c1 * d[i] + c2 * (dinv[i] * r[i]);
        rho = rho_next;
    }
    if (r_out) memcpy(r_out, r, sizeof(double) * (size_t)n);
    free(dinv); free(r); free(d); free(ad);
    return 0;
}

/* Gershgorin bound on the spectrum of D^-1 A:
 * max_i sum_j |a_ij| / |a_ii| (an upper bound on |lambda| for every
 * eigenvalue).  Returns ORC_EZERODIAG (and sets *bound to 0) when a row has
 * no nonzero diagonal. */
int orc_gershgorin(int32_t n, const int32_t *rowptr, const int32_t *col,
                   const double *val, double *bound)
{
    double m = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double diag = 0.0;
        long double s = 0.0L;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            s += fabsl((long double)val[k]);
            if (col[k] == i) diag = val[k];
        }
        if (diag == 0.0) {
            *bound = 0.0;
            return ORC_EZERODIAG;
        }
        const double g = (double)(s / fabsl((long double)diag));
        if (g > m) m = g;
    }
    *bound = m;
    return 0;
}

/* Factor step alone: A (n*n, row-major) is overwritten by L in its lower
 * triangle.  Returns 0, or -1 if A is not positive definite. */
int orc_dense_cholesky_factor(int32_t n, double *A)
{
    for (int32_t j = 0; j < n; ++j) {
        long double s = A[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k)
            s -= (long double)A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0.0L)) return -1;
        double ljj = (double)sqrtl(s);
        A[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            long double t = A[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k)
                t -= (long double)A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = (double)(t / ljj);
        }
    }
    return 0;
}

/* Substitution step alone: b <- L^-T L^-1 b with L from orc_dense_cholesky_factor. */
void orc_dense_cholesky_subst(int32_t n, const double *L, double *b)
{
    for (int32_t i = 0; i < n; ++i) { /* L y = b */
        long double t = b[i];
        for (int32_t k = 0; k < i; ++k) t -= (long double)L[(size_t)i * n + k] * b[k];
        b[i] = (double)(t / L[(size_t)i * n + i]);
    }
    for (int32_t i = n - 1; i >= 0; --i) { /* L^T x = y */
        long double t = b[i];
        for (int32_t k = i + 1; k < n; ++k) t -= (long double)L[(size_t)k * n + i] * b[k];
        b[i] = (double)(t / L[(size_t)i * n + i]);
    }
}

int orc_dense_cholesky_solve(int32_t n, double *A, double *b)
{
    if (orc_dense_cholesky_factor(n, A)) return -1;
    orc_dense_cholesky_subst(n, A, b);
    return 0;
}

/*
 * Geometric multigrid on a logically structured grid (Sec. 5.3: the
 * driven-cavity study runs PETSc's multigrid with Jacobi-preconditioned
 * Chebyshev smoothers on every level but the coarsest, which is solved
 * directly).  The paper fixes neither the grid transfers nor the coarse
 * operators; the reading taken here is aggregation:
 *  - a grid of shape (s_0, s_1, s_2) (s_0 fastest; unused dimensions 1)
 *    coarsens to shape ceil(s_d / 2), and fine point (i_0, i_1, i_2) belongs
 *    to the aggregate (floor(i_0/2), floor(i_1/2), floor(i_2/2));
 *  - prolongation P is piecewise constant over the aggregates (P_iI = 1 when
 *    i belongs to I), restriction is P^T, and the coarse operator is the
 *    Galerkin product A_c = P^T A P.
 * The cycle itself (smoothing, over-correction, V or W recursion, the direct
 * coarsest solve) is composed from these functions by the Python wrapper.
 */
void orc_mg_coarse_shape(int32_t dim, const int32_t *shape, int32_t *cshape)
{
    for (int32_t d = 0; d < 3; ++d) cshape[d] = d < dim ? (shape[d] + 1) / 2 : 1;
}

/* Grid coordinates of row i (s_0 fastest). */
static void grid_coords(int32_t dim, const int32_t *shape, int64_t i, int32_t *c)
{
    for (int32_t d = 0; d < 3; ++d) {
        const int32_t s = d < dim ? shape[d] : 1;
        c[d] = (int32_t)(i % s);
        i /= s;
    }
}

/* Coarse index of the aggregate that holds fine row i. */
static int32_t aggregate_of(int32_t dim, const int32_t *shape, const int32_t *cshape, int64_t i)
{
    int32_t c[3];
    grid_coords(dim, shape, i, c);
    return (c[0] / 2) + cshape[0] * ((c[1] / 2) + cshape[1] * (c[2] / 2));
}

/*
 * A_c = P^T A P:  (A_c)_IJ = sum of a_ij over fine i in I and j in J.
 * Written out by definition: for each coarse row I the entries of its fine
 * rows are accumulated (long double, rounded once) into the coarse columns
 * they map to, with a sparse accumulator; every coarse column that receives
 * at least one fine entry is stored, in ascending order, even if its sum is 0.
 * The output arrays need room for nc + 1 row pointers and (at most) nnz
 * entries.  Returns the coarse nnz, or a negative status (ORC_ENOMEM, or -1
 * for n different from the grid's point count).
 */
int64_t orc_mg_galerkin(int32_t n, const int32_t *rowptr, const int32_t *col,
                        const double *val, int32_t dim, const int32_t *shape,
                        int32_t *crowptr, int32_t *ccol, double *cval)
{
    int32_t cs[3], s[3];
    orc_mg_coarse_shape(dim, shape, cs);
    for (int32_t d = 0; d < 3; ++d) s[d] = d < dim ? shape[d] : 1;
    if ((int64_t)s[0] * s[1] * s[2] != n) return -1;
    const int32_t nc = cs[0] * cs[1] * cs[2];
    long double *acc = (long double *)malloc(sizeof(long double) * (size_t)(nc > 0 ? nc : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    if (!acc || !mark || !list) {
        free(acc); free(mark); free(list);
        return ORC_ENOMEM;
    }
    for (int32_t J = 0; J < nc; ++J) mark[J] = -1;
    int64_t nnz_c = 0;
    crowptr[0] = 0;
    for (int32_t I = 0; I < nc; ++I) {
        int32_t c[3];
        grid_coords(dim, cs, I, c);
        int32_t cnt = 0;
        /* the fine points of aggregate I: coordinates 2c_d and 2c_d + 1 where
         * they exist */
        for (int32_t a2 = 0; a2 < 2; ++a2)
            for (int32_t a1 = 0; a1 < 2; ++a1)
                for (int32_t a0 = 0; a0 < 2; ++a0) {
                    const int32_t f0 = 2 * c[0] + a0, f1 = 2 * c[1] + a1, f2 = 2 * c[2] + a2;
                    if (f0 >= s[0] || f1 >= s[1] || f2 >= s[2]) continue;
                    const int32_t i = f0 + s[0] * (f1 + s[1] * f2);
                    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                        const int32_t J = aggregate_of(dim, shape, cs, col[k]);
                        if (mark[J] != I) {
                            mark[J] = I;
                            acc[J] = 0.0L;
                            list[cnt++] = J;
                        }
                        acc[J] += (long double)val[k];
                    }
                }
        for (int32_t u = 1; u < cnt; ++u) { /* insertion sort of the columns */
            const int32_t v = list[u];
            int32_t w = u - 1;
            while (w >= 0 && list[w] > v) {
                list[w + 1] = list[w];
                --w;
            }
            list[w + 1] = v;
        }
        for (int32_t u = 0; u < cnt; ++u) {
            ccol[nnz_c] = list[u];
            cval[nnz_c] = (double)acc[list[u]];
            ++nnz_c;
        }
        crowptr[I + 1] = (int32_t)nnz_c;
    }
    free(acc); free(mark); free(list);
    return nnz_c;
}

/* Restriction b_c = P^T r: the sum of the fine values of each aggregate
 * (long double, rounded once). */
void orc_mg_restrict(int32_t dim, const int32_t *shape, const double *r, double *bc)
{
    int32_t cs[3], s[3];
    orc_mg_coarse_shape(dim, shape, cs);
    for (int32_t d = 0; d < 3; ++d) s[d] = d < dim ? shape[d] : 1;
    const int32_t nc = cs[0] * cs[1] * cs[2];
    for (int32_t I = 0; I < nc; ++I) {
        int32_t c[3];
        grid_coords(dim, cs, I, c);
        long double t = 0.0L;
        for (int32_t a2 = 0; a2 < 2; ++a2)
            for (int32_t a1 = 0; a1 < 2; ++a1)
                for (int32_t a0 = 0; a0 < 2; ++a0) {
                    const int32_t f0 = 2 * c[0] + a0, f1 = 2 * c[1] + a1, f2 = 2 * c[2] + a2;
                    if (f0 >= s[0] || f1 >= s[1] || f2 >= s[2]) continue;
                    t += r[f0 + s[0] * (f1 + s[1] * f2)];
                }
        bc[I] = (double)t;
    }
}

/* Coarse-grid correction x <- x + omega P x_c (product and sum rounded once). */
void orc_mg_prolong(int32_t dim, const int32_t *shape, double omega, const double *xc,
                    double *x)
{
    int32_t cs[3], s[3];
    orc_mg_coarse_shape(dim, shape, cs);
    for (int32_t d = 0; d < 3; ++d) s[d] = d < dim ? shape[d] : 1;
    const int64_t n = (int64_t)s[0] * s[1] * s[2];
    for (int64_t i = 0; i < n; ++i)
        x[i] = fma(omega, xc[aggregate_of(dim, shape, cs, i)], x[i]);
}
