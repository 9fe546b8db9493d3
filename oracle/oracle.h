/* CPU oracle for the CSR SpMV / Jacobi-PCG path -- TEST INFRASTRUCTURE ONLY.
 * Used by the test suite, the smoke check and the bench's CPU-baseline leg;
 * never by the product library.  Shares nothing with the HIP implementation. */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

enum {
    ORC_EZERODIAG = -4,
    ORC_ENOMEM = -2,
};

enum {
    ORC_CONVERGED_RTOL = 1,
    ORC_CONVERGED_ATOL = 2,
    ORC_DIVERGED_ITS = -1,
    ORC_DIVERGED_INDEFINITE_MAT = -2,
    ORC_DIVERGED_INDEFINITE_PC = -3,
    ORC_DIVERGED_NANORINF = -4,
    ORC_DIVERGED_BREAKDOWN = -5,
};

typedef struct {
    int32_t reason;
    int32_t iterations;
    int32_t restarts;
    int32_t pad_;
    double rnorm0;
    double rnorm;
    double bnorm;
    double true_rel_residual;
} orc_pcg_result;

void orc_spmv(int32_t n, const int32_t *rowptr, const int32_t *col,
              const double *val, const double *x, double *y);
void orc_spmv_f32(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const float *val, const float *x, float *y);
void orc_spmv_abs(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, const double *x, double *y);
void orc_spmv_rows(int32_t nrows, const int32_t *rows, const int32_t *rowptr,
                   const int32_t *col, const double *val, const double *x,
                   double *y, double *yabs);
double orc_dot(int32_t n, const double *x, const double *y);
double orc_nrm2(int32_t n, const double *x);
void orc_axpy(int32_t n, double alpha, const double *x, double *y);
void orc_aypx(int32_t n, double beta, const double *x, double *y);
int orc_diag_inv(int32_t n, const int32_t *rowptr, const int32_t *col,
                 const double *val, double *dinv);
void orc_jacobi_apply(int32_t n, const double *dinv, const double *r, double *z);
/* z = M^-1 r for a preconditioner M; returns 0 or a status that ends the solve. */
typedef int (*orc_pc_fn)(void *ctx, int32_t n, const double *r, double *z);

int orc_pcg(int32_t n, const int32_t *rowptr, const int32_t *col,
            const double *val, const double *b, double *x, double rtol,
            double atol, int32_t maxit, int32_t x0_nonzero, double *hist,
            int32_t hist_len, orc_pcg_result *res);
int orc_chebyshev(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, const double *b, double *x, double *r_out,
                  int32_t steps, double emin, double emax, int32_t x0_nonzero);
int orc_gershgorin(int32_t n, const int32_t *rowptr, const int32_t *col,
                   const double *val, double *bound);
int orc_pcg_sr(int32_t n, const int32_t *rowptr, const int32_t *col,
               const double *val, const double *b, double *x, double rtol,
               double atol, int32_t maxit, int32_t x0_nonzero, double *hist,
               int32_t hist_len, orc_pcg_result *res);
int orc_pcg_pc(int32_t n, const int32_t *rowptr, const int32_t *col,
               const double *val, const double *b, double *x, double rtol,
               double atol, int32_t maxit, int32_t x0_nonzero, orc_pc_fn pc,
               void *pc_ctx, double *hist, int32_t hist_len, orc_pcg_result *res);
int orc_dense_cholesky_solve(int32_t n, double *A, double *b);
int orc_dense_cholesky_factor(int32_t n, double *A);
void orc_dense_cholesky_subst(int32_t n, const double *L, double *b);
void orc_mg_coarse_shape(int32_t dim, const int32_t *shape, int32_t *cshape);
int64_t orc_mg_galerkin(int32_t n, const int32_t *rowptr, const int32_t *col,
                        const double *val, int32_t dim, const int32_t *shape,
                        int32_t *crowptr, int32_t *ccol, double *cval);
void orc_mg_restrict(int32_t dim, const int32_t *shape, const double *r, double *bc);
void orc_mg_prolong(int32_t dim, const int32_t *shape, double omega, const double *xc,
                    double *x);
/* Threads of the parallel build's loops (1 in the serial build). */
int orc_threads(void);

#endif
