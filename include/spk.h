/*
 * spk -- CSR sparse matrix-vector product and Jacobi-preconditioned conjugate
 * gradient for AMD MI355X (gfx950).  C ABI of libspk.so.
 *
 * The problem statement follows the paper (arXiv 2011.00715, Sec. 5.5
 * "OpenFOAM: An application perspective"): the application assembles a matrix
 * and vectors, hands them to the library, and the library solves A x = b with
 * a Krylov method that runs entirely on the GPU.  The API style follows Sec. 4:
 *  - plain pointers with an explicit memory type instead of pointer-attribute
 *    queries (Response A5 "Multiple memory types"; Challenge A5 notes the cost
 *    of such queries);
 *  - read-only inputs are `const`, outputs are write-only (the read/write
 *    accessor model of Response A4);
 *  - every call takes the caller's stream, so that the library and the
 *    application share one queue (Challenge / Response A6);
 *  - no call synchronises the device: the solve calls wait for their own
 *    stream, once per batch of iterations (Response A1); setup calls wait
 *    for the stream they were given; only the release of device memory in
 *    the *_destroy calls and when a handle re-plans (spk_mat_set_kernel)
 *    goes through hipFree, which HIP documents as waiting for the device.
 *
 * Conventions for every entry point:
 *  - `stream` is a hipStream_t passed as `void*`; NULL means the null stream.
 *  - Device pointers must be device memory of the current HIP device and must
 *    stay valid until the work queued on `stream` has finished.
 *  - Return value: SPK_OK (0) or a negative SPK_E* status.  Nothing aborts and
 *    nothing throws across the ABI.  spk_last_error() gives a thread-local
 *    message for the last failing call on the calling thread.
 *  - The caller owns every pointer it passes; the library never frees caller
 *    memory.  Handles own what they allocate and free it in *_destroy.
 *  - A handle may be used from one thread / one stream at a time.  It
 *    remembers the stream of its latest call; before moving a handle to
 *    another stream the caller orders the two streams (an event, or a
 *    synchronisation), as with any stream-ordered resource.
 */
#ifndef SPK_H
#define SPK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spk_mat spk_mat;
typedef struct spk_server spk_server;

/* memory types of caller buffers */
enum { SPK_MEM_HOST = 0, SPK_MEM_DEVICE = 1 };

/* solve precision (Challenge A7 / Response A7: per-solve precision flag).
 * Both mixed modes run FP32 inner CG on the FP32 values and keep the
 * residual r = b - A x, the update of x and the convergence test in FP64:
 *   SPK_PREC_MIXED     refinement by reliable updates: the FP32 search
 *                      direction is kept across refinements (CG continues
 *                      with the true residual), default trigger 0.05
 *   SPK_PREC_MIXED_IR  restarted iterative refinement: each refinement
 *                      solves A d = r / ||r|| from scratch to 1e-4 */
enum { SPK_PREC_FP64 = 0, SPK_PREC_MIXED = 1, SPK_PREC_MIXED_IR = 2 };

/* spk_mat_create_csr flags */
enum {
    SPK_MAT_MIXED = 1,     /* also keep an FP32 copy of the values (needed by
                              spk_mat_mult_f32 and mixed-precision solves) */
    SPK_MAT_VALIDATE = 2,  /* check the CSR on the device (monotone rowptr,
                              columns in range and strictly ascending) */
    SPK_MAT_BORROW = 4,    /* SPK_MEM_DEVICE only: keep the caller's rowptr,
                              col and values instead of copying them; the
                              caller keeps them alive and unchanged until
                              spk_mat_destroy */
    SPK_MAT_STREAM = 8     /* read the SELL layout with nontemporal loads
                              whatever its size.  Default: ordinary loads when
                              the layout (entries, slice offsets, row lengths
                              in the precision of the product) and the
                              vectors beside it fit the 256 MB Infinity Cache
                              -- 256 MiB with the 6 vectors of a Krylov
                              iteration, 288 MiB with x and y of a standalone
                              product -- so that it stays cached from one
                              product to the next; nontemporal loads above (a
                              matrix that cannot stay cached must not evict
                              the vectors).  Changes speed only: the results
                              are the same bits. */
};

/* SpMV kernel families (selected from row-length statistics at create) */
enum {
    SPK_KERNEL_AUTO = 0,
    SPK_KERNEL_STREAM = 1,  /* block-tile CSR stream: coalesced column/value
                               streams staged through LDS, short rows */
    SPK_KERNEL_VECTOR = 2,  /* L lanes per row (L = 64: one row per wavefront),
                               wavefront-shuffle reduction */
    SPK_KERNEL_MERGE = 3,   /* merge-path over rows + nonzeros, equal work per
                               tile, deterministic carry fix-up */
    SPK_KERNEL_SELL = 4,    /* sliced ELLPACK, 64-row slices (one per
                               wavefront), row-relative int16 column offsets
                               when they fit (10 instead of 12 bytes per FP64
                               nonzero); built from the CSR at selection */
    SPK_KERNEL_SLICED = 5,  /* column-sliced CSR for scattered columns: the
                               entries of each row split by which eighth of
                               [0, n) their column falls in; XCD s computes
                               the products of slice s (its eighth of x stays
                               in its own L2; a merge path over the stacked
                               slices, or lanes per slice row) into 8 partial
                               vectors that a second pass sums per row in
                               slice order.  A copy of the matrix built at
                               selection (12 nnz + 4 (8n + 1) bytes + 8n
                               partials) */
    SPK_KERNEL_SELL_SIGMA = 6  /* SELL-C-sigma (opt-in): SELL-64 over the rows
                                  ordered by length, longest first, within
                                  windows of sigma rows, so that the rows of a
                                  slice have similar lengths (less padding on
                                  skewed matrices); the layout carries the row
                                  permutation */
};

/* status codes */
enum {
    SPK_OK = 0,
    SPK_EINVAL = -1,     /* invalid argument or malformed CSR */
    SPK_ENOMEM = -2,     /* device or pinned host allocation failed */
    SPK_EHIP = -3,       /* a HIP runtime call failed (text in spk_last_error) */
    SPK_EZERODIAG = -4,  /* a row has no stored or a zero diagonal */
    SPK_EBUSY = -5,      /* server: request still in flight */
    SPK_EBUDGET = -6,    /* server: request can never fit the HBM budget */
    SPK_ENOTFOUND = -7   /* server: unknown or already collected ticket */
};

/* solver reasons (separate from the status: a solve that does not converge
 * returns SPK_OK with a negative reason) */
enum {
    SPK_CONVERGED_RTOL = 1,
    SPK_CONVERGED_ATOL = 2,
    SPK_RUNNING = 0,
    SPK_DIVERGED_ITS = -1,
    SPK_DIVERGED_INDEFINITE_MAT = -2,
    SPK_DIVERGED_INDEFINITE_PC = -3,
    SPK_DIVERGED_NANORINF = -4,
    SPK_DIVERGED_BREAKDOWN = -5,
    SPK_DIVERGED_STAGNATION = -6
};

typedef struct {
    int32_t n;
    int32_t kernel;          /* SPK_KERNEL_* in use */
    int64_t nnz;
    int32_t lanes;           /* VECTOR: lanes per row; STREAM: rows per tile;
                                MERGE: items per tile; SELL: column-offset
                                bits per entry (16 or 32), 0 with offsets
                                shared per slice */
    int32_t has_f32;         /* FP32 value copy present */
    int32_t row_min, row_max;
    int32_t row_p50, row_p99;  /* upper bounds from a log2 histogram */
    double row_mean, row_cv;
    int64_t bytes_spmv_f64;  /* algorithmic bytes of one FP64 SpMV:
                                12 nnz + 4 (n+1) + 16 n */
    int64_t bytes_spmv_f32;  /* FP32 values and vectors: 8 nnz + 4 (n+1) + 8 n */
    int64_t bytes_pcg_iter_f64;  /* one FP64 PCG iteration, algorithmic: the
                                    matrix once and 11 vector passes,
                                    12 nnz + 4 (n+1) + 88 n (the kernels move
                                    96 n: z is stored and read once) */
    int64_t bytes_pcg_iter_f32;  /* one FP32 inner iteration: 8 nnz + 4 (n+1) + 44 n */
    int64_t device_bytes;    /* device memory held by the handle */
    int32_t zero_diag_rows;  /* rows without a nonzero diagonal */
    int32_t cached_loads;    /* SELL layout read with ordinary (cache-allocating)
                                loads: bit 0 / 1 by the FP64 / FP32 Krylov and
                                smoother kernels, bit 2 / 3 by the FP64 / FP32
                                standalone products; otherwise nontemporal
                                (see SPK_MAT_STREAM); 0 for the other kernels */
    int64_t format_bytes_spmv_f64;  /* algorithmic bytes of one FP64 SpMV in the
                                       storage the selected kernel reads (equal
                                       to bytes_spmv_f64 except for SELL:
                                       (8 + w) padded_nnz + 4 slices + n + 16 n,
                                       w = 2 or 4 bytes per column offset;
                                       with shared offsets 8 padded_nnz +
                                       4 slices + 4 (offset-list entries) +
                                       4 n (masks) + 16 n) */
    int64_t format_bytes_spmv_f32;  /* same for FP32 values and vectors */
    int64_t stored_nnz;             /* entries the kernel reads, padding included */
    double gershgorin;              /* max_i sum_j |a_ij| / |a_ii|: a bound on the
                                       spectrum of D^-1 A (0 with a zero diagonal) */
    int32_t sell_sigma;             /* SPK_KERNEL_SELL_SIGMA: the window (rows) */
    int32_t pad_;
} spk_mat_info;

/*
 * Create a matrix from CSR arrays (the MATAIJ format of Sec. 4; 32-bit column
 * indices and FP64 values, the byte count of Challenge A7).
 *   n       rows = columns, 0 <= n < 2^31
 *   nnz     stored entries, 0 <= nnz < 2^31
 *   rowptr  int32[n+1], rowptr[0] = 0, non-decreasing, rowptr[n] = nnz
 *   colind  int32[nnz], 0 <= col < n; ascending within a row is required only
 *           with SPK_MAT_VALIDATE (the products do not depend on it)
 *   values  double[nnz]
 *   memtype SPK_MEM_HOST (copied through pinned staging) or SPK_MEM_DEVICE
 *   flags   SPK_MAT_* bits
 * The structure is always checked on the device before any other kernel
 * reads it (rowptr[0] = 0, non-decreasing, rowptr[n] = nnz, 0 <= col < n):
 * SPK_EINVAL with a message.  Rows without a nonzero diagonal are counted
 * (spk_mat_info.zero_diag_rows); the Jacobi preconditioner (Sec. 5.3, the
 * Jacobi smoother) needs 1/a_ii, so spk_pc_jacobi_apply and spk_ksp_solve
 * return SPK_EZERODIAG for such a matrix, while SpMV works on any matrix.
 * Work is queued on `stream`; the call returns after the setup has finished
 * (it reads a few bytes of row statistics back to choose the kernel).
 */
int spk_mat_create_csr(int32_t n, int64_t nnz, const int32_t *rowptr,
                       const int32_t *colind, const double *values, int memtype,
                       uint32_t flags, void *stream, spk_mat **out);

/* Force an SpMV kernel family (testing and A/B runs).  param: lanes per row
 * for VECTOR (1..64, power of two), rows per tile for STREAM (0 = automatic),
 * column offsets for SELL: 16 or 32 (bits per entry, one offset per lane;
 * SPK_EINVAL when the offsets do not fit or a row exceeds 65535 entries; row
 * lengths above 255 are stored in 16 bits), 1 (shared: each 64-row slice
 * stores its sorted list of distinct offsets once and each row a 32-bit mask
 * of the list positions it uses, the other positions holding zeros that are
 * never multiplied; SPK_EINVAL unless every row has strictly increasing
 * columns, every slice's rows use at most 32 distinct offsets and the
 * stored entries grow by at most 1/16) or 0 (automatic: shared when the
 * matrix qualifies, which stencils do, else 16 when the offsets fit, else
 * 32; deciding reads the column indices back to host memory once, 4 nnz
 * bytes, when no row exceeds 32 entries), the window sigma for SELL_SIGMA
 * (a multiple of 64; 0 = 4096; offsets per lane, 16 bits when they fit,
 * else 32), for SLICED 0
 * (automatic: the merge path over the slices when 8n + nnz < 2^31, else
 * lanes per slice row), a power of two in 1..64 (lanes per slice row) or
 * 2048 (merge path over the slices), ignored for MERGE.
 * Waits for the handle's earlier work (the stream of its latest call), then
 * builds the layout the family needs on `stream` and returns once it is
 * built (it synchronises `stream` only).  Invalidates cached solver graphs
 * and releases the solver workspaces, which the next solve re-creates. */
int spk_mat_set_kernel(spk_mat *A, int kernel, int32_t param, void *stream);

/* y = A x (Sec. 4: MatMult on an AIJ matrix).  x, y: device double[n],
 * must not overlap.  Queued on `stream`; no synchronisation. */
int spk_mat_mult(const spk_mat *A, const double *x, double *y, void *stream);

/* y = A32 x with FP32 values, FP32 x and y and FP32 accumulation (Challenge
 * A7: 64 instead of 96 bits per nonzero).  Needs SPK_MAT_MIXED. */
int spk_mat_mult_f32(const spk_mat *A, const float *x, float *y, void *stream);

int spk_mat_get_info(const spk_mat *A, spk_mat_info *info);

/* Jacobi preconditioner apply, z_i = r_i / a_ii (PCApply of the Jacobi
 * smoother, Sec. 5.3).  Device double[n]. */
int spk_pc_jacobi_apply(const spk_mat *A, const double *r, double *z, void *stream);

/*
 * Jacobi-preconditioned Chebyshev smoother (Sec. 5.3: the geometric multigrid
 * of the driven-cavity study smooths every level but the coarsest with it).
 * `steps` steps of Chebyshev acceleration on D^-1 A x = D^-1 b over the
 * spectral interval [emin, emax] of D^-1 A, D = diag(A):
 *   theta = (emax + emin)/2, delta = (emax - emin)/2, sigma = theta/delta
 *   r = b - A x (x = 0 unless x0_nonzero), d = D^-1 r / theta, rho = 1/sigma
 *   steps times: x += d; r -= A d; rho' = 1/(2 sigma - rho);
 *                d = rho' rho d + (2 rho'/delta) D^-1 r; rho = rho'
 * The coefficients are known in advance, so a step is one fused SpMV + update
 * pass with no inner product and no host round trip (the error after k steps
 * is T_k((theta - t)/delta) / T_k(sigma) on each eigencomponent t).
 *   b      device double[n], read only
 *   x      device double[n]: x0 in when x0_nonzero (else overwritten), result out
 *   r_out  optional device double[n] receiving the recursive residual
 *          b - A x_steps; with r_out NULL the last step skips its SpMV
 *   emax <= 0 takes the Gershgorin bound of D^-1 A (spk_mat_info.gershgorin);
 *   emin <= 0 takes emax / 10 (the smoother damps the upper 90 % of the
 *   interval)
 * Uses the handle's solver workspace (allocated on first use).  Errors:
 * SPK_EINVAL (NULL pointer, steps < 0, not 0 < emin < emax after the
 * defaults, b or r_out overlapping x), SPK_EZERODIAG.  Queued on `stream`.
 */
int spk_pc_chebyshev(const spk_mat *A, const double *b, double *x, double *r_out,
                     int32_t steps, double emin, double emax, int32_t x0_nonzero,
                     void *stream);

/* Waits for the handle's queued work (the stream of its latest call), then
 * frees everything it owns. */
int spk_mat_destroy(spk_mat *A);

/* ---------------------------------------------------------------- vectors
 * The Krylov vector kernels (Sec. 5.1: VecAXPY, 2 flops and 3 memory
 * accesses per entry; Sec. 4 Response F3: fused multiple inner products).
 * All are device double arrays of length n, queued on `stream`.  Reductions
 * write their result to device memory (`result`, 1 or 2 doubles) so that no
 * host synchronisation is needed; they are deterministic (fixed reduction
 * tree, no floating-point atomics). */
int spk_vec_axpy(int32_t n, double alpha, const double *x, double *y, void *stream);   /* y = a x + y */
int spk_vec_aypx(int32_t n, double beta, const double *x, double *y, void *stream);    /* y = x + b y */
int spk_vec_dot(int32_t n, const double *x, const double *y, double *result, void *stream);
int spk_vec_dot2(int32_t n, const double *x, const double *y, const double *w,
                 double *result, void *stream); /* result[0] = x.y, result[1] = x.w, one pass */
int spk_vec_nrm2(int32_t n, const double *x, double *result, void *stream);

/* spk_vec_dot2 without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Same arguments, kernels and result bits as
 * spk_vec_dot2; it calls no hipMalloc/hipFree or allocating routine.  Its
 * per-block partial sums live in a fixed array of 2 x 2048 doubles (32 KiB)
 * compiled into the library, one copy per GPU, held until the process ends;
 * a launch never has more than 2048 blocks, so every n >= 0 fits (a grid
 * beyond it would be refused with SPK_EINVAL).  Every call on one GPU shares
 * that GPU's array and leaves its partials in it: calls that overlap on one
 * GPU (different streams, or threads without ordering) race and may return
 * wrong sums; order them on one stream.  Devices 0..63. */
int spk_vec_dot2_noalloc(int32_t n, const double *x, const double *y, const double *w,
                         double *result, void *stream);

/* ---------------------------------------------------------------- solver */
typedef struct {
    double rtol;          /* default 1e-8 */
    double atol;          /* default 0 */
    int32_t maxit;        /* default 10000 (FP64 iterations, or inner
                             iterations in total for mixed) */
    int32_t precision;    /* SPK_PREC_FP64 (default) or SPK_PREC_MIXED */
    int32_t x0_nonzero;   /* 0: start from x = 0 (default); 1: from x */
    int32_t graph_k;      /* iterations per captured graph (default 8) */
    double inner_rtol;    /* mixed: refine once the FP32 residual fell by this
                             factor since the last refinement; 0 (default)
                             selects 0.05 for MIXED and 1e-4 for MIXED_IR */
    int32_t inner_maxit;  /* mixed: per inner solve (default 10000) */
    int32_t max_outer;    /* mixed: refinement steps (default 100) */
    double *hist;         /* optional host double[hist_len]: ||r_k||_2 of the
                             recursive residual, k = 0..iterations */
    int32_t hist_len;
    int32_t single_reduction;  /* FP64 only: 1 selects the single-reduction
                                  (Chronopoulos-Gear) recurrences, two kernels
                                  per iteration instead of three (default 0) */
    int32_t profile;      /* 1: time the SpMV product of every iteration (FP64,
                             or FP32 inner for mixed) with a HIP event pair on
                             `stream` (around the product kernel; the
                             one-wavefront-per-slice SELL product's one-block
                             fold of its partials is outside the pair);
                             kernels are then launched one iteration at a
                             time without graphs.  Results in
                             spk_ksp_result.product_*.  Not with
                             single_reduction (default 0) */
} spk_ksp_opts;

void spk_ksp_opts_default(spk_ksp_opts *o);

typedef struct {
    int32_t reason;            /* SPK_CONVERGED_* or SPK_DIVERGED_* */
    int32_t iterations;        /* FP64 iterations (all, incl. fallback) */
    int32_t inner_iterations;  /* mixed: FP32 inner iterations in total */
    int32_t outer_steps;       /* mixed: refinement steps */
    int32_t restarts;          /* true-residual restarts */
    int32_t fallback_fp64;     /* mixed: finished in FP64 after stagnation */
    double rnorm0, rnorm, bnorm;
    double true_rel_residual;  /* ||b - A x|| / ||b|| from a fresh FP64 SpMV */
    double seconds;            /* host wall time of the call */
    double product_ms;         /* opts.profile: summed event time of the
                                  product launches of the counted iterations
                                  (launches after the solve stopped excluded) */
    int32_t product_launches;  /* opts.profile: the launches product_ms covers */
    int32_t pad_;
} spk_ksp_result;

/*
 * Solve A x = b with Jacobi-preconditioned CG (Sec. 5.5 uses CG; Sec. 5.3
 * the Jacobi smoother).  b: device double[n], read only.  x: device
 * double[n], initial guess if opts->x0_nonzero, solution on return.
 * Convergence: ||r_k||_2 <= max(rtol ||b||_2, atol) on the recursive
 * residual, confirmed by the true residual (restart from it, at most 3
 * times, else BREAKDOWN).  MIXED runs FP32 inner CG on the FP32 values with
 * FP64 iterative refinement (residual, update and test in FP64).
 * Queued on `stream`; returns when the result is known (waits for the
 * stream about once per graph_k iterations, with two batches in flight).
 * opts may be NULL (defaults).  res must not be NULL.
 */
int spk_ksp_solve(spk_mat *A, const double *b, double *x, const spk_ksp_opts *opts,
                  spk_ksp_result *res, void *stream);

/*
 * Multiple right-hand sides (Sec. 4 Response F3: Krylov methods with several
 * right-hand sides read the matrix once for all of them and fuse the outer
 * loops of their solves).  Blocks of k vectors are row-major n x k device
 * double arrays: entry (i, j) at [i * k + j].  k must be 1, 2, 4, 8 or 16.
 */

/* Y = A X for k columns.  X, Y must not overlap.  SPK_EINVAL for a bad k or
 * NULL.  Queued on `stream`. */
int spk_mat_mult_multi(const spk_mat *A, int32_t k, const double *X, double *Y, void *stream);

/* k independent FP64 Jacobi-PCG solves A x_j = b_j sharing every SpMM: each
 * column keeps its own scalars, stopping test, true-residual restarts and
 * result, exactly as spk_ksp_solve on that column (hist is not recorded).
 * B: device n x k, read only; X: device n x k, initial guesses when
 * opts->x0_nonzero, solutions on return.  res: host spk_ksp_result[k].
 * SPK_EINVAL for a bad k, a mixed precision, NULL or overlapping B and X;
 * SPK_EZERODIAG.  The workspace (6 n k doubles) is kept on the handle for
 * the next call with the same k.  Returns when every column is done. */
int spk_ksp_solve_multi(spk_mat *A, int32_t k, const double *B, double *X,
                        const spk_ksp_opts *opts, spk_ksp_result *res, void *stream);

/* ---------------------------------------------------------------- multigrid
 * Geometric multigrid on a logically structured grid, as the preconditioner
 * of CG (Sec. 5.3: the driven-cavity study runs multigrid with
 * Jacobi-preconditioned Chebyshev smoothers on every level but the coarsest,
 * which is solved directly, in V- and W-cycles).  The paper fixes neither the
 * grid transfers nor the coarse operators; this library takes aggregation:
 *  - rows are grid points numbered with the first dimension fastest; a grid
 *    of extents (s_0, s_1, s_2) coarsens to ceil(s_d / 2), fine point
 *    (i_0, i_1, i_2) belonging to coarse point (i_0/2, i_1/2, i_2/2);
 *  - prolongation P is piecewise constant over these aggregates, restriction
 *    is P^T, and the coarse matrix is the Galerkin product P^T A P, formed on
 *    the device (the matrix may only couple points at most one grid step
 *    apart in each direction: 3/5/7/9/27-point stencils);
 *  - levels are added while the coarsest has more than coarse_max rows; the
 *    coarsest (at most 4096 rows) is inverted densely at setup and solved by
 *    one matrix-vector product.
 * One cycle on level l for b_l from x_l (zero unless stated):
 *   smooth_steps Chebyshev steps (spk_pc_chebyshev's recurrence on
 *   [emin_frac g_l, g_l], g_l the Gershgorin bound of D^-1 A_l);
 *   b_{l+1} = P^T (b_l - A_l x_l); x_{l+1} = cycle on level l+1 (a W-cycle
 *   runs it twice, the second from the first's result, except on the
 *   directly solved level); x_l += omega P x_{l+1}; smooth_steps Chebyshev
 *   steps from x_l.
 * The cycle is symmetric positive definite for every omega > 0, so CG may
 * use it; omega = 2 offsets the factor 2 by which piecewise-constant
 * prolongation underestimates the coarse correction of smooth errors.
 */
typedef struct spk_mg spk_mg;

typedef struct {
    int32_t max_levels;    /* levels including the finest, 1..16 (default 16) */
    int32_t coarse_max;    /* coarsen while a level has more rows, 1..4096 (default 1000) */
    int32_t smooth_steps;  /* Chebyshev steps before and after the coarse correction, 0..64 (default 2) */
    int32_t cycle;         /* 1: V-cycle (default), 2: W-cycle */
    double emin_frac;      /* smoother interval [emin_frac g, g], in (0, 1) (default 0.1) */
    double omega;          /* coarse-grid correction x += omega P x_c, > 0 (default 2.0) */
    int32_t precision;     /* SPK_PREC_FP64 (default), or SPK_PREC_MIXED: the cycle in FP32
                              (values, vectors, arithmetic; FP32 copies of every level's
                              values are made, the caller's matrix included) inside FP64 CG */
    int32_t pad_;
} spk_mg_opts;

void spk_mg_opts_default(spk_mg_opts *o);

typedef struct {
    int32_t levels;
    int32_t pad_;
    int32_t n[16];          /* rows per level (0: finest) */
    int64_t nnz[16];
    int32_t shape[16][3];   /* grid extents per level (unused dimensions 1) */
    int32_t kernel[16];     /* SPK_KERNEL_* of each level's SpMV */
    double emax[16];        /* smoother interval [emin_frac emax, emax] per level */
    int64_t device_bytes;   /* library-owned device memory of the hierarchy */
} spk_mg_info;

/* Builds the hierarchy for A on a grid of `dim` (1..3) extents shape[0..dim-1]
 * whose product is A's row count.  A stays the caller's: it must outlive the
 * hierarchy and keep its values.  opts NULL takes the defaults.  Errors:
 * SPK_EINVAL (bad grid or options, a coupling beyond one grid step, a
 * coarsest level above 4096 rows, a coarsest matrix that is not positive
 * definite), SPK_EZERODIAG, SPK_ENOMEM / SPK_EHIP.  Synchronises `stream`. */
int spk_mg_create(const spk_mat *A, int32_t dim, const int32_t *shape, const spk_mg_opts *opts,
                  void *stream, spk_mg **out);
int spk_mg_get_info(const spk_mg *M, spk_mg_info *info);
/* Host copies of level `level`'s CSR arrays (n + 1, nnz and nnz entries from
 * spk_mg_get_info); synchronises the device. */
int spk_mg_copy_level(const spk_mg *M, int32_t level, int32_t *rowptr, int32_t *col, double *val);
/* x = one cycle from zero for right-hand side b (device double[n], not
 * overlapping).  Queued on `stream`; uses the hierarchy's vectors, so calls
 * on one hierarchy must not overlap. */
int spk_mg_apply(spk_mg *M, const double *b, double *x, void *stream);
/* The same cycle `reps` times with events around each level's own kernels:
 * level_ms[l] (host double[levels]) receives the mean milliseconds per cycle
 * spent on level l (the per-level breakdown of the driven-cavity study).
 * Synchronises `stream`. */
int spk_mg_profile(spk_mg *M, const double *b, double *x, int32_t reps, double *level_ms, void *stream);
/* CG preconditioned by one cycle per iteration, FP64, with the stopping
 * rules, breakdown reasons, true-residual restarts and history of
 * spk_ksp_solve (precision must be SPK_PREC_FP64 and single_reduction 0).
 * graph_k iterations are captured per graph (0: no graph).  b, x: device
 * double[n] as in spk_ksp_solve.  Returns when the result is known. */
int spk_ksp_solve_mg(spk_mg *M, const double *b, double *x, const spk_ksp_opts *opts,
                     spk_ksp_result *res, void *stream);
int spk_mg_destroy(spk_mg *M);

/* ---------------------------------------------------------------- server
 * Continuous-batching solve server (Response A6: many different-size
 * problems solved simultaneously on the GPU).  Requests are admitted while
 * slots and the HBM budget allow; all active systems advance together in
 * batched kernels (one launch serves every system, per-system reductions),
 * so a system's result does not depend on what else is in the batch. */
typedef struct {
    int64_t hbm_budget_bytes;  /* device arena size (default 8 GiB) */
    int32_t max_slots;         /* concurrent systems (default 64) */
    int32_t graph_k;           /* iterations per batched step (default 8) */
    int32_t max_blocks_per_system;  /* blocks of one system in a batched launch
                                       (default 2048: a large system streams
                                       at full bandwidth; at most 8192) */
    int32_t pad_;
    int64_t pinned_bytes;      /* pinned host pool for submitted systems
                                  (default 1 GiB; 0 = pageable staging only) */
} spk_server_opts;

void spk_server_opts_default(spk_server_opts *o);

int spk_server_create(const spk_server_opts *o, void *stream, spk_server **out);

/* Submit A x = b from host CSR (copied before return).  opts may be NULL.
 * ticket: out, identifies the request.  SPK_EBUDGET if it can never fit.
 * Thread safety (the exception to the one-thread-per-handle rule): the
 * server calls serialise on a lock inside the server, and submit validates
 * and copies the system outside it, so client threads may submit while one
 * service thread calls spk_server_progress / completed / poll; the copy of
 * a large system (tens of MB) then does not hold back the batched steps. */
int spk_server_submit(spk_server *s, int32_t n, int64_t nnz, const int32_t *rowptr,
                      const int32_t *colind, const double *values, const double *b,
                      const spk_ksp_opts *opts, uint64_t *ticket);

/* Admit queued requests, run up to max_steps batched steps, retire finished
 * systems.  Returns the number of active + queued requests (>= 0) or a
 * status. */
int spk_server_progress(spk_server *s, int32_t max_steps);

/* Collect a finished request: copies x (host double[n]) and the result.
 * SPK_EBUSY while in flight; the ticket is released on success.
 * done_time (may be NULL): host monotonic time of retirement, seconds. */
int spk_server_poll(spk_server *s, uint64_t ticket, double *x_host, spk_ksp_result *res,
                    double *done_time);

/* Completion queue: copies up to cap tickets of requests that finished since
 * the last call (in completion order) and returns how many (>= 0), so a
 * client polls only those.  Each ticket is reported once; spk_server_poll
 * still collects it. */
int spk_server_completed(spk_server *s, uint64_t *tickets, int32_t cap);

int spk_server_destroy(spk_server *s);

/* ---------------------------------------------------------------- misc */
const char *spk_status_str(int status);
const char *spk_reason_str(int reason);
const char *spk_last_error(void);
/* host monotonic clock, seconds (same clock as done_time) */
double spk_now(void);
/* HIP runtime version the library is running on */
int spk_runtime_version(void);

/* Measurement helpers (Sec. 5.1: work-time spectrum of vector copies):
 * stream-copy n doubles from src to dst, and read `bytes` of scratch to
 * evict the Infinity Cache before a cold measurement (the cache then holds
 * clean scratch lines: the next kernel reads from HBM and writes back
 * nothing for the eviction).  scratch is device memory of at least `bytes`
 * bytes; its contents are left unchanged. */
int spk_bw_copy(int64_t n, const double *src, double *dst, void *stream);
int spk_cache_flush(void *scratch, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
