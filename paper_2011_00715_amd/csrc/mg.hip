// Geometric multigrid: hierarchy setup on the device (Galerkin coarse
// operators, dense inverse of the coarsest level), the V/W cycle, and CG
// preconditioned by one cycle per iteration with captured iteration graphs
// (Sec. 5.3: the driven-cavity study's multigrid with Chebyshev-Jacobi
// smoothers; Sec. 4 Response A1: keep the stream queue full).
#include <string.h>

#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include <algorithm>

#include "mg.hpp"
#include "runtime.hpp"

namespace spk {

struct MgLevel {
    spk_mat *A = nullptr;  // level 0: the caller's matrix (not owned)
    Grid3 g{1, 1, 1};
    int n = 0;
    double emax = 0.0, emin = 0.0;
    // vectors of the cycle's precision (double, or float for the FP32 cycle);
    // level 0's b and x are the call's own arrays in an FP64 cycle
    void *b = nullptr, *x = nullptr;
    void *r = nullptr, *d0 = nullptr, *d1 = nullptr, *tmp = nullptr;
    void *x2 = nullptr;  // second x buffer of the levels between the finest and the coarsest
    // where the level's x currently lives, and a last smoothing step d left
    // for the parent to add (set while a cycle is enqueued)
    void *xcur = nullptr;
    const void *dpend = nullptr;
};

// Level 0's connection to the FP64 data of a call: the cycle's right-hand
// side, where its result goes, and (inside CG) the partial sums of r . z.
struct CycleIo {
    const double *b64;
    double *z64;
    double *dotpart;  // null: no inner product
    int *np;
    const double *rcg;
};

// Events of a profiled cycle: (level, start, end) for each stretch of one
// level's own kernels.
struct MgTimer {
    std::vector<int> level;
    std::vector<hipEvent_t> ev;
};

}  // namespace spk

struct spk_mg {
    int device = 0;
    int dim = 0;
    spk_mg_opts o{};
    int nlev = 0;
    spk::MgLevel lev[spk::kMgMaxLevels];
    int f32 = 0;             // 1: the cycle runs in FP32 (values, vectors, arithmetic)
    void *cinv = nullptr;    // dense inverse of the coarsest matrix, row-major, cycle precision
    // solve workspace (allocated on first solve)
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *x = nullptr, *b = nullptr;
    double *tmp64 = nullptr; // FP64 SpMV output of the unfused families
    double *part = nullptr;  // 4 x kMgMaxPart partial sums
    double *hist = nullptr;
    int hist_cap = 0;
    spk::SysState *st = nullptr, *pst = nullptr;
    int32_t *pstatus = nullptr;
    hipEvent_t ev[4] = {};
    hipStream_t cap = nullptr;
    hipGraphExec_t g = nullptr;
    int gk = 0;
    int g_kernel = -1;      // level-0 SpMV family the graph was captured with
    const void *g_sell = nullptr;
    spk::MgTimer *timer = nullptr;  // set while a profiled cycle is enqueued
    int64_t bytes = 0;
    hipStream_t stream = nullptr;   // stream of the latest call that queued work
};

namespace spk {

#define SPK_TRY(x)                     \
    do {                               \
        const int rc_ = (x);           \
        if (rc_ != SPK_OK) return rc_; \
    } while (0)

enum { kPartRzMg = 0, kPartPqMg = 1, kPartRrMg = 2, kPartBbMg = 3 };

// Levels up to this many rows fold the prolongation into the post-smoother's
// residual pass (a CSR pass that forms x + omega P x_c for every gathered
// column); larger ones keep the two passes, whose SpMV uses the level's own
// family (on 64^3 the folded CSR pass took 14.8 us against 4.9 + 3.5 us).
constexpr int kMgFuseRows = 65536;

static int grid_n(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxBlocksSingle) g = kMaxBlocksSingle;
    return (int)(g < 1 ? 1 : g);
}

template <class T>
static int mg_alloc(spk_mg *M, T **p, int64_t count)
{
    const size_t b = sizeof(T) * (size_t)(count > 0 ? count : 1);
    SPK_HIP(hipMalloc((void **)p, b));
    M->bytes += (int64_t)b;
    return SPK_OK;
}

// A cycle vector of n entries (8 or 4 bytes each).
static int mg_vec(spk_mg *M, void **p, int64_t n)
{
    const size_t b = (M->f32 ? 4 : 8) * (size_t)(n > 0 ? n : 1);
    SPK_HIP(hipMalloc(p, b));
    M->bytes += (int64_t)b;
    return SPK_OK;
}

template <class V>
static const V *values_of(const spk_mat *A)
{
    return std::is_same<V, double>::value ? (const V *)A->val : (const V *)A->val32;
}

template <class V>
static const V *dinv_of(const spk_mat *A)
{
    return std::is_same<V, double>::value ? (const V *)A->dinv : (const V *)A->dinv32;
}

static double *part_of(spk_mg *M, int slot) { return M->part + (size_t)slot * kMgMaxPart; }

// One pass over the rows of A with y = A x handed to the epilogue f; the
// number of partial sums written to `part` (if not null) goes to *np.
template <class V, class F>
static int launch_rows(spk_mat *A, const V *x, F f, double *part, int *np, const SysState *gate, V *tmp,
                       hipStream_t s)
{
    constexpr bool f64 = std::is_same<V, double>::value;
    const int n = A->n;
    if (A->kernel == SPK_KERNEL_SELL) {
        const SellView sv{A->sell_ptr, A->sell_col, A->sell_len, A->sell_plain, A->sell_len16, A->sell_perm, A->sell_mask};
        const int grid = std::max(1, std::min(ceil_div(ceil_div(n, kSell), kBlock / kWave), kMgMaxPart));
        const V *sval = f64 ? (const V *)A->sell_val : (const V *)A->sell_val32;
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2)
                hipLaunchKernelGGL((k_mg_rows_sell<V, int16_t, U, F>), dim3(grid), dim3(kBlock), 0, s, n, sv, sval, x,
                                   f, part, gate);
            else
                hipLaunchKernelGGL((k_mg_rows_sell<V, int32_t, U, F>), dim3(grid), dim3(kBlock), 0, s, n, sv, sval, x,
                                   f, part, gate);
        });
        if (np) *np = grid;
    } else if (A->kernel == SPK_KERNEL_STREAM) {
        hipLaunchKernelGGL((k_mg_rows_stream<V, F>), dim3(A->nblk), dim3(kBlock), 0, s, n, A->R, A->ntiles, A->nblk,
                           A->rowptr, A->col, values_of<V>(A), x, f, part, gate);
        if (np) *np = A->nblk;
    } else {
        SPK_TRY(launch_spmv<V>(A, values_of<V>(A), x, tmp, s, gate, gate ? kGateInner64 : kGateNone));
        const int grid = grid_n(n);
        hipLaunchKernelGGL((k_mg_rows_y<V, F>), dim3(grid), dim3(kBlock), 0, s, n, (const V *)tmp, f, part, gate);
        if (np) *np = grid;
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int timer_mark(spk_mg *M, int level, hipStream_t s)
{
    if (!M->timer) return SPK_OK;
    hipEvent_t e;
    SPK_HIP(hipEventCreate(&e));
    M->timer->level.push_back(level);
    M->timer->ev.push_back(e);
    SPK_HIP(hipEventRecord(e, s));
    return SPK_OK;
}

// Level 0's result z = x + d (d null: z = x) in FP64, with the r . z partial
// sums when the call wants them.
template <class V>
static void finish(spk_mg *M, const V *d, const SysState *gate, const CycleIo *io, hipStream_t s)
{
    const MgLevel &L = M->lev[0];
    const int g = grid_n(L.n);
    hipLaunchKernelGGL((k_mg_finish<V>), dim3(g), dim3(kBlock), 0, s, L.n, d, (const V *)L.x, io->z64, io->rcg,
                       io->dotpart, gate);
    if (io->np) *io->np = g;
}

// Chebyshev steps on level l after the smoother's start (r, d_0 and the
// level's current x set).  keep_r: the last step also updates r (its result
// is restricted).  Otherwise the last step only adds d to x: on level 0 it
// is finish() (z = x + d in FP64, with the CG partial sums), on a coarser
// level with defer_last it is left to the parent's prolongation (L.dpend).
template <class V>
static int cheb_steps(spk_mg *M, int l, bool keep_r, bool defer_last, const CycleIo *io, const SysState *gate,
                      hipStream_t s)
{
    MgLevel &L = M->lev[l];
    spk_mat *A = L.A;
    const int n = L.n, steps = M->o.smooth_steps;
    const double theta = 0.5 * (L.emax + L.emin), delta = 0.5 * (L.emax - L.emin), sigma = theta / delta;
    V *x = (V *)L.xcur, *r = (V *)L.r, *tmp = (V *)L.tmp;
    V *d[2] = {(V *)L.d0, (V *)L.d1};
    const dim3 gn(grid_n(n)), tb(kBlock);
    L.dpend = nullptr;
    if (steps == 0) {
        if (!keep_r && l == 0) finish<V>(M, (const V *)nullptr, gate, io, s);
        SPK_HIP(hipGetLastError());
        return SPK_OK;
    }
    double rho = 1.0 / sigma;
    for (int k = 0; k < steps; ++k) {
        const bool last = k == steps - 1;
        if (last && !keep_r) {
            if (l == 0) finish<V>(M, (const V *)d[k & 1], gate, io, s);
            else if (defer_last) L.dpend = d[k & 1];
            else hipLaunchKernelGGL((k_cheb_last<V>), gn, tb, 0, s, n, (const V *)d[k & 1], x, gate);
            break;
        }
        const double rho_next = 1.0 / (2.0 * sigma - rho);
        ChebStep<V> c;
        c.dk = d[k & 1];
        c.dn = last ? nullptr : d[(k + 1) & 1];
        c.r = r;
        c.x = x;
        c.dinv = dinv_of<V>(A);
        c.c1 = (V)(rho_next * rho);
        c.c2 = (V)(2.0 * rho_next / delta);
        c.gate = gate;
        SPK_TRY(cheb_step<V>(A, c, tmp, s));
        rho = rho_next;
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// Smoother start on level l: from zero (x = 0, r = b, d_0 = D^-1 b / theta;
// on level 0 b comes from the call's FP64 right-hand side, which an FP32
// cycle keeps rounded in L.b), or from the level's current x.
template <class V>
static int smoother_start(spk_mg *M, int l, bool x0_nonzero, const CycleIo *io, const SysState *gate,
                          hipStream_t s)
{
    constexpr bool f32 = std::is_same<V, float>::value;
    MgLevel &L = M->lev[l];
    spk_mat *A = L.A;
    const int n = L.n;
    const V inv_theta = (V)(1.0 / (0.5 * (L.emax + L.emin)));
    V *b = (V *)L.b, *x = (V *)L.xcur, *r = (V *)L.r, *d0 = (V *)L.d0;
    const V *dinv = dinv_of<V>(A);
    const dim3 gn(grid_n(n)), tb(kBlock);
    if (x0_nonzero)
        SPK_TRY(launch_rows<V>(A, x, RowResid<V>{b, r, d0, dinv, inv_theta}, nullptr, nullptr, gate, (V *)L.tmp, s));
    else if (f32 && l == 0)  // the FP64 right-hand side, rounded and kept
        hipLaunchKernelGGL((k_cheb_init<V, double>), gn, tb, 0, s, n, io->b64, (const V *)nullptr, x, r, d0, dinv,
                           inv_theta, gate, b);
    else
        hipLaunchKernelGGL((k_cheb_init<V, V>), gn, tb, 0, s, n, (const V *)b, (const V *)nullptr, x, r, d0, dinv,
                           inv_theta, gate, (V *)nullptr);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

template <class V, int Lanes>
static void launch_resid_prolong(spk_mg *M, int l, const SysState *gate, hipStream_t s)
{
    MgLevel &L = M->lev[l];
    const MgLevel &C = M->lev[l + 1];
    spk_mat *A = L.A;
    V *xout = (V *)(L.xcur == L.x ? L.x2 : L.x);
    // one lane group per row: the pass is a few dependent gathers deep, so
    // rows are not looped over (a grid-stride loop made 64^3 three times slower)
    const int grid = std::max(1, std::min(ceil_div(L.n, kBlock / Lanes), kMgMaxPart));
    hipLaunchKernelGGL((k_mg_resid_prolong<V, Lanes>), dim3(grid), dim3(kBlock), 0, s, L.n,
                       (const int32_t *)A->rowptr, (const int32_t *)A->col, values_of<V>(A), dinv_of<V>(A),
                       (const V *)L.b, (const V *)L.xcur, (const V *)C.xcur, (const V *)C.dpend, (V)M->o.omega, L.g,
                       C.g, xout, (V *)L.r, (V *)L.d0, (V)(1.0 / (0.5 * (L.emax + L.emin))), gate);
    L.xcur = xout;
}

// One cycle on level l: x_l from b_l, or from x_l when x0_nonzero.
// pre_inited: the parent already formed this level's start from zero
// together with the restriction.  defer_last: leave the last smoothing
// step's x += d to the parent's prolongation.  io is set on level 0 only.
template <class V>
static int enqueue_cycle(spk_mg *M, int l, bool x0_nonzero, bool pre_inited, bool defer_last,
                         const SysState *gate, hipStream_t s, const CycleIo *io)
{
    constexpr bool f32 = std::is_same<V, float>::value;
    MgLevel &L = M->lev[l];
    if (l == M->nlev - 1) {  // direct solve (x0 does not matter)
        SPK_TRY(timer_mark(M, l, s));
        if (f32 && l == 0)
            hipLaunchKernelGGL(k_mg_round, dim3(grid_n(L.n)), dim3(kBlock), 0, s, L.n, io->b64, (float *)L.b, gate);
        hipLaunchKernelGGL((k_mg_gemv<V>), dim3(ceil_div(L.n, kBlock / kWave)), dim3(kBlock), 0, s, L.n,
                           (const V *)M->cinv, (const V *)L.b, (V *)L.x, gate);
        L.xcur = L.x;
        L.dpend = nullptr;
        if (l == 0) finish<V>(M, (const V *)nullptr, gate, io, s);
        SPK_HIP(hipGetLastError());
        SPK_TRY(timer_mark(M, l, s));
        return SPK_OK;
    }
    MgLevel &C = M->lev[l + 1];
    const bool c_direct = l + 1 == M->nlev - 1;
    SPK_TRY(timer_mark(M, l, s));
    if (!pre_inited) {
        if (!x0_nonzero) L.xcur = L.x;
        SPK_TRY(smoother_start<V>(M, l, x0_nonzero, io, gate, s));
    }
    SPK_TRY(cheb_steps<V>(M, l, true, false, io, gate, s));
    if (c_direct) {
        hipLaunchKernelGGL((k_mg_restrict<V>), dim3(grid_n(C.n)), dim3(kBlock), 0, s, L.g, C.g, (const V *)L.r,
                           (V *)C.b, gate);
    } else {  // restriction and the coarse level's start from zero in one pass
        C.xcur = C.x;
        hipLaunchKernelGGL((k_mg_init_restrict<V>), dim3(grid_n(C.n)), dim3(kBlock), 0, s, L.g, C.g,
                           (const V *)L.r, (V *)C.b, (V *)C.x, (V *)C.r, (V *)C.d0, dinv_of<V>(C.A),
                           (V)(1.0 / (0.5 * (C.emax + C.emin))), gate);
    }
    SPK_HIP(hipGetLastError());
    SPK_TRY(timer_mark(M, l, s));
    const bool twice = M->o.cycle == 2 && !c_direct;
    SPK_TRY(enqueue_cycle<V>(M, l + 1, false, !c_direct, !twice, gate, s, nullptr));
    if (twice) SPK_TRY(enqueue_cycle<V>(M, l + 1, true, false, true, gate, s, nullptr));
    SPK_TRY(timer_mark(M, l, s));
    if (l == 0 || L.n > kMgFuseRows) {  // large levels keep their family's SpMV: prolongation, then the residual pass
        hipLaunchKernelGGL((k_mg_prolong<V>), dim3(grid_n(L.n)), dim3(kBlock), 0, s, L.n, L.g, C.g, (V)M->o.omega,
                           (const V *)C.xcur, (const V *)C.dpend, (V *)L.xcur, gate);
        SPK_HIP(hipGetLastError());
        SPK_TRY(smoother_start<V>(M, l, true, io, gate, s));
    } else {
        launch_resid_prolong<V, 8>(M, l, gate, s);
        SPK_HIP(hipGetLastError());
    }
    SPK_TRY(cheb_steps<V>(M, l, false, defer_last, io, gate, s));
    SPK_TRY(timer_mark(M, l, s));
    return SPK_OK;
}

// A whole cycle for the FP64 data of io, in the hierarchy's precision.
static int run_cycle(spk_mg *M, const CycleIo &io, const SysState *gate, hipStream_t s)
{
    MgLevel &L0 = M->lev[0];
    if (M->f32) return enqueue_cycle<float>(M, 0, false, false, false, gate, s, &io);
    L0.b = const_cast<double *>(io.b64);
    L0.x = io.z64;
    return enqueue_cycle<double>(M, 0, false, false, false, gate, s, &io);
}

static int alloc_level_vectors(spk_mg *M, int l)
{
    MgLevel &L = M->lev[l];
    if (l > 0 || M->f32) {  // an FP64 cycle uses the call's arrays on level 0
        SPK_TRY(mg_vec(M, &L.b, L.n));
        SPK_TRY(mg_vec(M, &L.x, L.n));
    }
    if (l < M->nlev - 1) {
        SPK_TRY(mg_vec(M, &L.r, L.n));
        SPK_TRY(mg_vec(M, &L.d0, L.n));
        SPK_TRY(mg_vec(M, &L.d1, L.n));
        if (l > 0) SPK_TRY(mg_vec(M, &L.x2, L.n));
        // level 0's family may change later (spk_mat_set_kernel on the caller's matrix)
        if (l == 0 || (L.A->kernel != SPK_KERNEL_SELL && L.A->kernel != SPK_KERNEL_STREAM))
            SPK_TRY(mg_vec(M, &L.tmp, L.n));
    } else if (l == 0) {
        SPK_TRY(mg_vec(M, &L.tmp, L.n));
    }
    return SPK_OK;
}

// A_c = P^T A P of level l as a new matrix handle.
static int build_coarse(spk_mg *M, int l, const Grid3 &c, hipStream_t s, spk_mat **out)
{
    const MgLevel &L = M->lev[l];
    spk_mat *A = L.A;
    const int nc = c.s0 * c.s1 * c.s2;
    int32_t *cnt = nullptr, *crp = nullptr, *ccol = nullptr;
    double *cval = nullptr;
    int rc = SPK_OK;
    auto done = [&](int code) {
        hipFree(cnt);
        hipFree(crp);
        hipFree(ccol);
        hipFree(cval);
        return code;
    };
    hipError_t e = hipMalloc(&cnt, sizeof(int32_t) * (size_t)nc);
    if (e == hipSuccess) e = hipMalloc(&crp, sizeof(int32_t) * ((size_t)nc + 1));
    if (e != hipSuccess) return done(hip_fail(e, "hipMalloc", __FILE__, __LINE__));
    const int g = grid_n(nc);
    hipLaunchKernelGGL(k_mg_galerkin_count, dim3(g), dim3(kBlock), 0, s, nc, L.g, c, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, (const double *)A->val, cnt);
    hipLaunchKernelGGL(k_mg_scan, dim3(1), dim3(kBlock), 0, s, nc, (const int32_t *)cnt, crp);
    int32_t nnz_c = 0;
    e = hipMemcpyAsync(&nnz_c, crp + nc, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "coarse row counts", __FILE__, __LINE__));
    e = hipMalloc(&ccol, sizeof(int32_t) * (size_t)std::max(nnz_c, 1));
    if (e == hipSuccess) e = hipMalloc(&cval, sizeof(double) * (size_t)std::max(nnz_c, 1));
    if (e != hipSuccess) return done(hip_fail(e, "hipMalloc", __FILE__, __LINE__));
    hipLaunchKernelGGL(k_mg_galerkin_fill, dim3(g), dim3(kBlock), 0, s, nc, L.g, c, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, (const double *)A->val, (const int32_t *)crp, ccol, cval);
    e = hipGetLastError();
    if (e != hipSuccess) return done(hip_fail(e, "galerkin", __FILE__, __LINE__));
    rc = spk_mat_create_csr(nc, nnz_c, crp, ccol, cval, SPK_MEM_DEVICE, 0, s, out);
    if (rc == SPK_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "coarse matrix", __FILE__, __LINE__);
    }
    return done(rc);
}

static __global__ void k_mg_narrow(int64_t m, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// Dense inverse of the coarsest matrix by Gauss-Jordan elimination in FP64
// (rounded to FP32 for an FP32 cycle).
static int invert_coarsest(spk_mg *M, hipStream_t s)
{
    const MgLevel &L = M->lev[M->nlev - 1];
    const int n = L.n;
    const int64_t nn = (int64_t)n * n;
    double *inv = nullptr, *colk = nullptr;
    int32_t *bad = nullptr;
    auto done = [&](int code) {
        hipFree(colk);
        hipFree(bad);
        if (inv != M->cinv) hipFree(inv);
        return code;
    };
    hipError_t e = hipMalloc(&inv, sizeof(double) * (size_t)nn);
    if (e == hipSuccess) e = hipMalloc(&colk, sizeof(double) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&bad, sizeof(int32_t));
    if (e != hipSuccess) return done(hip_fail(e, "hipMalloc", __FILE__, __LINE__));
    int32_t hbad = 0;
    hipLaunchKernelGGL(k_mg_zero, dim3(grid_n(nn)), dim3(kBlock), 0, s, nn, inv);
    e = hipMemcpyAsync(bad, &hbad, sizeof(int32_t), hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_mg_dense, dim3(grid_n(n)), dim3(kBlock), 0, s, n, (const int32_t *)L.A->rowptr,
                       (const int32_t *)L.A->col, (const double *)L.A->val, inv);
    const dim3 gu(ceil_div(n, kBlock), n);
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kBlock), 0, s, n, k, inv, colk, bad);
        hipLaunchKernelGGL(k_gj_update, gu, dim3(kBlock), 0, s, n, k, inv, (const double *)colk);
        e = hipGetLastError();
    }
    if (e == hipSuccess) hipLaunchKernelGGL(k_mg_sym, gu, dim3(kBlock), 0, s, n, inv);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "coarse inverse", __FILE__, __LINE__));
    if (hbad) {
        set_error("the coarsest matrix (%d rows) is not positive definite", n);
        return done(SPK_EINVAL);
    }
    if (!M->f32) {
        M->cinv = inv;
        M->bytes += 8 * nn;
        return done(SPK_OK);
    }
    e = hipMalloc(&M->cinv, sizeof(float) * (size_t)nn);
    if (e != hipSuccess) return done(hip_fail(e, "hipMalloc", __FILE__, __LINE__));
    M->bytes += 4 * nn;
    hipLaunchKernelGGL(k_mg_narrow, dim3(grid_n(nn)), dim3(kBlock), 0, s, nn, (const double *)inv, (float *)M->cinv);
    e = hipStreamSynchronize(s);
    return done(e == hipSuccess ? SPK_OK : hip_fail(e, "coarse inverse", __FILE__, __LINE__));
}

static void destroy_mg(spk_mg *M)
{
    hipStreamSynchronize(M->stream);
    for (int l = 0; l < M->nlev; ++l) {
        MgLevel &L = M->lev[l];
        if (l > 0 || M->f32) {
            hipFree(L.b);
            hipFree(L.x);
        }
        if (l > 0) spk_mat_destroy(L.A);
        hipFree(L.r);
        hipFree(L.d0);
        hipFree(L.d1);
        hipFree(L.x2);
        hipFree(L.tmp);
    }
    hipFree(M->cinv);
    hipFree(M->r);
    hipFree(M->z);
    hipFree(M->p);
    hipFree(M->q);
    hipFree(M->x);
    hipFree(M->b);
    hipFree(M->tmp64);
    hipFree(M->part);
    hipFree(M->hist);
    hipFree(M->st);
    hipHostFree(M->pst);
    hipHostFree(M->pstatus);
    for (auto &e : M->ev)
        if (e) hipEventDestroy(e);
    if (M->g) hipGraphExecDestroy(M->g);
    if (M->cap) hipStreamDestroy(M->cap);
    delete M;
}

static int setup(spk_mg *M, spk_mat *A, const int32_t *shape, hipStream_t s)
{
    MgLevel &L0 = M->lev[0];
    L0.A = A;
    L0.n = A->n;
    L0.g = Grid3{shape[0], M->dim > 1 ? shape[1] : 1, M->dim > 2 ? shape[2] : 1};
    M->nlev = 1;
    // the Galerkin kernels need couplings of at most one grid step
    int32_t *bad = nullptr;
    SPK_HIP(hipMalloc(&bad, sizeof(int32_t)));
    int32_t hbad = 0;
    hipError_t e = hipMemcpyAsync(bad, &hbad, sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mg_reach, dim3(grid_n(A->n)), dim3(kBlock), 0, s, A->n, (const int32_t *)A->rowptr,
                           (const int32_t *)A->col, L0.g, bad);
        e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(bad);
    if (e != hipSuccess) return hip_fail(e, "stencil reach check", __FILE__, __LINE__);
    if (hbad) {
        set_error("%d entries couple grid points more than one step apart: the matrix is not a "
                  "nearest-neighbour stencil on the given grid", hbad);
        return SPK_EINVAL;
    }
    while (M->nlev < M->o.max_levels && M->lev[M->nlev - 1].n > M->o.coarse_max) {
        const MgLevel &F = M->lev[M->nlev - 1];
        const Grid3 c{(F.g.s0 + 1) / 2, (F.g.s1 + 1) / 2, (F.g.s2 + 1) / 2};
        if (c.s0 == F.g.s0 && c.s1 == F.g.s1 && c.s2 == F.g.s2) break;
        spk_mat *Ac = nullptr;
        SPK_TRY(build_coarse(M, M->nlev - 1, c, s, &Ac));
        MgLevel &C = M->lev[M->nlev];
        C.A = Ac;
        C.g = c;
        C.n = Ac->n;
        ++M->nlev;
        M->bytes += Ac->bytes;
    }
    if (M->lev[M->nlev - 1].n > kMgCoarseMax) {
        set_error("coarsest level has %d rows, more than the %d of the dense direct solve (raise max_levels)",
                  M->lev[M->nlev - 1].n, kMgCoarseMax);
        return SPK_EINVAL;
    }
    for (int l = 0; l < M->nlev; ++l) {
        MgLevel &L = M->lev[l];
        if (L.A->stats.zero_diag) {
            set_error("level %d: %d rows without a nonzero diagonal", l, L.A->stats.zero_diag);
            return SPK_EZERODIAG;
        }
        L.emax = L.A->info.gershgorin;
        L.emin = M->o.emin_frac * L.emax;
        if (l < M->nlev - 1 && !(L.emax > 0.0 && std::isfinite(L.emax))) {
            set_error("level %d: no finite spectral bound", l);
            return SPK_EINVAL;
        }
        if (M->f32 && l < M->nlev - 1) {  // FP32 values and D^-1 for the smoother (the caller's level 0 too)
            SPK_TRY(ensure_f32(L.A, s));
            SPK_HIP(hipStreamSynchronize(s));
            L.A->info.has_f32 = 1;
        }
        SPK_TRY(alloc_level_vectors(M, l));
    }
    SPK_TRY(invert_coarsest(M, s));
    SPK_HIP(hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking));
    return SPK_OK;
}

// ------------------------------------------------------------------ MG-preconditioned CG
static int get_solve_ws(spk_mg *M, int hist_len)
{
    const int n = M->lev[0].n;
    if (!M->r) {
        SPK_TRY(mg_alloc(M, &M->r, n));
        SPK_TRY(mg_alloc(M, &M->z, n));
        SPK_TRY(mg_alloc(M, &M->p, n));
        SPK_TRY(mg_alloc(M, &M->q, n));
        SPK_TRY(mg_alloc(M, &M->x, n));
        SPK_TRY(mg_alloc(M, &M->b, n));
        SPK_TRY(mg_alloc(M, &M->tmp64, n));
        SPK_TRY(mg_alloc(M, &M->part, 4 * (int64_t)kMgMaxPart));
        SPK_TRY(mg_alloc(M, &M->st, 1));
        SPK_HIP(hipHostMalloc((void **)&M->pst, sizeof(SysState), hipHostMallocDefault));
        SPK_HIP(hipHostMalloc((void **)&M->pstatus, sizeof(int32_t) * 8, hipHostMallocDefault));
        for (auto &e : M->ev) SPK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const int need = std::max(hist_len, 1);
    if (need > M->hist_cap) {
        hipFree(M->hist);
        M->hist = nullptr;
        SPK_TRY(mg_alloc(M, &M->hist, need));
        M->hist_cap = need;
        if (M->g) {  // the graph holds the old history pointer
            hipGraphExecDestroy(M->g);
            M->g = nullptr;
        }
    }
    return SPK_OK;
}

static int enqueue_iteration(spk_mg *M, hipStream_t s)
{
    MgLevel &L0 = M->lev[0];
    const int n = L0.n;
    const SysState *gate = M->st;
    int np = 0;
    const CycleIo io{M->r, M->z, part_of(M, kPartRzMg), &np, M->r};
    SPK_TRY(run_cycle(M, io, gate, s));
    hipLaunchKernelGGL(k_mg_fin_rho, dim3(1), dim3(kBlock), 0, s, M->st, (const double *)part_of(M, kPartRzMg), np);
    hipLaunchKernelGGL(k_mg_p, dim3(grid_n(n)), dim3(kBlock), 0, s, n, (const double *)M->z, M->p,
                       (const SysState *)M->st);
    SPK_TRY(launch_rows(L0.A, M->p, RowPq{M->p, M->q}, part_of(M, kPartPqMg), &np, gate, M->tmp64, s));
    hipLaunchKernelGGL(k_mg_fin_alpha, dim3(1), dim3(kBlock), 0, s, M->st, (const double *)part_of(M, kPartPqMg), np);
    const int g = grid_n(n);
    hipLaunchKernelGGL(k_mg_update, dim3(g), dim3(kBlock), 0, s, n, M->x, M->r, (const double *)M->p,
                       (const double *)M->q, (const SysState *)M->st, part_of(M, kPartRrMg));
    hipLaunchKernelGGL(k_mg_fin_rnorm, dim3(1), dim3(kBlock), 0, s, M->st, (const double *)part_of(M, kPartRrMg), g,
                       M->hist);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int get_graph(spk_mg *M, int K)
{
    const spk_mat *A0 = M->lev[0].A;
    if (M->g && M->gk == K && M->g_kernel == A0->kernel && M->g_sell == (const void *)A0->sell_val) return SPK_OK;
    if (M->g) {
        hipGraphExecDestroy(M->g);
        M->g = nullptr;
    }
    hipGraph_t graph = nullptr;
    SPK_HIP(hipStreamBeginCapture(M->cap, hipStreamCaptureModeThreadLocal));
    int rc = SPK_OK;
    for (int k = 0; k < K && rc == SPK_OK; ++k) rc = enqueue_iteration(M, M->cap);
    const hipError_t e = hipStreamEndCapture(M->cap, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    const hipError_t e2 = hipGraphInstantiate(&M->g, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        M->g = nullptr;
        return hip_fail(e2, "hipGraphInstantiate", __FILE__, __LINE__);
    }
    M->gk = K;
    M->g_kernel = A0->kernel;
    M->g_sell = A0->sell_val;
    return SPK_OK;
}

// Replays batches of K iterations, two in flight, until the device reports
// that the solve stopped.
static int run_batches(spk_mg *M, int K, bool use_graph, int max_batches, hipStream_t s)
{
    if (use_graph) SPK_TRY(get_graph(M, K));
    constexpr int kDepth = 2;
    int launched = 0, checked = 0;
    for (;;) {
        if (launched - checked < kDepth && launched < max_batches) {
            if (use_graph) SPK_HIP(hipGraphLaunch(M->g, s));
            else
                for (int k = 0; k < K; ++k) SPK_TRY(enqueue_iteration(M, s));
            const int slot = launched % 4;
            hipLaunchKernelGGL(k_mg_publish, dim3(1), dim3(64), 0, s, (const SysState *)M->st, &M->pstatus[slot]);
            SPK_HIP(hipEventRecord(M->ev[slot], s));
            ++launched;
            continue;
        }
        if (checked == launched) {
            SPK_HIP(hipStreamSynchronize(s));
            set_error("solver did not stop within %d batches of %d iterations", max_batches, K);
            return SPK_EHIP;
        }
        const int slot = checked % 4;
        SPK_HIP(hipEventSynchronize(M->ev[slot]));
        ++checked;
        if (M->pstatus[slot] != SPK_RUNNING) break;
    }
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

static int read_state(spk_mg *M, hipStream_t s)
{
    SPK_HIP(hipMemcpyAsync(M->pst, M->st, sizeof(SysState), hipMemcpyDeviceToHost, s));
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

static __global__ void k_mg_restart(SysState *st)
{
    if (threadIdx.x || blockIdx.x) return;
    st->status = SPK_RUNNING;
    st->fresh_p = 1;
    st->rnorm = st->rnorm_true;
}

static __global__ void k_mg_set_status(SysState *st, int status)
{
    if (threadIdx.x || blockIdx.x) return;
    st->status = status;
}

// True residual of M->x into M->r and its norm (state field rnorm_true).
static int true_residual(spk_mg *M, hipStream_t s)
{
    MgLevel &L0 = M->lev[0];
    int np = 0;
    SPK_TRY(launch_rows(L0.A, M->x, RowTrue{M->b, M->r}, part_of(M, kPartRrMg), &np, nullptr, M->tmp64, s));
    hipLaunchKernelGGL(k_mg_fin_true, dim3(1), dim3(kBlock), 0, s, M->st, (const double *)part_of(M, kPartRrMg), np);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int solve(spk_mg *M, const double *b, double *x, const spk_ksp_opts &o, spk_ksp_result *res, hipStream_t s)
{
    MgLevel &L0 = M->lev[0];
    const int n = L0.n;
    SPK_TRY(get_solve_ws(M, o.hist_len));
    SPK_HIP(hipMemcpyAsync(M->b, b, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (o.x0_nonzero) SPK_HIP(hipMemcpyAsync(M->x, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_mg_state_init, dim3(1), dim3(64), 0, s, M->st, o.rtol, o.atol, o.maxit, o.hist_len);
    const int g = grid_n(n);
    hipLaunchKernelGGL(k_mg_start, dim3(g), dim3(kBlock), 0, s, n, (const double *)M->b, M->x, M->r,
                       o.x0_nonzero ? 0 : 1, part_of(M, kPartBbMg));
    int nrr = 0;
    if (o.x0_nonzero)
        SPK_TRY(launch_rows(L0.A, M->x, RowTrue{M->b, M->r}, part_of(M, kPartRrMg), &nrr, nullptr, M->tmp64, s));
    hipLaunchKernelGGL(k_mg_fin_start, dim3(1), dim3(kBlock), 0, s, M->st, (const double *)part_of(M, kPartBbMg), g,
                       o.x0_nonzero ? (const double *)part_of(M, kPartRrMg) : (const double *)nullptr, nrr, M->hist);
    SPK_HIP(hipGetLastError());
    const int K = o.graph_k > 0 ? o.graph_k : 1;
    const bool use_graph = o.graph_k > 0;
    int restarts = 0;
    bool have_true = false;
    for (;;) {
        SPK_TRY(read_state(M, s));
        if (M->pst->status == SPK_RUNNING) {
            const int max_batches = (std::max(o.maxit - M->pst->iter, 0) + K - 1) / K + 2;
            SPK_TRY(run_batches(M, K, use_graph, max_batches, s));
            SPK_TRY(read_state(M, s));
        }
        const SysState &S = *M->pst;
        const bool conv = S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL;
        if (!(conv && S.bnorm > 0 && S.iter > 0)) break;
        // the recursive test passed: confirm with the true residual
        SPK_TRY(true_residual(M, s));
        SPK_TRY(read_state(M, s));
        have_true = true;
        if (M->pst->rnorm_true <= M->pst->thresh) {
            const SysState &T = *M->pst;
            const int reason = T.rnorm_true <= T.rtol * T.bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
            hipLaunchKernelGGL(k_mg_set_status, dim3(1), dim3(64), 0, s, M->st, reason);
            M->pst->status = reason;
            M->pst->rnorm = T.rnorm_true;
            break;
        }
        if (restarts == 3) {
            hipLaunchKernelGGL(k_mg_set_status, dim3(1), dim3(64), 0, s, M->st, (int)SPK_DIVERGED_BREAKDOWN);
            M->pst->status = SPK_DIVERGED_BREAKDOWN;
            M->pst->rnorm = M->pst->rnorm_true;
            break;
        }
        ++restarts;
        hipLaunchKernelGGL(k_mg_restart, dim3(1), dim3(64), 0, s, M->st);
        SPK_HIP(hipGetLastError());
        have_true = false;
    }
    SysState S = *M->pst;
    if (S.bnorm == 0.0) hipLaunchKernelGGL(k_mg_zero, dim3(g), dim3(kBlock), 0, s, (int64_t)n, M->x);
    if (!have_true && S.bnorm > 0.0) {
        SPK_TRY(true_residual(M, s));
        const int status = S.status;
        const double rn = S.rnorm;
        SPK_TRY(read_state(M, s));
        M->pst->status = status;
        M->pst->rnorm = rn;
        S = *M->pst;
    }
    SPK_HIP(hipMemcpyAsync(x, M->x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (o.hist && o.hist_len > 0) {
        const int cnt = std::min(o.hist_len, S.iter + 1);
        SPK_HIP(hipMemcpyAsync(o.hist, M->hist, sizeof(double) * (size_t)cnt, hipMemcpyDeviceToHost, s));
    }
    SPK_HIP(hipStreamSynchronize(s));
    res->reason = S.status;
    res->iterations = S.iter;
    res->restarts = restarts;
    res->rnorm0 = S.rnorm0;
    res->rnorm = S.rnorm;
    res->bnorm = S.bnorm;
    res->true_rel_residual = S.bnorm > 0.0 ? S.rnorm_true / S.bnorm : 0.0;
    return SPK_OK;
}

}  // namespace spk

using namespace spk;

extern "C" {

void spk_mg_opts_default(spk_mg_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_levels = kMgMaxLevels;
    o->coarse_max = 1000;
    o->smooth_steps = 2;
    o->cycle = 1;
    o->emin_frac = 0.1;
    o->omega = 2.0;
}

int spk_mg_create(const spk_mat *Ac, int32_t dim, const int32_t *shape, const spk_mg_opts *opts, void *stream,
                  spk_mg **out)
{
    if (!out) { set_error("out is NULL"); return SPK_EINVAL; }
    *out = nullptr;
    spk_mat *A = const_cast<spk_mat *>(Ac);
    if (!A || !shape) { set_error("A or shape is NULL"); return SPK_EINVAL; }
    if (dim < 1 || dim > 3) { set_error("dim = %d: need 1, 2 or 3", dim); return SPK_EINVAL; }
    int64_t pts = 1;
    for (int d = 0; d < dim; ++d) {
        if (shape[d] < 1) { set_error("shape[%d] = %d < 1", d, shape[d]); return SPK_EINVAL; }
        pts *= shape[d];
    }
    if (pts != A->n || A->n < 1) {
        set_error("grid of %lld points for a matrix of %d rows", (long long)pts, A->n);
        return SPK_EINVAL;
    }
    spk_mg_opts o;
    spk_mg_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_levels < 1 || o.max_levels > kMgMaxLevels) {
        set_error("max_levels = %d outside [1, %d]", o.max_levels, kMgMaxLevels);
        return SPK_EINVAL;
    }
    if (o.coarse_max < 1 || o.coarse_max > kMgCoarseMax) {
        set_error("coarse_max = %d outside [1, %d]", o.coarse_max, kMgCoarseMax);
        return SPK_EINVAL;
    }
    if (o.smooth_steps < 0 || o.smooth_steps > 64) {
        set_error("smooth_steps = %d outside [0, 64]", o.smooth_steps);
        return SPK_EINVAL;
    }
    if (o.cycle != 1 && o.cycle != 2) { set_error("cycle = %d: need 1 (V) or 2 (W)", o.cycle); return SPK_EINVAL; }
    if (!(o.emin_frac > 0.0 && o.emin_frac < 1.0)) {
        set_error("emin_frac = %g outside (0, 1)", o.emin_frac);
        return SPK_EINVAL;
    }
    if (!(o.omega > 0.0) || !std::isfinite(o.omega)) { set_error("omega = %g: need > 0", o.omega); return SPK_EINVAL; }
    if (o.precision != SPK_PREC_FP64 && o.precision != SPK_PREC_MIXED) {
        set_error("precision = %d: need SPK_PREC_FP64 or SPK_PREC_MIXED", o.precision);
        return SPK_EINVAL;
    }
    if (A->stats.zero_diag) {
        set_error("%d rows without a nonzero diagonal", A->stats.zero_diag);
        return SPK_EZERODIAG;
    }
    spk_mg *M = new (std::nothrow) spk_mg();
    if (!M) { set_error("out of host memory"); return SPK_ENOMEM; }
    M->dim = dim;
    M->o = o;
    M->f32 = o.precision == SPK_PREC_MIXED ? 1 : 0;
    hipGetDevice(&M->device);
    M->stream = (hipStream_t)stream;
    const int rc = setup(M, A, shape, (hipStream_t)stream);
    if (rc != SPK_OK) {
        destroy_mg(M);
        return rc;
    }
    *out = M;
    return SPK_OK;
}

int spk_mg_get_info(const spk_mg *M, spk_mg_info *info)
{
    if (!M || !info) { set_error("M or info is NULL"); return SPK_EINVAL; }
    memset(info, 0, sizeof(*info));
    info->levels = M->nlev;
    for (int l = 0; l < M->nlev; ++l) {
        const MgLevel &L = M->lev[l];
        info->n[l] = L.n;
        info->nnz[l] = L.A->nnz;
        info->shape[l][0] = L.g.s0;
        info->shape[l][1] = L.g.s1;
        info->shape[l][2] = L.g.s2;
        info->kernel[l] = L.A->kernel;
        info->emax[l] = L.emax;
    }
    info->device_bytes = M->bytes;
    return SPK_OK;
}

int spk_mg_copy_level(const spk_mg *M, int32_t level, int32_t *rowptr, int32_t *col, double *val)
{
    if (!M || !rowptr || !col || !val) { set_error("NULL argument"); return SPK_EINVAL; }
    if (level < 0 || level >= M->nlev) { set_error("level %d outside [0, %d)", level, M->nlev); return SPK_EINVAL; }
    const spk_mat *A = M->lev[level].A;
    // after the hierarchy's queued work, on its own stream
    hipStream_t s = M->stream;
    SPK_HIP(hipMemcpyAsync(rowptr, A->rowptr, sizeof(int32_t) * ((size_t)A->n + 1), hipMemcpyDeviceToHost, s));
    if (A->nnz > 0) {
        SPK_HIP(hipMemcpyAsync(col, A->col, sizeof(int32_t) * (size_t)A->nnz, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipMemcpyAsync(val, A->val, sizeof(double) * (size_t)A->nnz, hipMemcpyDeviceToHost, s));
    }
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

int spk_mg_apply(spk_mg *M, const double *b, double *x, void *stream)
{
    if (!M || !b || !x) { set_error("NULL argument"); return SPK_EINVAL; }
    const int64_t n = M->lev[0].n;
    if (b < x + n && x < b + n) { set_error("b and x must not overlap"); return SPK_EINVAL; }
    const CycleIo io{b, x, nullptr, nullptr, nullptr};
    M->stream = (hipStream_t)stream;
    return run_cycle(M, io, nullptr, (hipStream_t)stream);
}

int spk_mg_profile(spk_mg *M, const double *b, double *x, int32_t reps, double *level_ms, void *stream)
{
    if (!M || !b || !x || !level_ms) { set_error("NULL argument"); return SPK_EINVAL; }
    if (reps < 1) { set_error("reps = %d < 1", reps); return SPK_EINVAL; }
    const int64_t n = M->lev[0].n;
    if (b < x + n && x < b + n) { set_error("b and x must not overlap"); return SPK_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    M->stream = s;
    for (int l = 0; l < M->nlev; ++l) level_ms[l] = 0.0;
    MgLevel &L0 = M->lev[0];
    int rc = SPK_OK;
    for (int r = 0; r < reps && rc == SPK_OK; ++r) {
        MgTimer t;
        M->timer = &t;
        const CycleIo io{b, x, nullptr, nullptr, nullptr};
        rc = run_cycle(M, io, nullptr, s);
        M->timer = nullptr;
        hipError_t e = hipStreamSynchronize(s);
        if (rc == SPK_OK && e != hipSuccess) rc = hip_fail(e, "profiled cycle", __FILE__, __LINE__);
        for (size_t i = 0; rc == SPK_OK && i + 1 < t.ev.size(); i += 2) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime", __FILE__, __LINE__);
            else level_ms[t.level[i]] += ms / reps;
        }
        for (auto e2 : t.ev) hipEventDestroy(e2);
    }
    return rc;
}

int spk_ksp_solve_mg(spk_mg *M, const double *b, double *x, const spk_ksp_opts *opts, spk_ksp_result *res,
                     void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!M || !b || !x || !res) { set_error("NULL argument"); return SPK_EINVAL; }
    spk_ksp_opts o;
    spk_ksp_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != SPK_PREC_FP64 || o.single_reduction) {
        set_error("multigrid-preconditioned CG runs in FP64 with the two-reduction iteration");
        return SPK_EINVAL;
    }
    if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || o.maxit < 0 || o.graph_k < 0 || o.graph_k > 1024 || o.hist_len < 0 ||
        (o.hist_len > 0 && !o.hist)) {
        set_error("invalid solver options");
        return SPK_EINVAL;
    }
    const int64_t n = M->lev[0].n;
    if (b < x + n && x < b + n) { set_error("b and x must not overlap"); return SPK_EINVAL; }
    memset(res, 0, sizeof(*res));
    M->stream = (hipStream_t)stream;
    const int rc = solve(M, b, x, o, res, (hipStream_t)stream);
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int spk_mg_destroy(spk_mg *M)
{
    if (!M) return SPK_OK;
    destroy_mg(M);
    return SPK_OK;
}

}  // extern "C"
