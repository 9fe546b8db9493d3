// Geometric multigrid kernels (the multigrid of Sec. 5.3: Jacobi-preconditioned
// Chebyshev smoothing on every level but the coarsest, a direct solve on the
// coarsest, V- or W-cycles), and the kernels of CG preconditioned by one
// cycle per iteration.
//
// Grid transfers are aggregation on the logically structured grid: fine point
// (i0, i1, i2) (i0 fastest) belongs to coarse point (i0/2, i1/2, i2/2) of the
// grid with extents ceil(s/2); prolongation is piecewise constant, restriction
// its transpose, and the coarse operator the Galerkin product P^T A P.  For a
// matrix whose couplings reach at most one grid step in each direction (5-,
// 7-, 9- or 27-point stencils) the coarse operator keeps that reach, so coarse
// row I has at most 3^d entries, one per neighbour slot (dz, dy, dx).
//
// Every kernel that runs inside a captured solve takes the solve's state and
// does nothing once the solve stopped (gate null: always run).
#pragma once

#include "cheb.hpp"

namespace spk {

constexpr int kMgMaxLevels = 16;
constexpr int kMgCoarseMax = 4096;  // rows of the densely inverted coarsest level
constexpr int kMgMaxPart = 16384;   // partial sums per reduction (largest grid)

struct Grid3 {
    int s0, s1, s2;  // extents, s0 fastest; unused dimensions are 1
};

__device__ __forceinline__ void grid_coords(const Grid3 &g, int i, int &c0, int &c1, int &c2)
{
    c0 = i % g.s0;
    const int t = i / g.s0;
    c1 = t % g.s1;
    c2 = t / g.s1;
}

__device__ __forceinline__ bool mg_go(const SysState *gate)
{
    return !gate || gate_open(gate, kGateInner64);
}

// ------------------------------------------------------------------ setup
// Entries that couple grid points more than one step apart in some direction.
static __global__ void k_mg_reach(int n, const int32_t *__restrict__ rowptr,
                                  const int32_t *__restrict__ col, Grid3 g, int32_t *bad)
{
    int cnt = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int i0, i1, i2;
        grid_coords(g, i, i0, i1, i2);
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j0, j1, j2;
            grid_coords(g, col[k], j0, j1, j2);
            cnt += (abs(j0 - i0) > 1 || abs(j1 - i1) > 1 || abs(j2 - i2) > 1) ? 1 : 0;
        }
    }
    if (cnt) atomicAdd(bad, cnt);
}

// Coarse row I of P^T A P summed per neighbour slot: the aggregate's fine
// rows in the order (z, y, x) of their offsets, each row's entries in column
// order, so the sums are reproducible bit for bit.
__device__ __forceinline__ uint32_t galerkin_row(int I, const Grid3 &g, const Grid3 &c,
                                                 const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, double acc[27])
{
    int c0, c1, c2;
    grid_coords(c, I, c0, c1, c2);
    uint32_t mask = 0;
#pragma unroll
    for (int s = 0; s < 27; ++s) acc[s] = 0.0;
    for (int a2 = 0; a2 < 2; ++a2) {
        const int f2 = 2 * c2 + a2;
        if (f2 >= g.s2) continue;
        for (int a1 = 0; a1 < 2; ++a1) {
            const int f1 = 2 * c1 + a1;
            if (f1 >= g.s1) continue;
            for (int a0 = 0; a0 < 2; ++a0) {
                const int f0 = 2 * c0 + a0;
                if (f0 >= g.s0) continue;
                const int i = f0 + g.s0 * (f1 + g.s1 * f2);
                for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                    int j0, j1, j2;
                    grid_coords(g, col[k], j0, j1, j2);
                    const int slot = (j2 / 2 - c2 + 1) * 9 + (j1 / 2 - c1 + 1) * 3 + (j0 / 2 - c0 + 1);
                    acc[slot] += val[k];
                    mask |= 1u << slot;
                }
            }
        }
    }
    return mask;
}

static __global__ void k_mg_galerkin_count(int nc, Grid3 g, Grid3 c, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col,
                                           const double *__restrict__ val, int32_t *__restrict__ cnt)
{
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        double acc[27];
        cnt[I] = __popc(galerkin_row(I, g, c, rowptr, col, val, acc));
    }
}

// Slots in ascending (dz, dy, dx) order give ascending coarse columns.
static __global__ void k_mg_galerkin_fill(int nc, Grid3 g, Grid3 c, const int32_t *__restrict__ rowptr,
                                          const int32_t *__restrict__ col,
                                          const double *__restrict__ val,
                                          const int32_t *__restrict__ crowptr,
                                          int32_t *__restrict__ ccol, double *__restrict__ cval)
{
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        double acc[27];
        const uint32_t mask = galerkin_row(I, g, c, rowptr, col, val, acc);
        int c0, c1, c2;
        grid_coords(c, I, c0, c1, c2);
        int k = crowptr[I];
        for (int s = 0; s < 27; ++s) {
            if (!((mask >> s) & 1u)) continue;
            const int d2 = s / 9 - 1, d1 = (s / 3) % 3 - 1, d0 = s % 3 - 1;
            ccol[k] = (c0 + d0) + c.s0 * ((c1 + d1) + c.s1 * (c2 + d2));
            cval[k] = acc[s];
            ++k;
        }
    }
}

// Exclusive scan of n counts into rowptr[0..n] by one block: each thread
// sums a contiguous segment, the segment sums are scanned in order, then
// each thread writes its segment.
static __global__ __launch_bounds__(kBlock) void k_mg_scan(int n, const int32_t *__restrict__ cnt,
                                                           int32_t *__restrict__ rowptr)
{
    __shared__ long long part[kBlock];
    const int per = (n + kBlock - 1) / kBlock;
    const int b = min(n, (int)threadIdx.x * per), e = min(n, b + per);
    long long s = 0;
    for (int i = b; i < e; ++i) s += cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int t = 0; t < kBlock; ++t) {
            const long long v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    long long run = part[threadIdx.x];
    for (int i = b; i < e; ++i) {
        rowptr[i] = (int32_t)run;
        run += cnt[i];
    }
    if (threadIdx.x == kBlock - 1) rowptr[n] = (int32_t)run;
}

// Dense copy of a CSR matrix (M zeroed beforehand), row-major.
static __global__ void k_mg_dense(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                  const double *__restrict__ val, double *__restrict__ M)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) M[(size_t)i * n + col[k]] = val[k];
}

// In-place Gauss-Jordan inversion without pivoting (the matrix is SPD), step
// k in two launches.  First (one block): keep column k, then scale row k by
// 1/a_kk and store 1/a_kk on the diagonal.
static __global__ __launch_bounds__(kBlock) void k_gj_pivot(int n, int k, double *__restrict__ M,
                                                            double *__restrict__ colk, int32_t *bad)
{
    const double piv = M[(size_t)k * n + k];
    for (int i = threadIdx.x; i < n; i += kBlock) colk[i] = M[(size_t)i * n + k];
    __syncthreads();
    if (!(piv > 0.0)) {
        if (threadIdx.x == 0) atomicAdd(bad, 1);
        return;
    }
    const double inv = 1.0 / piv;
    for (int j = threadIdx.x; j < n; j += kBlock) {
        double *a = &M[(size_t)k * n + j];
        *a = j == k ? inv : *a * inv;
    }
}

// Second: eliminate column k from every other row, a_ij -= a_ik a_kj, and
// a_ik = -a_ik / a_kk (grid: x over columns, y over rows).
static __global__ void k_gj_update(int n, int k, double *__restrict__ M, const double *__restrict__ colk)
{
    const int i = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == k || j >= n) return;
    const double f = colk[i];
    double *a = &M[(size_t)i * n + j];
    if (j == k) *a = -f * M[(size_t)k * n + k];
    else *a = fma(-f, M[(size_t)k * n + j], *a);
}

// M = (M + M^T) / 2 (the inverse of a symmetric matrix, symmetric to the bit).
static __global__ void k_mg_sym(int n, double *__restrict__ M)
{
    const int i = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || j <= i) return;
    const double v = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
    M[(size_t)i * n + j] = v;
    M[(size_t)j * n + i] = v;
}

// ------------------------------------------------------------------ the cycle
// Kernels of the cycle take V = double, or float for the FP32 cycle of a
// mixed-precision preconditioner (FP32 values, vectors and arithmetic).

// Coarsest level: x = A_c^-1 b with the stored inverse, one wavefront per row.
template <class V>
__global__ __launch_bounds__(kBlock) void k_mg_gemv(int n, const V *__restrict__ M, const V *__restrict__ b,
                                                    V *__restrict__ x, const SysState *gate)
{
    if (!mg_go(gate)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int i = blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave;
    if (i >= n) return;
    const V *row = M + (size_t)i * n;
    V s = V(0);
    for (int j = lane; j < n; j += kWave) s = fma(row[j], b[j], s);
    s = wave_sum(s);
    if (lane == 0) x[i] = s;
}

// b_c = P^T r: the sum over each aggregate, fine points in (z, y, x) order.
template <class V>
__global__ void k_mg_restrict(Grid3 g, Grid3 c, const V *__restrict__ r, V *__restrict__ bc,
                              const SysState *gate)
{
    if (!mg_go(gate)) return;
    const int nc = c.s0 * c.s1 * c.s2;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        int c0, c1, c2;
        grid_coords(c, I, c0, c1, c2);
        V t = V(0);
        for (int a2 = 0; a2 < 2; ++a2) {
            const int f2 = 2 * c2 + a2;
            if (f2 >= g.s2) continue;
            for (int a1 = 0; a1 < 2; ++a1) {
                const int f1 = 2 * c1 + a1;
                if (f1 >= g.s1) continue;
                const V *rr = r + (size_t)g.s0 * (f1 + (size_t)g.s1 * f2);
                t += rr[2 * c0];
                if (2 * c0 + 1 < g.s0) t += rr[2 * c0 + 1];
            }
        }
        bc[I] = t;
    }
}

// Index of the aggregate holding fine point i.
__device__ __forceinline__ int aggregate_of(const Grid3 &g, const Grid3 &c, int i)
{
    int i0, i1, i2;
    grid_coords(g, i, i0, i1, i2);
    return (i0 >> 1) + c.s0 * ((i1 >> 1) + c.s1 * (i2 >> 1));
}

// The coarse result x_c, plus the coarse level's last smoothing step d_c
// when that step was left to this pass (dc null: already added).
template <class V>
__device__ __forceinline__ V coarse_value(const V *__restrict__ xc, const V *__restrict__ dc, int I)
{
    return dc ? xc[I] + dc[I] : xc[I];
}

// Coarse-grid correction x += omega P x_c.
template <class V>
__global__ void k_mg_prolong(int n, Grid3 g, Grid3 c, V omega, const V *__restrict__ xc, const V *__restrict__ dc,
                             V *__restrict__ x, const SysState *gate)
{
    if (!mg_go(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = fma(omega, coarse_value(xc, dc, aggregate_of(g, c, i)), x[i]);
}

// Restriction fused with the coarse level's smoother start from zero:
// b_c = P^T r (the sum over each aggregate, (z, y, x) order), x_c = 0,
// r_c = b_c, d_0 = D_c^-1 b_c / theta_c.
template <class V>
__global__ void k_mg_init_restrict(Grid3 g, Grid3 c, const V *__restrict__ r, V *__restrict__ bc,
                                   V *__restrict__ xc, V *__restrict__ rc, V *__restrict__ d0,
                                   const V *__restrict__ dinv, V inv_theta, const SysState *gate)
{
    if (!mg_go(gate)) return;
    const int nc = c.s0 * c.s1 * c.s2;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        int c0, c1, c2;
        grid_coords(c, I, c0, c1, c2);
        V t = V(0);
        for (int a2 = 0; a2 < 2; ++a2) {
            const int f2 = 2 * c2 + a2;
            if (f2 >= g.s2) continue;
            for (int a1 = 0; a1 < 2; ++a1) {
                const int f1 = 2 * c1 + a1;
                if (f1 >= g.s1) continue;
                const V *rr = r + (size_t)g.s0 * (f1 + (size_t)g.s1 * f2);
                t += rr[2 * c0];
                if (2 * c0 + 1 < g.s0) t += rr[2 * c0 + 1];
            }
        }
        bc[I] = t;
        xc[I] = V(0);
        rc[I] = t;
        d0[I] = dinv[I] * t * inv_theta;
    }
}

// Prolongation fused with the post-smoother's start on a coarse level (CSR,
// L lanes per row): with x' = x + omega P x_c formed for every gathered
// column, r = b - A x', d_0 = D^-1 r / theta, and x' of the row itself goes
// to x2 (x stays unchanged: other blocks still gather it).
template <class V, int L>
__global__ __launch_bounds__(kBlock) void k_mg_resid_prolong(int n, const int32_t *__restrict__ rowptr,
                                                             const int32_t *__restrict__ col,
                                                             const V *__restrict__ val, const V *__restrict__ dinv,
                                                             const V *__restrict__ b, const V *__restrict__ x,
                                                             const V *__restrict__ xc, const V *__restrict__ dc,
                                                             V omega, Grid3 g, Grid3 c, V *__restrict__ x2,
                                                             V *__restrict__ r, V *__restrict__ d0, V inv_theta,
                                                             const SysState *gate)
{
    if (!mg_go(gate)) return;
    const int lane = threadIdx.x % L;
    const int groups = gridDim.x * (kBlock / L);
    for (int i = blockIdx.x * (kBlock / L) + (int)threadIdx.x / L; i < n; i += groups) {
        V s = V(0);
        for (int k = rowptr[i] + lane; k < rowptr[i + 1]; k += L) {
            const int j = col[k];
            s = fma(val[k], fma(omega, coarse_value(xc, dc, aggregate_of(g, c, j)), x[j]), s);
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (lane == 0) {
            x2[i] = fma(omega, coarse_value(xc, dc, aggregate_of(g, c, i)), x[i]);
            const V ri = b[i] - s;
            r[i] = ri;
            d0[i] = dinv[i] * ri * inv_theta;
        }
    }
}

// Level-0 end of the cycle: z = x + d (the last smoothing step; d null when
// there is none) in FP64, and, when part is set, the partial sums of r . z
// (the CG inner product).  With V = double, x and z may be the same array.
template <class V>
__global__ __launch_bounds__(kBlock) void k_mg_finish(int n, const V *__restrict__ d, const V *x,
                                                      double *z, const double *__restrict__ r, double *part,
                                                      const SysState *gate)
{
    if (!mg_go(gate)) return;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double zi = (double)(d ? x[i] + d[i] : x[i]);
        z[i] = zi;
        if (part) acc += r[i] * zi;
    }
    if (part) {
        __shared__ double sh[kBlock / kWave];
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

// FP64 right-hand side rounded into the FP32 cycle's level-0 vector.
static __global__ void k_mg_round(int n, const double *__restrict__ a, float *__restrict__ b, const SysState *gate)
{
    if (!mg_go(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ SpMV rows with an epilogue
// Row epilogues: f(i, y = (A x)_i) stores what the row produces and returns
// its contribution to an inner product (0 when none is wanted).

// Smoother start from a nonzero x: r = b - A x, d_0 = D^-1 r / theta.
template <class V>
struct RowResid {
    const V *b;
    V *r, *d0;
    const V *dinv;
    V inv_theta;
    __device__ double operator()(int i, V y) const
    {
        const V ri = b[i] - y;
        r[i] = ri;
        d0[i] = dinv[i] * ri * inv_theta;
        return 0.0;
    }
};

// CG: q = A p and p.q.
struct RowPq {
    const double *p;
    double *q;
    __device__ double operator()(int i, double y) const
    {
        q[i] = y;
        return p[i] * y;
    }
};

// True residual r = b - A x and r.r.
struct RowTrue {
    const double *b;
    double *r;
    __device__ double operator()(int i, double y) const
    {
        const double ri = b[i] - y;
        r[i] = ri;
        return ri * ri;
    }
};

__device__ __forceinline__ void store_partial(double acc, double *part)
{
    __shared__ double sh[kBlock / kWave];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <class V, class CI, int U, class F>
__global__ __launch_bounds__(kBlock) void k_mg_rows_sell(int n, SellView sv, const V *__restrict__ val,
                                                         const V *__restrict__ x, F f, double *part,
                                                         const SysState *gate)
{
    double acc = 0.0;
    bool run = true;
    sell_slices<V, CI, U>(n, blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave,
                          gridDim.x * (kBlock / kWave), sv, val, x, [&] { return run = mg_go(gate); },
                          [&](int i, V y) { acc += f(i, y); });
    if (part && run) store_partial(acc, part);
}

template <class V, class F>
__global__ __launch_bounds__(kBlock) void k_mg_rows_stream(int n, int R, int ntiles, int nblk,
                                                           const int32_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ col,
                                                           const V *__restrict__ val, const V *__restrict__ x,
                                                           F f, double *part, const SysState *gate)
{
    if (!mg_go(gate)) return;
    __shared__ TileLds<V> sm;
    const int j = xcd_remap(blockIdx.x, nblk);
    int t0, t1;
    block_tiles(j, nblk, ntiles, t0, t1);
    double acc = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * R;
        const int r1 = min(r0 + R, n);
        stream_tile<V>(r0, r1, rowptr, col, val, x, sm, [&](int i, V y) { acc += f(i, y); });
    }
    if (part) store_partial(acc, part);
}

// Other families: y = A x came from the standalone SpMV.
template <class V, class F>
__global__ __launch_bounds__(kBlock) void k_mg_rows_y(int n, const V *__restrict__ y, F f, double *part,
                                                      const SysState *gate)
{
    if (!mg_go(gate)) return;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += f(i, y[i]);
    if (part) store_partial(acc, part);
}

// ------------------------------------------------------------------ CG around the cycle
// Start: partial b.b; for x0 = 0 also x = 0 and r = b.
static __global__ __launch_bounds__(kBlock) void k_mg_start(int n, const double *__restrict__ b,
                                                            double *__restrict__ x, double *__restrict__ r,
                                                            int zero_x, double *part)
{
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double bi = b[i];
        acc += bi * bi;
        if (zero_x) {
            x[i] = 0.0;
            r[i] = bi;
        }
    }
    store_partial(acc, part);
}

static __global__ void k_mg_state_init(SysState *st, double rtol, double atol, int maxit, int hist_len)
{
    if (threadIdx.x || blockIdx.x) return;
    SysState s{};
    s.status = SPK_RUNNING;
    s.phase = kPhaseInner;
    s.maxit = maxit;
    s.hist_len = hist_len;
    s.fresh_p = 1;
    s.rtol = rtol;
    s.atol = atol;
    *st = s;
}

// ||b||, ||r_0||, the threshold and the first test (one block).
static __global__ __launch_bounds__(kBlock) void k_mg_fin_start(SysState *st, const double *part_bb, int nbb,
                                                                const double *part_rr, int nrr,
                                                                double *hist)
{
    __shared__ double sh[kBlock / kWave];
    const double bb = reduce_partials(part_bb, nbb, sh);
    const double rr = part_rr ? reduce_partials(part_rr, nrr, sh) : bb;
    if (threadIdx.x) return;
    const double bn = sqrt(bb), rn = sqrt(rr);
    st->bnorm = bn;
    st->rnorm0 = rn;
    st->rnorm = rn;
    const double thresh = fmax(st->rtol * bn, st->atol);
    st->thresh = thresh;
    if (st->hist_len > 0) hist[0] = bn == 0.0 ? 0.0 : rn;
    if (bn == 0.0) st->status = SPK_CONVERGED_ATOL;
    else if (!isfinite(rn)) st->status = SPK_DIVERGED_NANORINF;
    else if (rn <= thresh) st->status = rn <= st->rtol * bn ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
}

// rho' = r.z with its checks; beta = rho'/rho, or p = z after a (re)start.
static __global__ __launch_bounds__(kBlock) void k_mg_fin_rho(SysState *st, const double *part, int np)
{
    if (st->status != SPK_RUNNING) return;
    __shared__ double sh[kBlock / kWave];
    const double rho = reduce_partials(part, np, sh);
    if (threadIdx.x) return;
    if (!isfinite(rho)) { st->status = SPK_DIVERGED_NANORINF; return; }
    if (rho < 0.0) { st->status = SPK_DIVERGED_INDEFINITE_PC; return; }
    if (rho == 0.0) { st->status = SPK_DIVERGED_BREAKDOWN; return; }
    st->cmode = st->fresh_p;  // 1: p = z
    st->beta = st->fresh_p ? 0.0 : rho / st->rho;
    st->fresh_p = 0;
    st->rho = rho;
}

static __global__ void k_mg_p(int n, const double *__restrict__ z, double *__restrict__ p, const SysState *st)
{
    if (st->status != SPK_RUNNING) return;
    const bool first = st->cmode != 0;
    const double beta = st->beta;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = first ? z[i] : fma(beta, p[i], z[i]);
}

// eta = p.Ap with its checks; alpha = rho / eta.
static __global__ __launch_bounds__(kBlock) void k_mg_fin_alpha(SysState *st, const double *part, int np)
{
    if (st->status != SPK_RUNNING) return;
    __shared__ double sh[kBlock / kWave];
    const double eta = reduce_partials(part, np, sh);
    if (threadIdx.x) return;
    if (!isfinite(eta)) { st->status = SPK_DIVERGED_NANORINF; return; }
    if (eta <= 0.0) { st->status = SPK_DIVERGED_INDEFINITE_MAT; return; }
    st->eta = eta;
    st->alpha = st->rho / eta;
}

// x += alpha p, r -= alpha q, and r.r.
static __global__ __launch_bounds__(kBlock) void k_mg_update(int n, double *__restrict__ x, double *__restrict__ r,
                                                             const double *__restrict__ p,
                                                             const double *__restrict__ q, const SysState *st,
                                                             double *part)
{
    if (st->status != SPK_RUNNING) return;
    const double alpha = st->alpha;
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        acc += ri * ri;
    }
    store_partial(acc, part);
}

// ||r_k||, the iteration count, the history and the stopping tests.
static __global__ __launch_bounds__(kBlock) void k_mg_fin_rnorm(SysState *st, const double *part, int np,
                                                                double *hist)
{
    if (st->status != SPK_RUNNING) return;
    __shared__ double sh[kBlock / kWave];
    const double rr = reduce_partials(part, np, sh);
    if (threadIdx.x) return;
    const double rn = sqrt(rr);
    const int k = st->iter + 1;
    st->iter = k;
    st->rnorm = rn;
    if (k < st->hist_len) hist[k] = rn;
    if (!isfinite(rn)) st->status = SPK_DIVERGED_NANORINF;
    else if (rn <= st->thresh) st->status = rn <= st->rtol * st->bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
    else if (k >= st->maxit) st->status = SPK_DIVERGED_ITS;
}

static __global__ __launch_bounds__(kBlock) void k_mg_fin_true(SysState *st, const double *part, int np)
{
    __shared__ double sh[kBlock / kWave];
    const double rr = reduce_partials(part, np, sh);
    if (threadIdx.x == 0) st->rnorm_true = sqrt(rr);
}

static __global__ void k_mg_publish(const SysState *st, int32_t *host)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) host[0] = st->status;
}

static __global__ void k_mg_zero(int64_t n, double *__restrict__ a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

}  // namespace spk
