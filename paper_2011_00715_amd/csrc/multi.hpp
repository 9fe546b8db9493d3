// Multiple right-hand sides (Sec. 4 Response F3: Krylov methods with several
// right-hand sides read the matrix once for all of them and fuse their outer
// loops).  Vectors are row-major n x K (entry (i, j) at i K + j), so a gather
// of row c fetches the K values of all columns with one or two vector loads.
//
//   k_spmm_*        Y = A X
//   k_m_*           K independent Jacobi-PCG recurrences that share every
//                   SpMM: per-column scalars and stopping tests, per-column
//                   per-block partial sums reduced in a fixed order by
//                   one-block finalize kernels, so each column's iterates are
//                   those of its own single-right-hand-side solve up to the
//                   rounding order of the SpMV and the dots.
#pragma once

#include "spmv.hpp"

namespace spk {

constexpr int kMultiMax = 16;

// Purpose of a residual launch: the setup of a solve, or the true residual.
enum { kMultiSetup = 0, kMultiTrue = 1 };

// Columns still iterating (bit j), written by the finalize kernels.
struct MultiCtl {
    int32_t mask;
    int32_t pad_;
};

struct MultiDesc {
    int32_t n, K, nblk, R, ntiles;
    int32_t sell;                // 1: the SELL layout drives the row walk
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *dinv;
    SellView sv;
    const double *sell_val;
    const double *B;
    double *X, *Rv, *Z, *P, *Q;  // n x K each
    double *partials;            // [kNumPart][K][nblk]
    SysState *st;                // K states
    MultiCtl *ctl;
};

// One (row, column) item per lane: a wavefront takes G = 64 / K consecutive
// rows and all K columns, lane t holding row t / K and column q = t % K, so
// the K values gathered for an entry are adjacent lanes' addresses (one
// contiguous 8K-byte segment per row) and the outputs are lane-contiguous.
// The lanes of a row load the same offsets and values (a broadcast).
// Entries in column order, FMA, U per round with the gathers issued together.
template <int K>
__device__ __forceinline__ double csr_item(int a, int e, int q, const int32_t *__restrict__ col,
                                           const double *__restrict__ val, const double *__restrict__ X)
{
    constexpr int U = 8;
    double acc = 0.0;
    for (int k0 = a; k0 < e; k0 += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u < e ? k0 + u : e - 1;
            c[u] = ld_stream(col + k);
            v[u] = ld_stream(val + k);
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[(size_t)c[u] * K + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < e) acc = fma(v[u], xv[u], acc);
    }
    return acc;
}

template <class CI, int K>
__device__ __forceinline__ double sell_item(const SellView &sv, const double *__restrict__ val,
                                            const double *__restrict__ X, int32_t b, int slen, int rlen,
                                            int so, int row, int q)
{
    constexpr int U = 8;
    const CI *__restrict__ col = reinterpret_cast<const CI *>(sv.col) + b + so;
    const double *__restrict__ v = val + b + so;
    double acc = 0.0;
    for (int j0 = 0; j0 < slen; j0 += U) {
        CI c[U];
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u < slen ? j0 + u : slen - 1;
            c[u] = ld_stream(col + (size_t)j * kSell);
            a[u] = ld_stream(v + (size_t)j * kSell);
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = X[(size_t)(row + (int)c[u]) * K + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < rlen) acc = fma(a[u], xv[u], acc);
    }
    return acc;
}

// Items of block l (of nblk): SELL row groups in round-robin order (slice s
// has K groups of G rows), or the block's contiguous tile range of CSR rows.
// fn(e, row, y) for item e = row K + q with y = (A X)[row, q].
template <class CI, int K, class Fn>
__device__ __forceinline__ void multi_items(const MultiDesc &d, int l, int j, const double *__restrict__ X,
                                            Fn &&fn)
{
    constexpr int G = kWave / K;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int q = lane % K, ro = lane / K;
    if (d.sell) {
        const int ns = (d.n + kSell - 1) / kSell;
        const int ngroups = ns * K;
        for (int g = l * (kBlock / kWave) + wv; g < ngroups; g += d.nblk * (kBlock / kWave)) {
            const int s = g / K, so = (g % K) * G + ro;
            const int row = s * kSell + so;
            if (row >= d.n) continue;
            const int32_t b = d.sv.ptr[s], e = d.sv.ptr[s + 1];
            const double y = sell_item<CI, K>(d.sv, d.sell_val, X, b, (e - b) / kSell, d.sv.len[row], so, row, q);
            fn((int64_t)row * K + q, row, y);
        }
    } else {
        int t0, t1;
        block_tiles(j, d.nblk, d.ntiles, t0, t1);
        const int rb = t0 * d.R, re = min(t1 * d.R, d.n);
        for (int r0 = rb + wv * G; r0 < re; r0 += (kBlock / kWave) * G) {
            const int row = r0 + ro;
            if (row >= re) continue;
            const double y = csr_item<K>(d.rowptr[row], d.rowptr[row + 1], q, d.col, d.val, X);
            fn((int64_t)row * K + q, row, y);
        }
    }
}

// Block sums when lane t always holds column t % K (flat n x K element
// walks with a stride that is a multiple of K): lanes of one column are
// combined by the butterfly levels at distances >= K, then the waves in order.
template <int K>
__device__ __forceinline__ void block_partials_flat(double v, double *sh /* [4][K] */, double *part,
                                                    int nblk, int j)
{
#pragma unroll
    for (int off = kWave / 2; off >= K; off >>= 1) v += __shfl_xor(v, off, kWave);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    __syncthreads();
    if (lane < K) sh[w * K + lane] = v;
    __syncthreads();
    if ((int)threadIdx.x < K) {
        const int q = threadIdx.x;
        double s = sh[q];
#pragma unroll
        for (int ww = 1; ww < kBlock / kWave; ++ww) s += sh[ww * K + q];
        part[(size_t)q * nblk + j] = s;
    }
}

// Elements [rb K, re K) of the block's rows in the flat n x K layout, with
// the lane's fixed column q = threadIdx.x % K; fn(e, i) for element e of row i.
template <int K, class Fn>
__device__ __forceinline__ void flat_walk(const MultiDesc &d, int j, Fn &&fn)
{
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const int64_t e0 = (int64_t)t0 * d.R * K, e1 = (int64_t)min(t1 * d.R, d.n) * K;
    constexpr int U = 4;
    for (int64_t eb = e0 + threadIdx.x; eb < e1; eb += (int64_t)kBlock * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (int64_t)u * kBlock;
            if (e < e1) fn(e, (int)(e / K));
        }
    }
}

__device__ __forceinline__ int multi_block(const MultiDesc &d, int &j)
{
    if ((int)blockIdx.x >= d.nblk) return -1;
    j = xcd_remap(blockIdx.x, d.nblk);
    return blockIdx.x;
}

// ------------------------------------------------------------------ SpMM
template <class CI, int K>
__global__ __launch_bounds__(kBlock) void k_spmm(MultiDesc d, const double *__restrict__ X, double *__restrict__ Y)
{
    int j;
    const int l = multi_block(d, j);
    if (l < 0) return;
    multi_items<CI, K>(d, l, j, X, [&](int64_t e, int, double y) { Y[e] = y; });
}

// ------------------------------------------------------------------ residual
// R = B - A X for the columns in `mask` (others untouched), per-column
// per-block r.r and b.b.
template <class CI, int K>
__global__ __launch_bounds__(kBlock) void k_m_resid(MultiDesc d, int32_t mask)
{
    __shared__ double sh[(kBlock / kWave) * K];
    int j;
    const int l = multi_block(d, j);
    if (l < 0) return;
    const int q = threadIdx.x % K;
    const bool on = (mask >> q) & 1;
    double rr = 0.0, bb = 0.0;
    multi_items<CI, K>(d, l, j, d.X, [&](int64_t e, int, double y) {
        if (!on) return;
        const double bi = d.B[e];
        const double ri = bi - y;
        d.Rv[e] = ri;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    });
    block_partials_flat<K>(rr, sh, d.partials + (size_t)kPartRr * K * d.nblk, d.nblk, j);
    block_partials_flat<K>(bb, sh, d.partials + (size_t)kPartBb * K * d.nblk, d.nblk, j);
}

// Column q's sum of partials part[q * nblk + 0 .. nblk), by one wavefront,
// in a fixed order (lane-strided, then the butterfly).
__device__ __forceinline__ double wave_reduce_col(const double *part, int nblk)
{
    const int lane = threadIdx.x & (kWave - 1);
    double s = 0.0;
    for (int i = lane; i < nblk; i += kWave) s += part[i];
    return wave_sum(s);
}

__device__ __forceinline__ void publish_mask(const MultiDesc &d)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = 0;
        for (int q = 0; q < d.K; ++q)
            if (d.st[q].status == SPK_RUNNING) m |= 1 << q;
        d.ctl->mask = m;
    }
}

// purpose kMultiSetup: norms, thresholds, stop at start; kMultiTrue: store the
// true residual norm of the columns in mask.
static __global__ __launch_bounds__(kBlock) void k_m_fin_resid(MultiDesc d, int purpose, int32_t mask)
{
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int q = w; q < d.K; q += kBlock / kWave) {
        if (!((mask >> q) & 1)) continue;
        const double RR = wave_reduce_col(d.partials + ((size_t)kPartRr * d.K + q) * d.nblk, d.nblk);
        const double BB = wave_reduce_col(d.partials + ((size_t)kPartBb * d.K + q) * d.nblk, d.nblk);
        if (lane != 0) continue;
        SysState *st = d.st + q;
        const double rn = sqrt(RR);
        if (purpose == kMultiTrue) {
            st->rnorm_true = rn;
            continue;
        }
        const double bn = sqrt(BB);
        st->bnorm = bn;
        st->thresh = fmax(st->rtol * bn, st->atol);
        st->rnorm = rn;
        st->rnorm0 = rn;
        if (bn == 0.0) st->status = SPK_CONVERGED_ATOL;
        else if (!isfinite(rn) || !isfinite(bn)) st->status = SPK_DIVERGED_NANORINF;
        else if (rn <= st->thresh) st->status = rn <= st->rtol * bn ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
    }
    publish_mask(d);
}

// ------------------------------------------------------------------ setup
// Z = D^-1 R, P = Z for the running columns in mask, per-block r.z.
template <int K>
__global__ __launch_bounds__(kBlock) void k_m_setup(MultiDesc d, int32_t mask)
{
    __shared__ double sh[(kBlock / kWave) * K];
    int j;
    if (multi_block(d, j) < 0) return;
    const int q = threadIdx.x % K;
    const bool run = ((mask >> q) & 1) && d.st[q].status == SPK_RUNNING;
    double rz = 0.0;
    if (run)
        flat_walk<K>(d, j, [&](int64_t e, int i) {
            const double ri = d.Rv[e];
            const double zi = d.dinv[i] * ri;
            d.Z[e] = zi;
            d.P[e] = zi;
            rz = fma(ri, zi, rz);
        });
    block_partials_flat<K>(rz, sh, d.partials + (size_t)kPartRz * K * d.nblk, d.nblk, j);
}

static __global__ __launch_bounds__(kBlock) void k_m_fin_setup(MultiDesc d, int32_t mask)
{
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int q = w; q < d.K; q += kBlock / kWave) {
        if (!((mask >> q) & 1)) continue;
        SysState *st = d.st + q;
        if (st->status != SPK_RUNNING) continue;
        const double RZ = wave_reduce_col(d.partials + ((size_t)kPartRz * d.K + q) * d.nblk, d.nblk);
        if (lane != 0) continue;
        st->cmode = 0;
        if (!isfinite(RZ)) st->status = SPK_DIVERGED_NANORINF;
        else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
        else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
        else if (st->iter >= st->maxit) { st->status = SPK_DIVERGED_ITS; st->rho = RZ; }
        else st->rho = RZ;
    }
    publish_mask(d);
}

// Restart the columns in mask from their true residual (already in R).
static __global__ void k_m_restart(MultiDesc d, int32_t mask)
{
    const int q = threadIdx.x;
    if (q < d.K && ((mask >> q) & 1)) {
        d.st[q].status = SPK_RUNNING;
        d.st[q].cmode = 0;
    }
}

// ------------------------------------------------------------------ iteration
// A: Q = A P, per-column per-block p.q (columns that stopped are multiplied
// too: the matrix is read once either way; their partials are ignored).
template <class CI, int K>
__global__ __launch_bounds__(kBlock) void k_m_spmm_pq(MultiDesc d)
{
    __shared__ double sh[(kBlock / kWave) * K];
    int j;
    const int l = multi_block(d, j);
    if (l < 0) return;
    if (d.ctl->mask == 0) return;
    double pq = 0.0;
    multi_items<CI, K>(d, l, j, d.P, [&](int64_t e, int, double y) {
        d.Q[e] = y;
        pq = fma(y, d.P[e], pq);
    });
    block_partials_flat<K>(pq, sh, d.partials + (size_t)kPartPq * K * d.nblk, d.nblk, j);
}

// F_A: eta = p.q and alpha per running column; eta <= 0 stops the column.
static __global__ __launch_bounds__(kBlock) void k_m_fin_pq(MultiDesc d)
{
    if (d.ctl->mask == 0) return;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int q = w; q < d.K; q += kBlock / kWave) {
        SysState *st = d.st + q;
        if (st->status != SPK_RUNNING) continue;
        const double eta = wave_reduce_col(d.partials + ((size_t)kPartPq * d.K + q) * d.nblk, d.nblk);
        if (lane != 0) continue;
        st->eta = eta;
        st->cmode = 0;
        if (!isfinite(eta)) st->status = SPK_DIVERGED_NANORINF;
        else if (eta <= 0.0) st->status = SPK_DIVERGED_INDEFINITE_MAT;
        else st->alpha = st->rho / eta;
    }
    publish_mask(d);
}

// B: R -= alpha Q, Z = D^-1 R for the running columns, per-block r.z, r.r.
template <int K>
__global__ __launch_bounds__(kBlock) void k_m_update(MultiDesc d)
{
    __shared__ double sh[(kBlock / kWave) * K];
    int j;
    if (multi_block(d, j) < 0) return;
    const int mask = d.ctl->mask;
    if (mask == 0) return;
    const int q = threadIdx.x % K;
    const bool run = (mask >> q) & 1;
    const double nal = run ? -d.st[q].alpha : 0.0;
    double rz = 0.0, rr = 0.0;
    if (run)
        flat_walk<K>(d, j, [&](int64_t e, int i) {
            const double ri = fma(nal, d.Q[e], d.Rv[e]);
            const double zi = d.dinv[i] * ri;
            d.Rv[e] = ri;
            d.Z[e] = zi;
            rz = fma(ri, zi, rz);
            rr = fma(ri, ri, rr);
        });
    block_partials_flat<K>(rz, sh, d.partials + (size_t)kPartRz * K * d.nblk, d.nblk, j);
    block_partials_flat<K>(rr, sh, d.partials + (size_t)kPartRr * K * d.nblk, d.nblk, j);
}

// F_B: per running column: iteration count, convergence, breakdowns, beta;
// cmode 2 (x and p updates), 1 (last x update), as in the single solve.
static __global__ __launch_bounds__(kBlock) void k_m_fin_update(MultiDesc d)
{
    const int mask0 = d.ctl->mask;
    if (mask0 == 0) {  // every column has stopped: the p/x kernel does nothing
        __syncthreads();
        if (threadIdx.x == 0) d.ctl->pad_ = 0;
        return;
    }
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int q = w; q < d.K; q += kBlock / kWave) {
        if (!((mask0 >> q) & 1)) continue;
        SysState *st = d.st + q;
        const double RZ = wave_reduce_col(d.partials + ((size_t)kPartRz * d.K + q) * d.nblk, d.nblk);
        const double RR = wave_reduce_col(d.partials + ((size_t)kPartRr * d.K + q) * d.nblk, d.nblk);
        if (lane != 0) continue;
        const int k = ++st->iter;
        const double rn = sqrt(RR);
        st->rnorm = rn;
        st->cmode = 1;
        if (!isfinite(rn)) st->status = SPK_DIVERGED_NANORINF;
        else if (rn <= st->thresh)
            st->status = rn <= st->rtol * st->bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        else if (k >= st->maxit) st->status = SPK_DIVERGED_ITS;
        else if (!isfinite(RZ)) st->status = SPK_DIVERGED_NANORINF;
        else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
        else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
        else { st->beta = RZ / st->rho; st->rho = RZ; st->cmode = 2; }
    }
    __syncthreads();
    // the p/x kernel needs the pre-update mask (columns stopping now still
    // take their last x update): keep it in pad_
    if (threadIdx.x == 0) d.ctl->pad_ = mask0;
    publish_mask(d);
}

// C: per column, cmode 2: x += alpha p, p = z + beta p; cmode 1: x += alpha p.
template <int K>
__global__ __launch_bounds__(kBlock) void k_m_px(MultiDesc d)
{
    int j;
    if (multi_block(d, j) < 0) return;
    const int mask0 = d.ctl->pad_;
    if (mask0 == 0) return;
    const int q = threadIdx.x % K;
    const int cm = ((mask0 >> q) & 1) ? d.st[q].cmode : 0;
    if (cm == 0) return;  // no barrier follows
    const double al = d.st[q].alpha, be = d.st[q].beta;
    flat_walk<K>(d, j, [&](int64_t e, int) {
        const double pi = d.P[e];
        d.X[e] = fma(al, pi, d.X[e]);
        if (cm == 2) d.P[e] = fma(be, pi, d.Z[e]);
    });
}

// Per-column state for a new solve (FP64, one thread per column), all
// columns running until the setup kernels decide otherwise.
static __global__ void k_m_init(MultiDesc d, double rtol, double atol, int maxit)
{
    const int q = threadIdx.x;
    if (q < d.K) {
        SysState *st = d.st + q;
        *st = SysState{};
        st->status = SPK_RUNNING;
        st->phase = kPhaseInner;
        st->maxit = maxit;
        st->rtol = rtol;
        st->atol = atol;
    }
    if (q == 0) {
        d.ctl->mask = (1 << d.K) - 1;
        d.ctl->pad_ = 0;
    }
}

// x = 0 for the columns in mask (right-hand sides that are zero).
template <int K>
__global__ void k_m_zero_cols(MultiDesc d, int32_t mask)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += gridDim.x * blockDim.x)
#pragma unroll
        for (int q = 0; q < K; ++q)
            if ((mask >> q) & 1) d.X[(size_t)i * K + q] = 0.0;
}

// The running-column mask to pinned host memory (one thread's store).
static __global__ void k_m_publish(const MultiCtl *ctl, int32_t *host)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) host[0] = ctl->mask;
}

}  // namespace spk
