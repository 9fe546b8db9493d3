// Single-reduction Jacobi-PCG (Chronopoulos & Gear): the inner products of
// an iteration, r.u, r.r and (A u).u, are all formed after the same vector
// pass, so an iteration is two kernels instead of four (Sec. 4 Challenge A1:
// every synchronisation point drains the GPU's queue):
//   V_i  every block sums the partials of iteration i (same fixed order, so
//        all blocks take the same decision), block 0 records the decision;
//        then p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//        u = D^-1 r, partials of r.u and r.r
//   A_i  w = A u, partials of w.u
// Scalars of iteration i live in slot i & 1 and partials in set i & 1, so a
// kernel never reads what another block of the same kernel writes.  The
// iteration index i = base + m: m is the kernel's position in a captured
// batch, base (device) advances by the batch length after each batch.
#pragma once

#include "krylov.hpp"

namespace spk {

struct SrScal {
    double gamma[2];  // r.u of iteration i in slot i & 1
    double alpha[2];  // alpha of iteration i; 0 marks "no previous step"
    int32_t base;
    int32_t pad_;
};

struct SrDesc {
    SysDesc d;        // r, z (= u), q (= w), p, x, dinv, st, hist, matrix
    double *s;        // s = A p
    double *part;     // [2 sets][gamma, rr, delta][nblk]
    SrScal *sc;
};

enum { kSrGamma = 0, kSrRr = 1, kSrDelta = 2 };

__device__ __forceinline__ double *sr_part(const SrDesc &a, int set, int t)
{
    return a.part + (size_t)(set * 3 + t) * a.d.nblk;
}

__device__ __forceinline__ bool sr_locate(const SrDesc &a, int &j)
{
    if ((int)blockIdx.x >= a.d.nblk) return false;
    j = xcd_remap(blockIdx.x, a.d.nblk);
    return true;
}

// u = D^-1 r, partials of r.u and r.r into `set` (start and restarts).
static __global__ __launch_bounds__(kBlock) void k_sr_setup(SrDesc a, int set)
{
    __shared__ double red[kBlock / kWave];
    int j;
    if (!sr_locate(a, j)) return;
    const SysDesc &d = a.d;
    if (d.st->status != SPK_RUNNING) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double *__restrict__ r = d.r;
    const double *__restrict__ dinv = d.dinv;
    double *__restrict__ u = d.z;
    double ru = 0.0, rr = 0.0;
    rows_unrolled(rb, re, [&](int i) {
        const double ri = r[i];
        const double ui = dinv[i] * ri;
        u[i] = ui;
        ru = fma(ri, ui, ru);
        rr = fma(ri, ri, rr);
    });
    ru = block_sum(ru, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        sr_part(a, set, kSrGamma)[j] = ru;
        sr_part(a, set, kSrRr)[j] = rr;
    }
}

// A_i, SELL: w = A u, partials of w.u into set (i + 1) & 1.
template <class CI, int U>
__global__ __launch_bounds__(kBlock) void k_sr_spmv_sell(SrDesc a, int m)
{
    __shared__ double red[kBlock / kWave];
    int j;
    if (!sr_locate(a, j)) return;
    const SysDesc &d = a.d;
    const Gate g = load_gate(d.st);
    const int i = a.sc->base + m;
    const double *__restrict__ u = d.z;
    double *__restrict__ w = d.q;
    const SellView sv{d.sell_ptr, d.sell_col, d.sell_len, d.sell_plain, d.sell_len16, d.sell_perm, d.sell_mask};
    const bool run = gate_ok(g, kGateInner64);
    double wu = 0.0;
    sell_slices<double, CI, U>(d.n, sell_first((int)blockIdx.x), d.nblk * (kBlock / kWave), sv, d.sell_val, u,
                               [&] { return run; }, [&](int r, double y) {
                                   w[r] = y;
                                   wu = fma(y, u[r], wu);
                               });
    if (!run) return;
    wu = block_sum(wu, red);
    if (threadIdx.x == 0) sr_part(a, (i + 1) & 1, kSrDelta)[j] = wu;
}

// A_i, stream tiles.
static __global__ __launch_bounds__(kBlock) void k_sr_spmv_stream(SrDesc a, int m)
{
    __shared__ TileLds<double> sm;
    __shared__ double red[kBlock / kWave];
    int j;
    if (!sr_locate(a, j)) return;
    const SysDesc &d = a.d;
    if (!gate_open(d.st, kGateInner64)) return;
    const int i = a.sc->base + m;
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const double *__restrict__ u = d.z;
    double *__restrict__ w = d.q;
    double wu = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * d.R;
        const int r1 = min(r0 + d.R, d.n);
        stream_tile<double>(r0, r1, d.rowptr, d.col, d.val, u, sm, [&](int r, double y) {
            w[r] = y;
            wu = fma(y, u[r], wu);
        });
    }
    wu = block_sum(wu, red);
    if (threadIdx.x == 0) sr_part(a, (i + 1) & 1, kSrDelta)[j] = wu;
}

// A_i, other families: w was written by the standalone SpMV; partials of w.u.
static __global__ __launch_bounds__(kBlock) void k_sr_dot(SrDesc a, int m)
{
    __shared__ double red[kBlock / kWave];
    int j;
    if (!sr_locate(a, j)) return;
    const SysDesc &d = a.d;
    if (!gate_open(d.st, kGateInner64)) return;
    const int i = a.sc->base + m;
    int rb, re;
    row_range(d, j, rb, re);
    const double *__restrict__ u = d.z;
    const double *__restrict__ w = d.q;
    double wu = 0.0;
    rows_unrolled(rb, re, [&](int r) { wu = fma(w[r], u[r], wu); });
    wu = block_sum(wu, red);
    if (threadIdx.x == 0) sr_part(a, (i + 1) & 1, kSrDelta)[j] = wu;
}

// V_i.
static __global__ __launch_bounds__(kBlock) void k_sr_update(SrDesc a, int m)
{
    __shared__ double red[kBlock / kWave];
    int j;
    if (!sr_locate(a, j)) return;
    const SysDesc &d = a.d;
    SysState *st = d.st;
    const Gate g = load_gate(st);
    if (!gate_ok(g, kGateInner64)) return;
    const int i = a.sc->base + m;
    const int cur = i & 1, prv = cur ^ 1;
    const double gamma_prev = a.sc->gamma[prv], alpha_prev = a.sc->alpha[prv];
    const double thresh = st->thresh, rtol = st->rtol, bnorm = st->bnorm;
    const int maxit = st->maxit, hist_len = st->hist_len;
    double gamma, rr, delta;
    reduce_partials3(sr_part(a, cur, kSrGamma), sr_part(a, cur, kSrRr), sr_part(a, cur, kSrDelta), d.nblk, red,
                     gamma, rr, delta);
    // the decision of iteration i, identical in every block
    const double rn = sqrt(rr);
    int stop = 0;
    double alpha = 0.0, beta = 0.0;
    const bool first = !(alpha_prev > 0.0);
    if (!finite(rn)) stop = SPK_DIVERGED_NANORINF;
    else if (rn <= thresh) stop = rn <= rtol * bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
    else if (i >= maxit) stop = SPK_DIVERGED_ITS;
    else if (!finite(gamma)) stop = SPK_DIVERGED_NANORINF;
    else if (gamma < 0.0) stop = SPK_DIVERGED_INDEFINITE_PC;
    else if (gamma == 0.0) stop = SPK_DIVERGED_BREAKDOWN;
    else {
        const double den = first ? delta : delta - (gamma / gamma_prev) * gamma / alpha_prev;
        if (!finite(den)) stop = SPK_DIVERGED_NANORINF;
        else if (den <= 0.0) stop = SPK_DIVERGED_INDEFINITE_MAT;
        else {
            beta = first ? 0.0 : gamma / gamma_prev;
            alpha = gamma / den;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = i;
        st->rnorm = rn;
        if (d.hist && i > 0 && i < hist_len) d.hist[i] = rn;
        if (stop) st->status = stop;
        else {
            a.sc->gamma[cur] = gamma;
            a.sc->alpha[cur] = alpha;
        }
    }
    if (stop) return;
    int rb, re;
    row_range(d, j, rb, re);
    double *__restrict__ p = d.p;
    double *__restrict__ s = a.s;
    double *__restrict__ x = d.x;
    double *__restrict__ r = d.r;
    double *__restrict__ u = d.z;
    const double *__restrict__ w = d.q;
    const double *__restrict__ dinv = d.dinv;
    double ru = 0.0, rs = 0.0;
    rows_unrolled(rb, re, [&](int k) {
        const double uk = u[k], wk = w[k];
        const double pk = first ? uk : fma(beta, p[k], uk);
        const double sk = first ? wk : fma(beta, s[k], wk);
        p[k] = pk;
        s[k] = sk;
        x[k] = fma(alpha, pk, x[k]);
        const double rk = fma(-alpha, sk, r[k]);
        r[k] = rk;
        const double un = dinv[k] * rk;
        u[k] = un;
        ru = fma(rk, un, ru);
        rs = fma(rk, rk, rs);
    });
    ru = block_sum(ru, red);
    rs = block_sum(rs, red);
    if (threadIdx.x == 0) {
        sr_part(a, cur ^ 1, kSrGamma)[j] = ru;
        sr_part(a, cur ^ 1, kSrRr)[j] = rs;
    }
}

// base += K after a batch of K iterations.
static __global__ void k_sr_advance(SrScal *sc, int K)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->base += K;
}

// Start (or restart) at iteration b: no previous step.
static __global__ void k_sr_rebase(SrScal *sc, int b)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->base = b;
        sc->alpha[(b + 1) & 1] = 0.0;  // slot (b - 1) & 1
    }
}

}  // namespace spk
