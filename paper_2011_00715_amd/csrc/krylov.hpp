// Batched Jacobi-PCG kernels.  Every kernel serves a table of systems: block b
// belongs to system s (binary search over blk_start), and the system's
// logical block j (XCD-aware) owns the same contiguous run of tiles/rows in
// every kernel.  Per-system reductions are per-block partials reduced by the
// system's last-arriving block in a fixed order, so the result of a system
// does not depend on which other systems share the launch.
//
// One PCG iteration (textbook preconditioned CG; the paper names CG in
// Sec. 5.5 and the Jacobi smoother in Sec. 5.3) is three kernels:
//   A  q = A p and p.q            -> last block: eta, alpha = rho / eta
//   B  r -= alpha q, z = D^-1 r,  r.z and r.r (one pass, Sec. 4 Response F3:
//      several inner products fused)  -> last block: convergence test, beta
//   C  x += alpha p, p = z + beta p
// The scalars live on the device, and every kernel becomes a no-op once the
// system has stopped, so a captured graph of many iterations can be replayed
// without host round trips (Challenge A1: kernel fusion, graphs, pipelining).
#pragma once

#include "spmv.hpp"

namespace spk {

struct Batch {
    const SysDesc *sys;
    const int32_t *blk_start;  // nsys + 1 entries
    int nsys;
};

template <class V> struct Vecs;
template <> struct Vecs<double> {
    __device__ static const double *val(const SysDesc &d) { return d.val; }
    __device__ static const double *dinv(const SysDesc &d) { return d.dinv; }
    __device__ static double *r(const SysDesc &d) { return d.r; }
    __device__ static double *z(const SysDesc &d) { return d.z; }
    __device__ static double *p(const SysDesc &d) { return d.p; }
    __device__ static double *q(const SysDesc &d) { return d.q; }
    __device__ static double *x(const SysDesc &d) { return d.x; }
    static constexpr int gate = kGateInner64;
};
template <> struct Vecs<float> {
    __device__ static const float *val(const SysDesc &d) { return d.val32; }
    __device__ static const float *dinv(const SysDesc &d) { return d.dinv32; }
    __device__ static float *r(const SysDesc &d) { return d.r32; }
    __device__ static float *z(const SysDesc &d) { return d.z32; }
    __device__ static float *p(const SysDesc &d) { return d.p32; }
    __device__ static float *q(const SysDesc &d) { return d.q32; }
    __device__ static float *x(const SysDesc &d) { return d.d32; }
    static constexpr int gate = kGateInner32;
};

// Block -> (system, logical block).  False for padding blocks.
__device__ __forceinline__ bool locate(const Batch &a, int &s, int &j)
{
    s = find_sys(a.blk_start, a.nsys, blockIdx.x);
    const int l = blockIdx.x - a.blk_start[s];
    const int nb = a.sys[s].nblk;
    if (l >= nb) return false;
    j = xcd_remap(l, nb);
    return true;
}

__device__ __forceinline__ void row_range(const SysDesc &d, int j, int &rb, int &re)
{
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    rb = t0 * d.R;
    re = min(t1 * d.R, d.n);
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// ------------------------------------------------------------------ state init
// One thread per system: reset the scalars for a new solve.
static __global__ void k_state_init(SysState *st, double rtol, double atol, int maxit, int mixed,
                             double inner_rtol, int inner_maxit, int max_outer, int hist_len)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->status = SPK_RUNNING;
    st->phase = mixed ? kPhaseResid : kPhaseInner;
    st->iter = 0;
    st->inner_iter = 0;
    st->outer = 0;
    st->x_pending = 0;
    st->maxit = maxit;
    st->inner_maxit = inner_maxit;
    st->max_outer = max_outer;
    st->stagnant = 0;
    st->mixed = mixed;
    st->hist_len = hist_len;
    for (int i = 0; i < kNumCnt; ++i) st->counter[i] = 0;
    st->rho = st->alpha = st->beta = st->eta = 0.0;
    st->rnorm = st->rnorm0 = st->bnorm = st->thresh = 0.0;
    st->rtol = rtol;
    st->atol = atol;
    st->inner_rtol = inner_rtol;
    st->inner_thresh = 0.0;
    st->s = st->s_prev = 0.0;
    st->rnorm_true = 0.0;
}

// Restart from the true residual already in r (FP64 solves).
static __global__ void k_state_restart(SysState *st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->status = SPK_RUNNING;
    st->phase = kPhaseInner;
    st->x_pending = 0;
}

// ------------------------------------------------------------------ residual
// Purpose of a residual launch.
enum { kResSetup = 0, kResTrue = 1, kResOuter = 2 };

__device__ __forceinline__ void resid_finish_scalars(const SysDesc &d, double rr, double bb,
                                                     int purpose)
{
    SysState *st = d.st;
    const double rn = sqrt(rr);
    if (purpose == kResTrue) {
        st->rnorm_true = rn;
        return;
    }
    const double bn = sqrt(bb);
    st->bnorm = bn;
    st->thresh = fmax(st->rtol * bn, st->atol);
    if (purpose == kResSetup) {
        st->rnorm = rn;
        st->rnorm0 = rn;
        if (d.hist && st->hist_len > 0) d.hist[0] = rn;
        if (bn == 0.0) { st->status = SPK_CONVERGED_ATOL; return; }
        if (!finite(rn) || !finite(bn)) { st->status = SPK_DIVERGED_NANORINF; return; }
        if (rn <= st->thresh) st->status = rn <= st->rtol * bn ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        return;
    }
    // kResOuter: one FP64 refinement residual of a mixed solve (after the
    // update x += s d when coming from kPhaseUpdate)
    if (st->phase == kPhaseUpdate) ++st->outer;
    const int k = st->outer;
    if (k == 0) st->rnorm0 = rn;
    if (d.hist && k < st->hist_len) d.hist[k] = rn;
    st->rnorm = rn;
    st->s = rn;
    if (bn == 0.0) { st->status = SPK_CONVERGED_ATOL; return; }
    if (!finite(rn) || !finite(bn)) { st->status = SPK_DIVERGED_NANORINF; return; }
    if (rn <= st->thresh) {
        st->status = rn <= st->rtol * bn ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        return;
    }
    if (k >= st->max_outer || st->iter >= st->maxit) { st->status = SPK_DIVERGED_ITS; return; }
    if (k > 0 && rn > 0.5 * st->s_prev) {
        if (++st->stagnant >= 2) { st->status = SPK_DIVERGED_STAGNATION; return; }
    } else {
        st->stagnant = 0;
    }
    st->s_prev = rn;
    st->phase = kPhaseSetup;
}

// r = b - A x in FP64 with the stream tile kernel, r.r and b.b fused.
template <int kGate>
__global__ __launch_bounds__(kBlock) void k_resid_stream(Batch a, int purpose)
{
    __shared__ TileLds<double> sm;
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    if (kGate != kGateNone && !gate_open(d.st, kGate)) return;
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const double *b = d.b;
    double *r = d.r;
    double rr = 0.0, bb = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * d.R;
        const int r1 = min(r0 + d.R, d.n);
        stream_tile<double>(r0, r1, d.rowptr, d.col, d.val, d.x, sm, [&](int i, double y) {
            const double bi = b[i];
            const double ri = bi - y;
            r[i] = ri;
            rr = fma(ri, ri, rr);
            bb = fma(bi, bi, bb);
        });
    }
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRr * d.nblk + j] = rr;
        d.partials[kPartBb * d.nblk + j] = bb;
    }
    if (last_block_arrive(&d.st->counter[kCntRes], d.nblk)) {
        const double RR = reduce_partials(d.partials + kPartRr * d.nblk, d.nblk, red);
        const double BB = reduce_partials(d.partials + kPartBb * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) resid_finish_scalars(d, RR, BB, purpose);
    }
}

// r = b - y where y = A x was written into r by a standalone SpMV kernel.
template <int kGate>
__global__ __launch_bounds__(kBlock) void k_resid_finish(Batch a, int purpose)
{
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    if (kGate != kGateNone && !gate_open(d.st, kGate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    double rr = 0.0, bb = 0.0;
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
        const double bi = d.b[i];
        const double ri = bi - d.r[i];
        d.r[i] = ri;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    }
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRr * d.nblk + j] = rr;
        d.partials[kPartBb * d.nblk + j] = bb;
    }
    if (last_block_arrive(&d.st->counter[kCntRes], d.nblk)) {
        const double RR = reduce_partials(d.partials + kPartRr * d.nblk, d.nblk, red);
        const double BB = reduce_partials(d.partials + kPartBb * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) resid_finish_scalars(d, RR, BB, purpose);
    }
}

// ------------------------------------------------------------------ setup
// FP64 start / restart from the residual in r: z = D^-1 r, p = z, rho = r.z.
static __global__ __launch_bounds__(kBlock) void k_setup64(Batch a)
{
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    if (d.st->status != SPK_RUNNING) return;
    int rb, re;
    row_range(d, j, rb, re);
    double rz = 0.0;
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
        const double ri = d.r[i];
        const double zi = d.dinv[i] * ri;
        d.z[i] = zi;
        d.p[i] = zi;
        rz = fma(ri, zi, rz);
    }
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) d.partials[kPartRz * d.nblk + j] = rz;
    if (last_block_arrive(&d.st->counter[kCntSet], d.nblk)) {
        const double RZ = reduce_partials(d.partials + kPartRz * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) {
            SysState *st = d.st;
            if (!finite(RZ)) st->status = SPK_DIVERGED_NANORINF;
            else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
            else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
            else if (st->iter >= st->maxit) { st->status = SPK_DIVERGED_ITS; st->rho = RZ; }
            else st->rho = RZ;
        }
    }
}

// Mixed: start an FP32 inner solve on r32 = r / s (unit norm):
// z32 = dinv32 r32, p32 = z32, d32 = 0, rho = r32.z32.
static __global__ __launch_bounds__(kBlock) void k_setup32(Batch a)
{
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    SysState *st = d.st;
    if (!(st->status == SPK_RUNNING && st->mixed == 1 && st->phase == kPhaseSetup)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double inv = 1.0 / st->s;
    float rz = 0.f, rr = 0.f;
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
        const float ri = (float)(d.r[i] * inv);
        const float zi = d.dinv32[i] * ri;
        d.r32[i] = ri;
        d.z32[i] = zi;
        d.p32[i] = zi;
        d.d32[i] = 0.f;
        rz = fmaf(ri, zi, rz);
        rr = fmaf(ri, ri, rr);
    }
    const double RZb = block_sum((double)rz, red);
    const double RRb = block_sum((double)rr, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRz * d.nblk + j] = RZb;
        d.partials[kPartRr * d.nblk + j] = RRb;
    }
    if (last_block_arrive(&st->counter[kCntSet], d.nblk)) {
        const double RZ = reduce_partials(d.partials + kPartRz * d.nblk, d.nblk, red);
        const double RR = reduce_partials(d.partials + kPartRr * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) {
            st->inner_iter = 0;
            st->inner_thresh = st->inner_rtol * sqrt(RR);
            if (!finite(RZ) || !finite(RR)) st->status = SPK_DIVERGED_NANORINF;
            else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
            else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
            else { st->rho = RZ; st->phase = kPhaseInner; }
        }
    }
}

// Mixed: x += s d (FP64 update from the FP32 correction).
static __global__ __launch_bounds__(kBlock) void k_update_x(Batch a)
{
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    const SysState *st = d.st;
    if (!(st->status == SPK_RUNNING && st->mixed == 1 && st->phase == kPhaseUpdate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double sc = st->s;
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock)
        d.x[i] = fma(sc, (double)d.d32[i], d.x[i]);
}

// ------------------------------------------------------------------ iteration
__device__ __forceinline__ void pq_finish_scalars(SysState *st, double eta)
{
    st->eta = eta;
    if (!finite(eta)) st->status = SPK_DIVERGED_NANORINF;
    else if (eta <= 0.0) {
        if (st->mixed) { st->phase = kPhaseUpdate; }  // inner breakdown: refine
        else st->status = SPK_DIVERGED_INDEFINITE_MAT;
    } else st->alpha = st->rho / eta;
}

// A: q = A p with the stream tile kernel, p.q fused into the row epilogue.
template <class V>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv_stream(Batch a)
{
    __shared__ TileLds<V> sm;
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    if (!gate_open(d.st, Vecs<V>::gate)) return;
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const V *p = Vecs<V>::p(d);
    V *q = Vecs<V>::q(d);
    V acc = V(0);
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * d.R;
        const int r1 = min(r0 + d.R, d.n);
        stream_tile<V>(r0, r1, d.rowptr, d.col, Vecs<V>::val(d), p, sm, [&](int i, V y) {
            q[i] = y;
            acc = fma(y, p[i], acc);
        });
    }
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
    if (last_block_arrive(&d.st->counter[kCntPq], d.nblk)) {
        const double eta = reduce_partials(d.partials + kPartPq * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) pq_finish_scalars(d.st, eta);
    }
}

// A (other SpMV kernels): q already holds A p; form p.q.
template <class V>
__global__ __launch_bounds__(kBlock) void k_pcg_pq(Batch a)
{
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    if (!gate_open(d.st, Vecs<V>::gate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const V *p = Vecs<V>::p(d);
    const V *q = Vecs<V>::q(d);
    V acc = V(0);
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) acc = fma(q[i], p[i], acc);
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
    if (last_block_arrive(&d.st->counter[kCntPq], d.nblk)) {
        const double eta = reduce_partials(d.partials + kPartPq * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) pq_finish_scalars(d.st, eta);
    }
}

// B: r -= alpha q, z = D^-1 r, r.z and r.r in one pass.
template <class V>
__global__ __launch_bounds__(kBlock) void k_pcg_update(Batch a)
{
    __shared__ double red[kBlock / kWave];
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    SysState *st = d.st;
    if (!gate_open(st, Vecs<V>::gate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const V nalpha = (V)(-st->alpha);
    V *r = Vecs<V>::r(d);
    V *z = Vecs<V>::z(d);
    const V *q = Vecs<V>::q(d);
    const V *dinv = Vecs<V>::dinv(d);
    V rz = V(0), rr = V(0);
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
        const V ri = fma(nalpha, q[i], r[i]);
        const V zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
    }
    const double RZb = block_sum((double)rz, red);
    const double RRb = block_sum((double)rr, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRz * d.nblk + j] = RZb;
        d.partials[kPartRr * d.nblk + j] = RRb;
    }
    if (last_block_arrive(&st->counter[kCntUpd], d.nblk)) {
        const double RZ = reduce_partials(d.partials + kPartRz * d.nblk, d.nblk, red);
        const double RR = reduce_partials(d.partials + kPartRr * d.nblk, d.nblk, red);
        if (threadIdx.x == 0) {
            const int k = ++st->iter;
            const double rn = sqrt(RR);
            st->x_pending = 1;  // cleared below if the iteration continues
            if (!st->mixed) {
                st->rnorm = rn;
                if (d.hist && k < st->hist_len) d.hist[k] = rn;
                if (!finite(rn)) st->status = SPK_DIVERGED_NANORINF;
                else if (rn <= st->thresh)
                    st->status = rn <= st->rtol * st->bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
                else if (k >= st->maxit) st->status = SPK_DIVERGED_ITS;
                else if (!finite(RZ)) st->status = SPK_DIVERGED_NANORINF;
                else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
                else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
                else { st->beta = RZ / st->rho; st->rho = RZ; st->x_pending = 0; }
            } else {
                const int ki = ++st->inner_iter;
                if (!finite(rn) || !finite(RZ)) st->status = SPK_DIVERGED_NANORINF;
                else if (rn <= st->inner_thresh || ki >= st->inner_maxit || k >= st->maxit || RZ <= 0.0)
                    st->phase = kPhaseUpdate;
                else { st->beta = RZ / st->rho; st->rho = RZ; st->x_pending = 0; }
            }
        }
    }
}

// C: x += alpha p (d for mixed), and p = z + beta p while iterating.
template <class V>
__global__ __launch_bounds__(kBlock) void k_pcg_px(Batch a)
{
    int s, j;
    if (!locate(a, s, j)) return;
    const SysDesc &d = a.sys[s];
    SysState *st = d.st;
    const bool iterating = gate_open(st, Vecs<V>::gate);
    const bool pending = st->x_pending && st->mixed == (Vecs<V>::gate == kGateInner32 ? 1 : 0);
    if (!iterating && !pending) return;
    int rb, re;
    row_range(d, j, rb, re);
    const V alpha = (V)st->alpha;
    const V beta = (V)st->beta;
    V *x = Vecs<V>::x(d);
    V *p = Vecs<V>::p(d);
    const V *z = Vecs<V>::z(d);
    if (iterating && !pending) {
        for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
            const V pi = p[i];
            x[i] = fma(alpha, pi, x[i]);
            p[i] = fma(beta, pi, z[i]);
        }
    } else {
        for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) x[i] = fma(alpha, p[i], x[i]);
        if (last_block_arrive(&st->counter[kCntPx], d.nblk))
            if (threadIdx.x == 0) st->x_pending = 0;
    }
}

}  // namespace spk
