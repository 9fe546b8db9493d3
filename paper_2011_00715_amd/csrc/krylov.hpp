// Batched Jacobi-PCG kernels.  Every kernel serves a table of systems: block b
// belongs to system s (binary search over blk_start), and the system's
// logical block j (XCD-aware) owns the same contiguous run of tiles/rows in
// every kernel.  Reductions write one partial per block; a finalize kernel
// with one block per system then sums the partials in a fixed order and
// updates the system's scalars.  No kernel synchronises across its own
// blocks (a device-scope fence writes back and invalidates the XCD's L2), and
// there are no floating-point atomics, so a system's bits depend only on the
// system itself, never on the rest of the batch.
//
// One PCG iteration (textbook preconditioned CG; the paper names CG in
// Sec. 5.5 and the Jacobi smoother in Sec. 5.3), three kernels:
//   A   q = A p, per-block p.q
//   B   eta = p.q and alpha = rho / eta (each block sums A's partials in the
//       same fixed order), r -= alpha q, z = D^-1 r, per-block r.z and r.r
//       (one pass; Sec. 4 Response F3: fused inner products); block 0 also
//       records the scalars it used (state snap_*)
//   C   every block sums B's r.z and r.r partials in the same fixed order
//       and takes the same decision from the recorded scalars (convergence
//       and breakdown tests, beta); block 0 stores it; then x += alpha p and,
//       while iterating, p = z + beta p
// Systems with the SELL product on the persistent grid fuse C into the next
// iteration's A (kernel F, see k_pcg_fused_sell): two kernels per iteration.
// Scalars live on the device and every kernel is a no-op once its system has
// stopped, so a captured graph of many iterations replays without host round
// trips (Challenge A1: fusion, graphs, pipelining).
#pragma once

#include "spmv.hpp"

namespace spk {

// The systems of one launch: `Batch` is a device table (the batched server);
// `One` carries a single system's descriptor by value in the kernel
// arguments, so that every field is a uniform scalar and no block pays
// dependent global loads to find its system.
struct Batch {
    const SysDesc *sys;
    const int32_t *blk_start;  // nsys + 1 entries
    int nsys;
};
struct One {
    SysDesc d;
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
    __device__ static double *p2(const SysDesc &d) { return d.p2; }
    __device__ static bool present(const SysDesc &) { return true; }
    static constexpr int gate = kGateInner64;
    static constexpr int mixed = 0;
};
template <> struct Vecs<float> {
    __device__ static const float *val(const SysDesc &d) { return d.val32; }
    __device__ static const float *dinv(const SysDesc &d) { return d.dinv32; }
    __device__ static float *r(const SysDesc &d) { return d.r32; }
    __device__ static float *z(const SysDesc &d) { return d.z32; }
    __device__ static float *p(const SysDesc &d) { return d.p32; }
    __device__ static float *q(const SysDesc &d) { return d.q32; }
    __device__ static float *x(const SysDesc &d) { return d.d32; }
    __device__ static float *p2(const SysDesc &d) { return d.p2_32; }
    // FP64 systems of a mixed batch have no FP32 vectors
    __device__ static bool present(const SysDesc &d) { return d.r32 != nullptr; }
    static constexpr int gate = kGateInner32;
    static constexpr int mixed = 1;
};

// Block -> (system, logical block); the descriptor is copied into registers
// (stores through the system's vectors cannot alias it).  False for padding.
__device__ __forceinline__ bool locate(const Batch &a, int &j, SysDesc &d)
{
    const int s = find_sys(a.blk_start, a.nsys, blockIdx.x);
    const int l = blockIdx.x - a.blk_start[s];
    d = a.sys[s];
    if (l >= d.nblk) return false;
    j = xcd_remap(l, d.nblk);
    return true;
}

__device__ __forceinline__ bool locate(const One &a, int &j, SysDesc &d)
{
    d = a.d;
    if ((int)blockIdx.x >= d.nblk) return false;
    j = xcd_remap(blockIdx.x, d.nblk);
    return true;
}

// Physical block index within its system (the SELL kernels walk slices in
// physical block order).
__device__ __forceinline__ int local_block(const Batch &a)
{
    return (int)blockIdx.x - a.blk_start[find_sys(a.blk_start, a.nsys, blockIdx.x)];
}
__device__ __forceinline__ int local_block(const One &) { return (int)blockIdx.x; }

__device__ __forceinline__ void row_range(const SysDesc &d, int j, int &rb, int &re)
{
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    rb = t0 * d.R;
    re = min(t1 * d.R, d.n);
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// Loop over [rb, re) with 4 independent rows per lane in flight.
template <class F>
__device__ __forceinline__ void rows_unrolled(int rb, int re, F &&f)
{
    constexpr int U = 4;
    for (int i0 = rb + (int)threadIdx.x; i0 < re; i0 += kBlock * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            if (i < re) f(i);
        }
    }
}

// Like rows_unrolled, but the loads of the first chunk are issued before
// `mid()` runs, so that the latency of mid's own loads (state, partial sums)
// overlaps them.  mid runs once in every thread (it may hold barriers) and
// returns false to stop before anything is stored.
template <class L, class Mid, class F>
__device__ __forceinline__ void rows_prefetched(int rb, int re, L &&load, Mid &&mid, F &&use)
{
    constexpr int U = 4;
    using T = decltype(load(0));
    T v[U];
    int i0 = rb + (int)threadIdx.x;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kBlock;
        if (i < re) v[u] = load(i);
    }
    if (!mid()) return;
    while (i0 < re) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            if (i < re) use(i, v[u]);
        }
        i0 += kBlock * U;
        if (i0 >= re) break;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            if (i < re) v[u] = load(i);
        }
    }
}

// reduce_partials in two halves for nblk <= kBlock * 8 (one chunk per
// thread): the loads first, the sum later, in the same order and so with the
// same bits.  Vector loads complete in issue order, so partials loaded after
// a kernel's row loads could only be summed once every row had arrived;
// loaded before them, their sum and the block reduction overlap the rows.
constexpr int kPartChunk = 8;
__device__ __forceinline__ void partials_load(const double *part, int nblk, double v[kPartChunk])
{
#pragma unroll
    for (int u = 0; u < kPartChunk; ++u) {
        const int i = (int)threadIdx.x + u * kBlock;
        v[u] = i < nblk ? part[i] : 0.0;
    }
}
__device__ __forceinline__ double partials_sum(const double v[kPartChunk], double *sh)
{
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kPartChunk; ++u) s += v[u];
    return block_sum(s, sh);
}

template <class V> struct Trio {
    V a, b, c;
};

// ------------------------------------------------------------------ state init
// One thread: reset the scalars of one system for a new solve.
// mixed: 0 FP64, 1 FP32 inner with reliable updates, 2 FP32 inner restarted.
static __global__ void k_state_init(SysState *st, double rtol, double atol, int maxit, int mixed,
                                    double inner_rtol, int inner_maxit, int max_outer,
                                    int hist_len)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->ru = mixed == 1;
    st->fresh_p = 1;
    st->scale = 1.0;
    mixed = mixed != 0;
    st->status = SPK_RUNNING;
    st->phase = mixed ? kPhaseResid : kPhaseInner;
    st->iter = 0;
    st->inner_iter = 0;
    st->outer = 0;
    st->cmode = 0;
    st->maxit = maxit;
    st->inner_maxit = inner_maxit;
    st->max_outer = max_outer;
    st->stagnant = 0;
    st->mixed = mixed;
    st->hist_len = hist_len;
    st->rho = st->alpha = st->beta = st->eta = 0.0;
    st->rnorm = st->rnorm0 = st->bnorm = st->thresh = 0.0;
    st->rtol = rtol;
    st->atol = atol;
    st->inner_rtol = inner_rtol;
    st->inner_thresh = 0.0;
    st->s = st->s_prev = 0.0;
    st->rnorm_true = 0.0;
    // fused iteration: p in buffer 0, nothing to start or decide yet
    st->pbuf = st->snap_pbuf = 0;
    st->snap_mode = 1;
    st->snap_status = SPK_DIVERGED_BREAKDOWN;
}

// Restart from the true residual already in r (FP64 solves).
static __global__ void k_state_restart(SysState *st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->status = SPK_RUNNING;
    st->phase = kPhaseInner;
    st->cmode = 0;
}

// Finalize kernels run one block per system: blockIdx.x = system.
__device__ __forceinline__ bool fin_locate(const Batch &a, SysDesc &d)
{
    if ((int)blockIdx.x >= a.nsys) return false;
    d = a.sys[blockIdx.x];
    return true;
}

__device__ __forceinline__ bool fin_locate(const One &a, SysDesc &d)
{
    d = a.d;
    return blockIdx.x == 0;
}

// ------------------------------------------------------------------ residual
// Purpose of a residual launch.
enum { kResSetup = 0, kResTrue = 1, kResOuter = 2 };

// r = b - A x in FP64 with the stream tile kernel, per-block r.r and b.b.
template <int kGate, class B>
__global__ __launch_bounds__(kBlock) void k_resid_stream(B a)
{
    __shared__ TileLds<double> sm;
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (kGate != kGateNone && !gate_open(d.st, kGate)) return;
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const double *__restrict__ b = d.b;
    double *__restrict__ r = d.r;
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
}

template <class V> __device__ __forceinline__ const V *sell_vals(const SysDesc &d);
template <> __device__ __forceinline__ const double *sell_vals<double>(const SysDesc &d) { return d.sell_val; }
template <> __device__ __forceinline__ const float *sell_vals<float>(const SysDesc &d) { return d.sell_val32; }

// SELL slices of a block: 4 (block) + wave, stride 4 nblk.
__device__ __forceinline__ int sell_first(int l) { return l * (kBlock / kWave) + (int)threadIdx.x / kWave; }

// r = b - A x in FP64 with the SELL-64 layout, per-block r.r and b.b.
template <int kGate, class CI, int U, class B>
__global__ __launch_bounds__(kBlock) void k_resid_sell(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (kGate != kGateNone && !gate_open(d.st, kGate)) return;
    const double *__restrict__ b = d.b;
    double *__restrict__ r = d.r;
    const SellView sv{d.sell_ptr, d.sell_col, d.sell_len, d.sell_plain, d.sell_len16, d.sell_perm, d.sell_mask};
    double rr = 0.0, bb = 0.0;
    sell_slices<double, CI, U>(d.n, sell_first(local_block(a)), d.nblk * (kBlock / kWave), sv,
                               d.sell_val, d.x, [] { return true; }, [&](int i, double y) {
        const double bi = b[i];
        const double ri = bi - y;
        r[i] = ri;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    });
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRr * d.nblk + j] = rr;
        d.partials[kPartBb * d.nblk + j] = bb;
    }
}

// r = b - y where y = A x was written into r by a standalone SpMV kernel.
template <int kGate, class B>
__global__ __launch_bounds__(kBlock) void k_resid_combine(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (kGate != kGateNone && !gate_open(d.st, kGate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double *__restrict__ b = d.b;
    double *__restrict__ r = d.r;
    double rr = 0.0, bb = 0.0;
    rows_unrolled(rb, re, [&](int i) {
        const double bi = b[i];
        const double ri = bi - r[i];
        r[i] = ri;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    });
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRr * d.nblk + j] = rr;
        d.partials[kPartBb * d.nblk + j] = bb;
    }
}

template <int kGate, class B>
__global__ __launch_bounds__(kBlock) void k_fin_resid(B a, int purpose)
{
    __shared__ double red[kBlock / kWave];
    SysDesc d;
    if (!fin_locate(a, d)) return;
    SysState *st = d.st;
    if (kGate != kGateNone && !gate_open(st, kGate)) return;
    double rr, bb;
    reduce_partials2(d.partials + kPartRr * d.nblk, d.partials + kPartBb * d.nblk, d.nblk, red,
                     rr, bb);
    if (threadIdx.x != 0) return;
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
    // restarted refinement solves each correction at unit scale; reliable
    // updates keep the first scale so that p stays valid across refinements
    if (k == 0 || !st->ru) st->scale = rn > 0.0 ? rn : 1.0;
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

// ------------------------------------------------------------------ setup
// FP64 start / restart from the residual in r: z = D^-1 r, p = z, per-block r.z.
template <class B>
__global__ __launch_bounds__(kBlock) void k_setup64(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (d.st->status != SPK_RUNNING) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double *__restrict__ r = d.r;
    const double *__restrict__ dinv = d.dinv;
    double *__restrict__ z = d.z;
    double *__restrict__ p = d.p;
    double rz = 0.0;
    rows_unrolled(rb, re, [&](int i) {
        const double ri = r[i];
        const double zi = dinv[i] * ri;
        z[i] = zi;
        p[i] = zi;
        rz = fma(ri, zi, rz);
    });
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) d.partials[kPartRz * d.nblk + j] = rz;
}

template <class B>
__global__ __launch_bounds__(kBlock) void k_fin_setup64(B a)
{
    __shared__ double red[kBlock / kWave];
    SysDesc d;
    if (!fin_locate(a, d)) return;
    SysState *st = d.st;
    if (st->status != SPK_RUNNING) return;
    const double RZ = reduce_partials(d.partials + kPartRz * d.nblk, d.nblk, red);
    if (threadIdx.x != 0) return;
    if (!finite(RZ)) st->status = SPK_DIVERGED_NANORINF;
    else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
    else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
    else if (st->iter >= st->maxit) { st->status = SPK_DIVERGED_ITS; st->rho = RZ; }
    else st->rho = RZ;
    st->snap_mode = 0;  // the fused iteration starts with p = z
    st->snap_pbuf = st->pbuf;
}

__device__ __forceinline__ bool in_phase(const SysState *st, int phase)
{
    return st->status == SPK_RUNNING && st->mixed == 1 && st->phase == phase;
}

// Mixed: (re)start the FP32 inner iteration on the FP64 residual,
// r32 = r / scale, z32 = dinv32 r32, d32 = 0, per-block r32.z32 and r32.r32.
// p32 = z32 for a restarted refinement (or the first one); with reliable
// updates p32 is kept and p32 = z32 + beta p32 follows once beta is known.
template <class B>
__global__ __launch_bounds__(kBlock) void k_setup32(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    const SysState *st = d.st;
    if (!in_phase(st, kPhaseSetup)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double inv = 1.0 / st->scale;
    const bool fresh = !st->ru || st->fresh_p;
    const double *__restrict__ r = d.r;
    const float *__restrict__ dinv = d.dinv32;
    float *__restrict__ r32 = d.r32;
    float *__restrict__ z32 = d.z32;
    float *__restrict__ p32 = d.p32;
    float *__restrict__ d32 = d.d32;
    float rz = 0.f, rr = 0.f;
    rows_unrolled(rb, re, [&](int i) {
        const float ri = (float)(r[i] * inv);
        const float zi = dinv[i] * ri;
        r32[i] = ri;
        z32[i] = zi;
        if (fresh) p32[i] = zi;
        d32[i] = 0.f;
        rz = fmaf(ri, zi, rz);
        rr = fmaf(ri, ri, rr);
    });
    const double RZb = block_sum((double)rz, red);
    const double RRb = block_sum((double)rr, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRz * d.nblk + j] = RZb;
        d.partials[kPartRr * d.nblk + j] = RRb;
    }
}

template <class B>
__global__ __launch_bounds__(kBlock) void k_fin_setup32(B a)
{
    __shared__ double red[kBlock / kWave];
    SysDesc d;
    if (!fin_locate(a, d)) return;
    SysState *st = d.st;
    if (!in_phase(st, kPhaseSetup)) return;
    double RZ, RR;
    reduce_partials2(d.partials + kPartRz * d.nblk, d.partials + kPartRr * d.nblk, d.nblk, red,
                     RZ, RR);
    if (threadIdx.x != 0) return;
    st->inner_iter = 0;
    // refine again once the inner residual fell by inner_rtol, or as soon as it
    // predicts that the target is met
    st->inner_thresh = fmax(st->inner_rtol * sqrt(RR), st->thresh / st->scale);
    st->cmode = 0;
    if (!finite(RZ) || !finite(RR)) st->status = SPK_DIVERGED_NANORINF;
    else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
    else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
    else {
        st->snap_mode = 0;  // fused iteration: p32 = z32 ...
        if (st->ru && !st->fresh_p) {
            // reliable update: continue the same CG with the true residual
            st->beta = RZ / st->rho;
            st->cmode = 3;      // p32 = z32 + beta p32 before the next SpMV
            st->snap_mode = 3;  // ... or the same inside the fused product
        }
        st->snap_pbuf = st->pbuf;
        st->fresh_p = 0;
        st->rho = RZ;
        st->phase = kPhaseInner;
    }
}

// Mixed: x += s d (FP64 update from the FP32 correction).
template <class B>
__global__ __launch_bounds__(kBlock) void k_update_x(B a)
{
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    const SysState *st = d.st;
    if (!in_phase(st, kPhaseUpdate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const double sc = st->scale;
    const float *__restrict__ d32 = d.d32;
    double *__restrict__ x = d.x;
    rows_unrolled(rb, re, [&](int i) { x[i] = fma(sc, (double)d32[i], x[i]); });
}

// ------------------------------------------------------------------ iteration
// A: q = A p with the stream tile kernel, p.q fused into the row epilogue.
template <class V, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv_stream(B a)
{
    __shared__ TileLds<V> sm;
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!gate_open(d.st, Vecs<V>::gate)) return;
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const V *__restrict__ p = Vecs<V>::p(d);
    V *__restrict__ q = Vecs<V>::q(d);
    const V *__restrict__ val = Vecs<V>::val(d);
    V acc = V(0);
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * d.R;
        const int r1 = min(r0 + d.R, d.n);
        stream_tile<V>(r0, r1, d.rowptr, d.col, val, p, sm, [&](int i, V y) {
            q[i] = y;
            acc = fma(y, p[i], acc);
        });
    }
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
}

// A with the SELL-64 layout: one slice of 64 rows per wavefront, p.q fused.
template <class V, class CI, int U, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv_sell(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    const Gate g = load_gate(d.st);
    const V *__restrict__ p = Vecs<V>::p(d);
    V *__restrict__ q = Vecs<V>::q(d);
    const V *__restrict__ val = sell_vals<V>(d);
    const SellView sv{d.sell_ptr, d.sell_col, d.sell_len, d.sell_plain, d.sell_len16, d.sell_perm, d.sell_mask};
    V acc = V(0);
    const bool run = gate_ok(g, Vecs<V>::gate);
    sell_slices<V, CI, U>(
        d.n, sell_first(local_block(a)), d.nblk * (kBlock / kWave), sv, val, p, [&] { return run; },
        [&](int i, V y) {
            q[i] = y;
            acc = fma(y, p[i], acc);
        });
    if (!run) return;
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
}

// A for large SELL matrices: one wavefront per slice (ceil(slices / 4)
// blocks, each slice once) and one p.q partial per block in wpart, which
// k_fin_pq folds.  The persistent grid above walks many slices per wave and
// streams a large matrix slower (160^3 27-point: 245 against 226 us).
template <class V, class CI, int U>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv_sell_wide(One a, double *__restrict__ wpart)
{
    __shared__ double red[kBlock / kWave];
    const SysDesc &d = a.d;
    const Gate g = load_gate(d.st);
    const V *__restrict__ p = Vecs<V>::p(d);
    V *__restrict__ q = Vecs<V>::q(d);
    const V *__restrict__ val = sell_vals<V>(d);
    const SellView sv{d.sell_ptr, d.sell_col, d.sell_len, d.sell_plain, d.sell_len16, d.sell_perm, d.sell_mask};
    V acc = V(0);
    const bool run = gate_ok(g, Vecs<V>::gate);
    sell_slices<V, CI, U>(
        d.n, sell_first((int)blockIdx.x), (int)gridDim.x * (kBlock / kWave), sv, val, p, [&] { return run; },
        [&](int i, V y) {
            q[i] = y;
            acc = fma(y, p[i], acc);
        });
    if (!run) return;
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) wpart[blockIdx.x] = blk;
}

// The wide A's nw partials summed into slot 0 of the p.q partials and zeros
// into the other nblk - 1 slots, so that the update pass, which sums those
// slots, gets exactly this sum.  One block of 1024 threads: lane t
// sums partials t, t + 1024, ... in order, then the 16 wave sums in order
// (a 256-thread block took 6.6 us for the 16,000 partials of C3).
constexpr int kFinPqThreads = 1024;
template <class V>
__global__ __launch_bounds__(kFinPqThreads) void k_fin_pq(One a, const double *__restrict__ wpart, int nw)
{
    constexpr int W = kFinPqThreads / kWave, U = 8;
    __shared__ double red[W];
    const SysDesc &d = a.d;
    if (!gate_ok(load_gate(d.st), Vecs<V>::gate)) return;
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < nw; i0 += kFinPqThreads * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kFinPqThreads;
            v[u] = i < nw ? wpart[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    double eta = red[0];
#pragma unroll
    for (int w = 1; w < W; ++w) eta += red[w];
    double *pq = d.partials + kPartPq * d.nblk;
    for (int i = threadIdx.x; i < d.nblk; i += kFinPqThreads) pq[i] = i == 0 ? eta : 0.0;
}

// A (other SpMV kernels): q already holds A p; per-block p.q.
template <class V, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_pq(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!gate_open(d.st, Vecs<V>::gate)) return;
    int rb, re;
    row_range(d, j, rb, re);
    const V *__restrict__ p = Vecs<V>::p(d);
    const V *__restrict__ q = Vecs<V>::q(d);
    V acc = V(0);
    rows_unrolled(rb, re, [&](int i) { acc = fma(q[i], p[i], acc); });
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
}

// B: eta = p.q and alpha = rho / eta (every block sums the p.q partials
// itself, in the same fixed order, so all blocks hold the same bits), then
// r -= alpha q, z = D^-1 r, per-block r.z and r.r.  With eta <= 0 or not
// finite the block changes nothing; C records the reason.  Block 0 records
// the gate, iteration counts, rho and eta it used for C (every B launch of
// the system's precision does, gate open or not).
template <class V, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_update(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!Vecs<V>::present(d)) return;
    const SysState *st = d.st;
    int rb, re;
    row_range(d, j, rb, re);
    V *__restrict__ r = Vecs<V>::r(d);
    V *__restrict__ z = Vecs<V>::z(d);
    const V *__restrict__ q = Vecs<V>::q(d);
    const V *__restrict__ dinv = Vecs<V>::dinv(d);
    V nalpha = V(0);
    V rz = V(0), rr = V(0);
    bool run = false;
    const double *pq = d.partials + kPartPq * d.nblk;
    const bool one_chunk = d.nblk <= kBlock * kPartChunk;
    double pv[kPartChunk];
    if (one_chunk) partials_load(pq, d.nblk, pv);
    rows_prefetched(
        rb, re, [&](int i) { return Trio<V>{r[i], q[i], dinv[i]}; },
        [&]() {
            const Gate g = load_gate(st);
            const double rho = st->rho;
            const double eta = one_chunk ? partials_sum(pv, red) : reduce_partials(pq, d.nblk, red);
            if (j == 0 && threadIdx.x == 0 && g.mixed == Vecs<V>::mixed) {
                // what C decides from: C's block 0 rewrites the live fields
                SysState *w = d.st;
                w->snap_status = g.status;
                w->snap_phase = g.phase;
                w->snap_iter = st->iter;
                w->snap_inner_iter = st->inner_iter;
                w->snap_rho = rho;
                w->snap_eta = eta;
                w->snap_mode = 1;
                w->snap_pbuf = st->pbuf;
            }
            if (!gate_ok(g, Vecs<V>::gate) || !(eta > 0.0) || !finite(eta)) return false;
            nalpha = (V)(-(rho / eta));
            run = true;
            return true;
        },
        [&](int i, const Trio<V> &v) {
            const V ri = fma(nalpha, v.b, v.a);
            const V zi = v.c * ri;
            r[i] = ri;
            z[i] = zi;
            rz = fma(ri, zi, rz);
            rr = fma(ri, ri, rr);
        });
    if (!run) return;
    const double RZb = block_sum((double)rz, red);
    const double RRb = block_sum((double)rr, red);
    if (threadIdx.x == 0) {
        d.partials[kPartRz * d.nblk + j] = RZb;
        d.partials[kPartRr * d.nblk + j] = RRb;
    }
}

// The decision of one iteration from B's recorded scalars and the r.z, r.r
// sums; identical in every block of C.  cmode: 2 = x and p updates, 1 = the
// last x update only, 0 = nothing.
struct Step {
    int cmode = 0;
    int status = SPK_RUNNING;  // new status (SPK_RUNNING: unchanged)
    int to_update = 0;         // mixed: the inner solve ends, refine next
    int fresh_p = 0;           // mixed: the next refinement restarts p from z
    double alpha = 0.0, beta = 0.0, rn = 0.0;
};

__device__ __forceinline__ Step pcg_decide(int mixed, int iter, int inner_iter, double rho, double eta,
                                           double RZ, double RR, const SysState *st)
{
    Step t;
    if (!finite(eta)) { t.status = SPK_DIVERGED_NANORINF; return t; }
    if (eta <= 0.0) {
        if (mixed) { t.to_update = 1; t.fresh_p = 1; }  // inner breakdown: refine, fresh p
        else t.status = SPK_DIVERGED_INDEFINITE_MAT;
        return t;
    }
    t.alpha = rho / eta;
    const int k = iter + 1;
    t.rn = sqrt(RR);
    t.cmode = 1;  // stop unless the tests below continue
    if (!mixed) {
        if (!finite(t.rn)) t.status = SPK_DIVERGED_NANORINF;
        else if (t.rn <= st->thresh)
            t.status = t.rn <= st->rtol * st->bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        else if (k >= st->maxit) t.status = SPK_DIVERGED_ITS;
        else if (!finite(RZ)) t.status = SPK_DIVERGED_NANORINF;
        else if (RZ < 0.0) t.status = SPK_DIVERGED_INDEFINITE_PC;
        else if (RZ == 0.0) t.status = SPK_DIVERGED_BREAKDOWN;
        else { t.beta = RZ / rho; t.cmode = 2; }
    } else {
        const int ki = inner_iter + 1;
        if (!finite(t.rn) || !finite(RZ)) t.status = SPK_DIVERGED_NANORINF;
        else if (t.rn <= st->inner_thresh || ki >= st->inner_maxit || k >= st->maxit || RZ <= 0.0) {
            t.to_update = 1;
            t.fresh_p = RZ <= 0.0;
        } else { t.beta = RZ / rho; t.cmode = 2; }
    }
    return t;
}

// The scalars B recorded for the decision of its iteration (read by C / F,
// whose block 0 rewrites only the live fields).
struct Snap {
    int mixed;
    Gate g;
    int iter, inner_iter;
    double rho, eta;
};

__device__ __forceinline__ Snap load_snap(const SysState *st)
{
    Snap s;
    s.mixed = st->mixed;
    s.g = Gate{st->snap_status, st->snap_phase, s.mixed};
    s.iter = st->snap_iter;
    s.inner_iter = st->snap_inner_iter;
    s.rho = st->snap_rho;
    s.eta = st->snap_eta;
    return s;
}

// Block 0 of C / F: store decision t into the live fields.
__device__ __forceinline__ void pcg_store(SysState *st, const SysDesc &d, const Snap &sn, const Step &t,
                                          double RZ)
{
    st->cmode = 0;  // a pending p continuation has been served
    st->eta = sn.eta;
    if (t.status != SPK_RUNNING) st->status = t.status;
    if (t.to_update) {
        st->phase = kPhaseUpdate;
        if (t.fresh_p) st->fresh_p = 1;
    }
    if (sn.eta > 0.0 && finite(sn.eta)) {
        const int k = sn.iter + 1;
        st->alpha = t.alpha;
        st->iter = k;
        if (sn.mixed) st->inner_iter = sn.inner_iter + 1;
        else {
            st->rnorm = t.rn;
            if (d.hist && k < st->hist_len) d.hist[k] = t.rn;
        }
        if (t.cmode == 2) {
            st->beta = t.beta;
            st->rho = RZ;
        }
    }
}

// B's r.z and r.r partial sums, identical in every block: loads first
// (before the caller's row loads), sums later.
struct RzRr {
    double vz[kPartChunk], vr[kPartChunk];
    bool one_chunk;
    __device__ __forceinline__ void load(const SysDesc &d)
    {
        one_chunk = d.nblk <= kBlock * kPartChunk;
        if (one_chunk) {
            partials_load(d.partials + kPartRz * d.nblk, d.nblk, vz);
            partials_load(d.partials + kPartRr * d.nblk, d.nblk, vr);
        }
    }
    __device__ __forceinline__ void sum(const SysDesc &d, double *red, double &RZ, double &RR)
    {
        if (one_chunk) {
            RZ = partials_sum(vz, red);
            RR = partials_sum(vr, red);
        } else {
            reduce_partials2(d.partials + kPartRz * d.nblk, d.partials + kPartRr * d.nblk, d.nblk, red, RZ, RR);
        }
    }
};

// C: the iteration's decision (see pcg_decide), stored by block 0, then
// x += alpha p (d for mixed) and, while iterating, p = z + beta p.
template <class V, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_px(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!Vecs<V>::present(d) || Vecs<V>::p2(d)) return;  // fused systems: F does it
    SysState *st = d.st;
    int rb, re;
    row_range(d, j, rb, re);
    V *__restrict__ x = Vecs<V>::x(d);
    V *__restrict__ p = Vecs<V>::p(d);
    const V *__restrict__ z = Vecs<V>::z(d);
    RzRr part;
    part.load(d);
    int cm = 0;
    V alpha = V(0), beta = V(0);
    rows_prefetched(
        rb, re, [&](int i) { return Trio<V>{p[i], z[i], x[i]}; },
        [&]() {
            const Snap sn = load_snap(st);
            double RZ, RR;
            part.sum(d, red, RZ, RR);
            if (sn.mixed != Vecs<V>::mixed || !gate_ok(sn.g, Vecs<V>::gate)) return false;
            const Step t = pcg_decide(sn.mixed, sn.iter, sn.inner_iter, sn.rho, sn.eta, RZ, RR, st);
            if (j == 0 && threadIdx.x == 0) pcg_store(st, d, sn, t, RZ);
            cm = t.cmode;
            alpha = (V)t.alpha;
            beta = (V)t.beta;
            return cm != 0;
        },
        [&](int i, const Trio<V> &v) {
            x[i] = fma(alpha, v.a, v.c);
            if (cm == 2) p[i] = fma(beta, v.a, v.b);
        });
}

// F: C of iteration k fused with A of iteration k + 1, for systems with the
// SELL product on the persistent grid and a second p buffer (p2).  An
// iteration is then two kernels (B, F) and moves 88n vector bytes, the
// lower bound (the p update rides in the product's gather), instead of 96n
// and a third launch.  The p of iteration k + 1 is formed wherever the
// product gathers it, p' = z + beta p, the same FMA as C's and so the same
// bits in every block that forms element j, and the lane that owns row j
// stores it into the other buffer, so p of iteration k stays intact while
// other blocks still gather it.  The results are those of A, B, C bit for
// bit.  kStart: the first product of a CG sequence, launched after the setup
// finalizers (snap_mode 0: p' = z; 3: p' = z + beta p after a reliable
// update, beta from the refinement); otherwise snap_mode 1: B's recorded
// decision, then x += alpha p and, while iterating, the product.
template <class V, class CI, int U, bool kStart, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_fused_sell(B a)
{
    __shared__ double red[kBlock / kWave];
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!Vecs<V>::present(d) || !Vecs<V>::p2(d)) return;
    SysState *st = d.st;
    // written by B and the setup finalizers only, never by this kernel
    const int mode = st->snap_mode;
    if (kStart ? mode == 1 : mode != 1) return;
    RzRr part;
    if (!kStart) part.load(d);
    const int pb = st->snap_pbuf;
    int cm = 2;  // 2: (x update and) product; 1: the last x update
    bool fresh = false;
    V alpha = V(0), beta = V(0);
    if (kStart) {
        if (!gate_ok(load_gate(st), Vecs<V>::gate)) return;
        fresh = mode == 0;
        beta = fresh ? V(0) : (V)st->beta;  // the finalizer's beta (F stores beta only when deciding)
        if (j == 0 && threadIdx.x == 0) {
            st->pbuf = pb ^ 1;
            st->cmode = 0;
        }
    } else {
        const Snap sn = load_snap(st);
        double RZ, RR;
        part.sum(d, red, RZ, RR);
        if (sn.mixed != Vecs<V>::mixed || !gate_ok(sn.g, Vecs<V>::gate)) return;
        const Step t = pcg_decide(sn.mixed, sn.iter, sn.inner_iter, sn.rho, sn.eta, RZ, RR, st);
        if (j == 0 && threadIdx.x == 0) {
            pcg_store(st, d, sn, t, RZ);
            if (t.cmode == 2) st->pbuf = pb ^ 1;
        }
        cm = t.cmode;
        if (cm == 0) return;
        alpha = (V)t.alpha;
        beta = (V)t.beta;
    }
    const V *__restrict__ pold = pb ? Vecs<V>::p2(d) : Vecs<V>::p(d);
    V *__restrict__ pnew = pb ? Vecs<V>::p(d) : Vecs<V>::p2(d);
    const V *__restrict__ z = Vecs<V>::z(d);
    V *__restrict__ x = Vecs<V>::x(d);
    V *__restrict__ q = Vecs<V>::q(d);
    if (cm == 1) {  // the solve (or the inner solve) stops: x update only
        int rb, re;
        row_range(d, j, rb, re);
        rows_unrolled(rb, re, [&](int i) { x[i] = fma(alpha, pold[i], x[i]); });
        return;
    }
    auto pn = [&](int c) -> V { return fresh ? z[c] : fma(beta, pold[c], z[c]); };
    const SellView sv{d.sell_ptr, d.sell_col, d.sell_len, d.sell_plain, d.sell_len16, d.sell_perm, d.sell_mask};
    V acc = V(0);
    sell_slices_g<V, CI, U>(d.n, sell_first(local_block(a)), d.nblk * (kBlock / kWave), sv, sell_vals<V>(d), pn,
                            [] { return true; }, [&](int i, V y) {
                                const V pi = pn(i);
                                if (!kStart) x[i] = fma(alpha, pold[i], x[i]);
                                pnew[i] = pi;
                                q[i] = y;
                                acc = fma(y, pi, acc);
                            });
    const double blk = block_sum((double)acc, red);
    if (threadIdx.x == 0) d.partials[kPartPq * d.nblk + j] = blk;
}

// p = z + beta p where the last refinement asked for it (cmode 3: CG
// continues after a reliable update, with beta from k_fin_setup32).
template <class V, class B>
__global__ __launch_bounds__(kBlock) void k_pcg_p_continue(B a)
{
    int j;
    SysDesc d;
    if (!locate(a, j, d)) return;
    if (!Vecs<V>::present(d) || Vecs<V>::p2(d)) return;  // fused systems: F does it
    const SysState *st = d.st;
    int rb, re;
    row_range(d, j, rb, re);
    V *__restrict__ p = Vecs<V>::p(d);
    const V *__restrict__ z = Vecs<V>::z(d);
    V beta = V(0);
    rows_prefetched(
        rb, re, [&](int i) { return Trio<V>{p[i], z[i], V(0)}; },
        [&]() {
            beta = (V)st->beta;
            return st->mixed == Vecs<V>::mixed && st->status == SPK_RUNNING && st->cmode == 3;
        },
        [&](int i, const Trio<V> &v) { p[i] = fma(beta, v.a, v.b); });
}

}  // namespace spk
