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

// Y-rows = A X-rows for one row, K columns, entries [a, e) of CSR; U
// entries per round with their gathers issued together.
template <int K>
__device__ __forceinline__ void csr_row_multi(int a, int e, const int32_t *__restrict__ col,
                                              const double *__restrict__ val,
                                              const double *__restrict__ X, double acc[K])
{
    constexpr int U = K >= 8 ? 1 : 8 / K;
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    for (int k0 = a; k0 < e; k0 += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u < e ? k0 + u : e - 1;
            c[u] = ld_stream(col + k);
            v[u] = ld_stream(val + k);
        }
        double xv[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < K; ++q) xv[u][q] = X[(size_t)c[u] * K + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < e)
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] = fma(v[u], xv[u][q], acc[q]);
    }
}

// Same for lane `lane` of a SELL slice (b, slen), the row having rlen
// entries.  The offset and value pairs of up to kMultiPairs pairs are loaded
// together (one paired load of offsets and of values each), then the K
// gathers of pair p + 1 (or of the slice's odd last entry) are issued before
// the FMAs of pair p, so the gathers of consecutive pairs overlap instead of
// costing one memory round trip each (K = 8 on the 7-point 128^3 product:
// 118 -> 95 us with the staged stores below).  K = 16 keeps one pair in
// registers at a time (double buffering would take 128 more VGPRs).  Sums
// run in column order either way.
//
// kOneRound (standalone SpMM): a slice of at most kOneRoundPairs pairs loads
// them and issues every gather (the odd entry's too) before the first FMA,
// one memory round trip per slice at the cost of holding all gathered rows
// (K = 8: 152 VGPRs, three wavefronts per SIMD).  The product inside the
// multi-RHS solve keeps the pipelined walk: there the extra registers cost
// more than the round trips they save.
constexpr int kMultiPairs = 4;
constexpr int kOneRoundPairs = 3;

//
// SH: shared offsets (see the SELL-64 notes): offsets from the slice's list,
// rlen the row's position mask, gathered rows clamped into [0, n).
//
// pdiag (the pipelined walk only; null otherwise): where to keep the row's
// own gathered X row, the gather of its diagonal entry (offset 0; the
// solve's matrices have one in every row), so that the caller need not read
// it again.
template <class CI, int K, bool kOneRound = false, bool SH = false>
__device__ __forceinline__ void sell_row_multi(const SellView &sv, const double *__restrict__ val,
                                               const double *__restrict__ X, int32_t b, int slen,
                                               int rlen, int lane, int row, int n, double acc[K],
                                               double *pdiag = nullptr)
{
    static_assert(!SH || std::is_same<CI, int32_t>::value, "shared offsets are int32");
    constexpr int PM = K <= 8 ? kMultiPairs : 1;
    using CP = typename Pair2<CI>::type;
    using VP = typename Pair2<double>::type;
    const CP *__restrict__ cp = reinterpret_cast<const CP *>(reinterpret_cast<const CI *>(sv.col) + b) + lane;
    const int32_t *__restrict__ ou =
        reinterpret_cast<const int32_t *>(sv.col) + (__builtin_amdgcn_readfirstlane(b) >> 6);
    const VP *__restrict__ vp = reinterpret_cast<const VP *>(val + b) + lane;
    auto offsets = [&](int p) -> CP {
        if constexpr (SH) {
            CP c;
            c.x = ou[2 * p];
            c.y = ou[2 * p + 1];
            return c;
        } else {
            return ld_stream(cp + (size_t)p * kSell);
        }
    };
    auto real = [&](int k) -> bool {
        if constexpr (SH) return ((unsigned)rlen >> k) & 1u;
        else return k < rlen;
    };
    const int np = slen >> 1;
    const bool odd = slen & 1;
    CI ct = CI(0);
    double at = 0.0;
    if (odd) {
        const size_t t = (size_t)b + (size_t)np * (2 * kSell) + lane;
        if constexpr (SH) ct = ou[2 * np];
        else ct = ld_stream(reinterpret_cast<const CI *>(sv.col) + t);
        at = ld_stream(val + t);
    }
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    auto gather = [&](int off, double xr[K]) {
        int j = row + off;
        if constexpr (SH) j = min(max(j, 0), n - 1);
#pragma unroll
        for (int q = 0; q < K; ++q) xr[q] = X[(size_t)j * K + q];
    };
    auto madd = [&](double a, const double xr[K]) {
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fma(a, xr[q], acc[q]);
    };
    auto keep = [&](int off, const double xr[K]) {
        if (pdiag && off == 0)
#pragma unroll
            for (int q = 0; q < K; ++q) pdiag[q] = xr[q];
    };
    if (kOneRound && K <= 8 && np <= kOneRoundPairs) {
        // every pair index is clamped into the slice (a slice without pairs
        // loads none: its gathers then fetch the lane's own row, unused)
        constexpr int P1 = kOneRoundPairs;
        CP c[P1];
        VP a[P1];
#pragma unroll
        for (int u = 0; u < P1; ++u) {
            c[u].x = c[u].y = CI(0);
            a[u].x = a[u].y = 0.0;
        }
        if (np > 0)
#pragma unroll
            for (int u = 0; u < P1; ++u) {
                const int p = u < np ? u : np - 1;
                c[u] = offsets(p);
                a[u] = ld_stream(vp + (size_t)p * kSell);
            }
        double xv[2 * P1 + 1][K];
#pragma unroll
        for (int u = 0; u < P1; ++u) {
            gather((int)c[u].x, xv[2 * u]);
            gather((int)c[u].y, xv[2 * u + 1]);
        }
        gather((int)ct, xv[2 * P1]);
#pragma unroll
        for (int u = 0; u < P1; ++u)
            if (u < np) {
                if (real(2 * u)) madd(a[u].x, xv[2 * u]);
                if (real(2 * u + 1)) madd(a[u].y, xv[2 * u + 1]);
            }
        if (odd && real(slen - 1)) madd(at, xv[2 * P1]);
        return;
    }
    if (PM > 1 && np >= 1 && np <= PM) {
        // the slice's pairs in one load round, gathers one pair ahead
        CP c[PM];
        VP a[PM];
#pragma unroll
        for (int u = 0; u < PM; ++u) {
            const int p = u < np ? u : np - 1;
            c[u] = offsets(p);
            a[u] = ld_stream(vp + (size_t)p * kSell);
        }
        double xa[2][K], xb[2][K];
        gather((int)c[0].x, xa[0]);
        gather((int)c[0].y, xa[1]);
#pragma unroll
        for (int u = 0; u < PM; ++u) {
            if (u + 1 < PM && u + 1 < np) {
                gather((int)c[u + 1].x, xb[0]);
                gather((int)c[u + 1].y, xb[1]);
            }
            if (u < np) {
                if (real(2 * u)) {
                    madd(a[u].x, xa[0]);
                    keep((int)c[u].x, xa[0]);
                }
                if (real(2 * u + 1)) {
                    madd(a[u].y, xa[1]);
                    keep((int)c[u].y, xa[1]);
                }
            }
#pragma unroll
            for (int q = 0; q < K; ++q) {
                xa[0][q] = xb[0][q];
                xa[1][q] = xb[1][q];
            }
        }
    } else {
        // wide slices (or K = 16): one pair per round
        for (int p = 0; p < np; ++p) {
            const CP c = offsets(p);
            const VP a = ld_stream(vp + (size_t)p * kSell);
            double x0[K], x1[K];
            gather((int)c.x, x0);
            gather((int)c.y, x1);
            if (real(2 * p)) {
                madd(a.x, x0);
                keep((int)c.x, x0);
            }
            if (real(2 * p + 1)) {
                madd(a.y, x1);
                keep((int)c.y, x1);
            }
        }
    }
    if (odd && real(slen - 1)) {
        double xt[K];
        gather((int)ct, xt);
        madd(at, xt);
        keep((int)ct, xt);
    }
}

// SELL slices of block l with the K products of each row staged in LDS
// (stage: this wave's 64 x K doubles), then handed out flat: flat(e0, cnt)
// for the slice's cnt elements starting at element e0 of the row-major
// n x K layout, which the caller walks with lane t taking elements t, t + 64,
// ... of the stage (so always column t % K, as 64 % K == 0).  A lane's K
// products are 8K contiguous bytes, so storing them from the lanes directly
// writes 64 partial segments per instruction; the flat pass writes whole
// ones (K = 8: 118 -> 99 us on the 7-point 128^3 product).
template <class CI, int K, bool kOneRound, bool SH, class Flat>
__device__ __forceinline__ void multi_sell_walk(const MultiDesc &d, int l, const double *__restrict__ X,
                                                double *stage, double *pstage, Flat &&flat)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int ns = (d.n + kSell - 1) / kSell;
    for (int s = l * (kBlock / kWave) + (int)threadIdx.x / kWave; s < ns; s += d.nblk * (kBlock / kWave)) {
        const int32_t b = d.sv.ptr[s], e = d.sv.ptr[s + 1];
        const int row = s * kSell + lane;
        if (row < d.n) {
            double acc[K];
            const int rl = SH ? (int)d.sv.mask[row] : (int)d.sv.len[row];
            sell_row_multi<CI, K, kOneRound, SH>(d.sv, d.sell_val, X, b, (e - b) / kSell, rl, lane, row, d.n,
                                                 acc, pstage ? pstage + lane * K : nullptr);
#pragma unroll
            for (int q = 0; q < K; ++q) stage[lane * K + q] = acc[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        flat((int64_t)s * kSell * K, (min(d.n, (s + 1) * kSell) - s * kSell) * K);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <class CI, int K, bool kOneRound, class Flat>
__device__ __forceinline__ void multi_sell_staged(const MultiDesc &d, int l, const double *__restrict__ X,
                                                  double *stage, double *pstage, Flat &&flat)
{
    if constexpr (std::is_same<CI, int32_t>::value) {
        if (d.sv.mask) {
            multi_sell_walk<CI, K, kOneRound, true>(d, l, X, stage, pstage, flat);
            return;
        }
    }
    multi_sell_walk<CI, K, kOneRound, false>(d, l, X, stage, pstage, flat);
}

// Row walk of block l (of nblk) of a multi kernel: SELL slices in
// round-robin order, or CSR rows of the block's contiguous tile range with
// one row per lane.  fn(row, acc) gets the K products of the row.
template <class CI, int K, class Fn>
__device__ __forceinline__ void multi_rows(const MultiDesc &d, int l, int j, const double *__restrict__ X,
                                           Fn &&fn)
{
    double acc[K];
    if (d.sell) {
        const int lane = threadIdx.x & (kWave - 1);
        const int ns = (d.n + kSell - 1) / kSell;
        for (int s = l * (kBlock / kWave) + (int)threadIdx.x / kWave; s < ns; s += d.nblk * (kBlock / kWave)) {
            const int32_t b = d.sv.ptr[s], e = d.sv.ptr[s + 1];
            const int row = s * kSell + lane;
            if (row < d.n) {
                if constexpr (std::is_same<CI, int32_t>::value) {
                    if (d.sv.mask) {
                        sell_row_multi<CI, K, false, true>(d.sv, d.sell_val, X, b, (e - b) / kSell,
                                                           (int)d.sv.mask[row], lane, row, d.n, acc);
                        fn(row, acc);
                        continue;
                    }
                }
                sell_row_multi<CI, K>(d.sv, d.sell_val, X, b, (e - b) / kSell, d.sv.len[row], lane, row, d.n, acc);
                fn(row, acc);
            }
        }
    } else {
        int t0, t1;
        block_tiles(j, d.nblk, d.ntiles, t0, t1);
        const int rb = t0 * d.R, re = min(t1 * d.R, d.n);
        for (int row = rb + (int)threadIdx.x; row < re; row += kBlock) {
            csr_row_multi<K>(d.rowptr[row], d.rowptr[row + 1], d.col, d.val, X, acc);
            fn(row, acc);
        }
    }
}

// Block sums of K per-lane values, one partial per column: part[q * nblk + j].
template <int K>
__device__ __forceinline__ void block_partials(double v[K], double *sh /* [4][K] */, double *part,
                                               int nblk, int j)
{
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = wave_sum(v[q]);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) sh[w * K + q] = v[q];
    __syncthreads();
    if ((int)threadIdx.x < K) {
        const int q = threadIdx.x;
        double s = sh[q];
#pragma unroll
        for (int ww = 1; ww < kBlock / kWave; ++ww) s += sh[ww * K + q];
        part[(size_t)q * nblk + j] = s;
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

// flat_walk with every load of a chunk issued before its stores: ld(e)
// returns what element e needs, st(e, v) writes it back.  Used where a store
// is conditional per lane, which otherwise keeps the compiler from moving
// the next element's loads above it.
template <int K, class Ld, class St>
__device__ __forceinline__ void flat_walk_batched(const MultiDesc &d, int j, Ld &&ld, St &&st)
{
    int t0, t1;
    block_tiles(j, d.nblk, d.ntiles, t0, t1);
    const int64_t e0 = (int64_t)t0 * d.R * K, e1 = (int64_t)min(t1 * d.R, d.n) * K;
    constexpr int U = 4;
    using T = decltype(ld(int64_t(0)));
    for (int64_t eb = e0 + threadIdx.x; eb < e1; eb += (int64_t)kBlock * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (int64_t)u * kBlock;
            if (e < e1) v[u] = ld(e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (int64_t)u * kBlock;
            if (e < e1) st(e, v[u]);
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
// Physical block l runs on XCD l % 8.  Logical blocks in runs of R per XCD:
// ((l / 8) / R) 8R + (l % 8) R + (l / 8) % R, a bijection when nblk is a
// multiple of 8R (else the identity), so that R consecutive logical blocks
// (4R consecutive slices for the SpMM) share an L2.
__device__ __forceinline__ int xcd_runs(int l, int nblk, int R)
{
    if (nblk % (kXcd * R)) return l;
    const int x = l % kXcd, k = l / kXcd;
    return (k / R) * (kXcd * R) + x * R + k % R;
}

template <class CI, int K>
__global__ __launch_bounds__(kBlock) void k_spmm(MultiDesc d, const double *__restrict__ X, double *__restrict__ Y)
{
    __shared__ double stage[(kBlock / kWave) * kWave * (K > 1 ? K : 1)];
    int j;
    int l = multi_block(d, j);
    if (l < 0) return;
    if (d.sell && K > 1) {
        // runs of 4 blocks (16 slices) per XCD keep the +-1-line gathers of
        // neighbouring slices in one L2
        l = xcd_runs(l, d.nblk, 4);
        // flat stores of two elements (K is even): 1 KB per instruction
        using VP = typename Pair2<double>::type;
        const int lane = threadIdx.x & (kWave - 1);
        double *st = stage + (threadIdx.x / kWave) * kWave * K;
        multi_sell_staged<CI, K, true>(d, l, X, st, nullptr, [&](int64_t e0, int cnt) {
            const VP *src = reinterpret_cast<const VP *>(st);
            VP *dst = reinterpret_cast<VP *>(Y + e0);
            for (int t = lane; t < cnt / 2; t += kWave) __builtin_nontemporal_store(src[t], dst + t);
        });
        return;
    }
    multi_rows<CI, K>(d, l, j, X, [&](int row, const double *acc) {
#pragma unroll
        for (int q = 0; q < K; ++q) Y[(size_t)row * K + q] = acc[q];
    });
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
    const double *__restrict__ X = d.X;
    const double *__restrict__ Bv = d.B;
    double *__restrict__ Rv = d.Rv;
    double rr[K], bb[K];
#pragma unroll
    for (int q = 0; q < K; ++q) rr[q] = bb[q] = 0.0;
    multi_rows<CI, K>(d, l, j, X, [&](int row, const double *acc) {
        double br[K];  // the row of B, loaded before any store of R
#pragma unroll
        for (int q = 0; q < K; ++q) br[q] = Bv[(size_t)row * K + q];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            if (!((mask >> q) & 1)) continue;
            const double bi = br[q];
            const double ri = bi - acc[q];
            Rv[(size_t)row * K + q] = ri;
            rr[q] = fma(ri, ri, rr[q]);
            bb[q] = fma(bi, bi, bb[q]);
        }
    });
    block_partials<K>(rr, sh, d.partials + (size_t)kPartRr * K * d.nblk, d.nblk, j);
    block_partials<K>(bb, sh, d.partials + (size_t)kPartBb * K * d.nblk, d.nblk, j);
}

// The finalize kernels run one block per column (q = blockIdx.x): the block
// sums the column's nblk partials in a fixed order (reduce_partials), thread
// 0 runs the column's scalar logic, and a column that stops clears its bit
// of the running mask with an integer atomic (the only cross-block write).
__device__ __forceinline__ const double *col_part(const MultiDesc &d, int part, int q)
{
    return d.partials + ((size_t)part * d.K + q) * d.nblk;
}

__device__ __forceinline__ void stop_column(const MultiDesc &d, int q)
{
    atomicAnd(&d.ctl->mask, ~(1 << q));
}

// purpose kMultiSetup: norms, thresholds, stop at start; kMultiTrue: store the
// true residual norm of the columns in mask.
static __global__ __launch_bounds__(kBlock) void k_m_fin_resid(MultiDesc d, int purpose, int32_t mask)
{
    __shared__ double red[kBlock / kWave];
    const int q = blockIdx.x;
    if (q >= d.K || !((mask >> q) & 1)) return;
    double RR, BB;
    reduce_partials2(col_part(d, kPartRr, q), col_part(d, kPartBb, q), d.nblk, red, RR, BB);
    if (threadIdx.x != 0) return;
    SysState *st = d.st + q;
    const double rn = sqrt(RR);
    if (purpose == kMultiTrue) {
        st->rnorm_true = rn;
        return;
    }
    const double bn = sqrt(BB);
    st->bnorm = bn;
    st->thresh = fmax(st->rtol * bn, st->atol);
    st->rnorm = rn;
    st->rnorm0 = rn;
    if (bn == 0.0) st->status = SPK_CONVERGED_ATOL;
    else if (!isfinite(rn) || !isfinite(bn)) st->status = SPK_DIVERGED_NANORINF;
    else if (rn <= st->thresh) st->status = rn <= st->rtol * bn ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
    if (st->status != SPK_RUNNING) stop_column(d, q);
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
    const double *__restrict__ Rv = d.Rv;
    const double *__restrict__ dinv = d.dinv;
    double *__restrict__ Z = d.Z;
    double *__restrict__ P = d.P;
    double rz = 0.0;
    if (run)
        flat_walk<K>(d, j, [&](int64_t e, int i) {
            const double ri = Rv[e];
            const double zi = dinv[i] * ri;
            Z[e] = zi;
            P[e] = zi;
            rz = fma(ri, zi, rz);
        });
    block_partials_flat<K>(rz, sh, d.partials + (size_t)kPartRz * K * d.nblk, d.nblk, j);
}

static __global__ __launch_bounds__(kBlock) void k_m_fin_setup(MultiDesc d, int32_t mask)
{
    __shared__ double red[kBlock / kWave];
    const int q = blockIdx.x;
    if (q >= d.K || !((mask >> q) & 1)) return;
    SysState *st = d.st + q;
    if (st->status != SPK_RUNNING) return;
    const double RZ = reduce_partials(col_part(d, kPartRz, q), d.nblk, red);
    if (threadIdx.x != 0) return;
    st->cmode = 0;
    if (!isfinite(RZ)) st->status = SPK_DIVERGED_NANORINF;
    else if (RZ < 0.0) st->status = SPK_DIVERGED_INDEFINITE_PC;
    else if (RZ == 0.0) st->status = SPK_DIVERGED_BREAKDOWN;
    else if (st->iter >= st->maxit) { st->status = SPK_DIVERGED_ITS; st->rho = RZ; }
    else st->rho = RZ;
    if (st->status != SPK_RUNNING) stop_column(d, q);
}

// Restart the columns in mask from their true residual (already in R).
static __global__ void k_m_restart(MultiDesc d, int32_t mask)
{
    const int q = threadIdx.x;
    if (q < d.K && ((mask >> q) & 1)) {
        d.st[q].status = SPK_RUNNING;
        d.st[q].cmode = 0;
    }
    if (q == 0) d.ctl->mask |= mask;
}

// ------------------------------------------------------------------ iteration
// A: Q = A P, per-column per-block p.q (columns that stopped are multiplied
// too: the matrix is read once either way; their partials are ignored).
template <class CI, int K>
__global__ __launch_bounds__(kBlock, K <= 8 ? 4 : 1) void k_m_spmm_pq(MultiDesc d)
{
    __shared__ double sh[(kBlock / kWave) * K];
    __shared__ double stage[(kBlock / kWave) * kWave * (K > 1 ? K : 1)];
    // each row's own P row, kept from its diagonal gather (every row of a
    // solved matrix has one): the flat pass's p.q reads it here instead of
    // fetching P a second time (the rows were gathered moments before, but
    // read again from memory they cost a third of the kernel's traffic)
    __shared__ double pstage[(kBlock / kWave) * kWave * (K > 1 ? K : 1)];
    int j;
    const int l = multi_block(d, j);
    if (l < 0) return;
    if (d.ctl->mask == 0) return;
    // Q never aliases P: without the qualifiers the compiler orders every
    // gather of P behind the stores of Q
    const double *__restrict__ P = d.P;
    double *__restrict__ Q = d.Q;
    if (d.sell && K > 1) {
        // flat pass: lane t always holds column t % K
        double pqv = 0.0;
        const int lane = threadIdx.x & (kWave - 1);
        const double *st = stage + (threadIdx.x / kWave) * kWave * K;
        const double *pst = pstage + (threadIdx.x / kWave) * kWave * K;
        multi_sell_staged<CI, K, false>(d, l, P, stage + (threadIdx.x / kWave) * kWave * K,
                                        pstage + (threadIdx.x / kWave) * kWave * K,
                                        [&](int64_t e0, int cnt) {
                                            for (int t = lane; t < cnt; t += kWave) {
                                                const double v = st[t], pe = pst[t];
                                                Q[e0 + t] = v;
                                                pqv = fma(v, pe, pqv);
                                            }
                                        });
        block_partials_flat<K>(pqv, sh, d.partials + (size_t)kPartPq * K * d.nblk, d.nblk, j);
        return;
    }
    double pq[K];
#pragma unroll
    for (int q = 0; q < K; ++q) pq[q] = 0.0;
    multi_rows<CI, K>(d, l, j, P, [&](int row, const double *acc) {
        double pr[K];  // the row of P, loaded before any store of Q
#pragma unroll
        for (int q = 0; q < K; ++q) pr[q] = P[(size_t)row * K + q];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Q[(size_t)row * K + q] = acc[q];
            pq[q] = fma(acc[q], pr[q], pq[q]);
        }
    });
    block_partials<K>(pq, sh, d.partials + (size_t)kPartPq * K * d.nblk, d.nblk, j);
}

// F_A: eta = p.q and alpha per running column; eta <= 0 stops the column.
static __global__ __launch_bounds__(kBlock) void k_m_fin_pq(MultiDesc d)
{
    __shared__ double red[kBlock / kWave];
    const int q = blockIdx.x;
    if (q >= d.K) return;
    SysState *st = d.st + q;
    if (st->status != SPK_RUNNING) return;
    const double eta = reduce_partials(col_part(d, kPartPq, q), d.nblk, red);
    if (threadIdx.x != 0) return;
    st->eta = eta;
    st->cmode = 0;
    if (!isfinite(eta)) st->status = SPK_DIVERGED_NANORINF;
    else if (eta <= 0.0) st->status = SPK_DIVERGED_INDEFINITE_MAT;
    else st->alpha = st->rho / eta;
    if (st->status != SPK_RUNNING) stop_column(d, q);
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
    const double *__restrict__ Q = d.Q;
    const double *__restrict__ dinv = d.dinv;
    double *__restrict__ Rv = d.Rv;
    double *__restrict__ Z = d.Z;
    double rz = 0.0, rr = 0.0;
    if (run)
        flat_walk<K>(d, j, [&](int64_t e, int i) {
            const double ri = fma(nal, Q[e], Rv[e]);
            const double zi = dinv[i] * ri;
            Rv[e] = ri;
            Z[e] = zi;
            rz = fma(ri, zi, rz);
            rr = fma(ri, ri, rr);
        });
    block_partials_flat<K>(rz, sh, d.partials + (size_t)kPartRz * K * d.nblk, d.nblk, j);
    block_partials_flat<K>(rr, sh, d.partials + (size_t)kPartRr * K * d.nblk, d.nblk, j);
}

// F_B: per running column: iteration count, convergence, breakdowns, beta;
// cmode 2 (x and p updates) or 1 (the last x update), as in the single
// solve; a column that is not running gets cmode 0, so the p/x kernel of a
// later replay leaves it alone.
static __global__ __launch_bounds__(kBlock) void k_m_fin_update(MultiDesc d)
{
    __shared__ double red[kBlock / kWave];
    const int q = blockIdx.x;
    if (q >= d.K) return;
    SysState *st = d.st + q;
    if (st->status != SPK_RUNNING) {
        if (threadIdx.x == 0) st->cmode = 0;
        return;
    }
    double RZ, RR;
    reduce_partials2(col_part(d, kPartRz, q), col_part(d, kPartRr, q), d.nblk, red, RZ, RR);
    if (threadIdx.x != 0) return;
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
    if (st->status != SPK_RUNNING) stop_column(d, q);
}

// C: per column, cmode 2: x += alpha p, p = z + beta p; cmode 1: x += alpha p.
// It keeps no partial sums, so it runs on a grid of its own (kMultiPxBlocks
// at most): block b takes the b-th chunk of the flat n x K range, a multiple
// of 256 elements, in physical block order (a streaming pass gains nothing
// from XCD-contiguous ranges; on the 128^3 k = 8 block, 1024 blocks with
// those ranges took 131.5 us, 8192 in order 120.8).
constexpr int kMultiPxBlocks = 8192;
template <int K>
__global__ __launch_bounds__(kBlock) void k_m_px(MultiDesc d)
{
    const int q = threadIdx.x % K;
    const int cm = d.st[q].cmode;
    if (cm == 0) return;  // no barrier follows
    const double al = d.st[q].alpha, be = d.st[q].beta;
    double *__restrict__ X = d.X;
    double *__restrict__ P = d.P;
    const double *__restrict__ Z = d.Z;
    const int64_t nk = (int64_t)d.n * K;
    const int64_t per = ((nk + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min(nk, e0 + per);
    constexpr int U = 4;
    for (int64_t eb = e0 + threadIdx.x; eb < e1; eb += (int64_t)kBlock * U) {
        double p[U], x[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (int64_t)u * kBlock;
            if (e < e1) {
                p[u] = P[e];
                x[u] = X[e];
                z[u] = Z[e];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (int64_t)u * kBlock;
            if (e < e1) {
                X[e] = fma(al, p[u], x[u]);
                if (cm == 2) P[e] = fma(be, p[u], z[u]);
            }
        }
    }
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
    if (q < d.K) d.st[q].cmode = 0;
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
