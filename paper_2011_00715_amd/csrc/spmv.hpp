// CSR SpMV kernels for gfx950 (y = A x, the MatMult on AIJ of Sec. 4).
//
// Three families, chosen from row-length statistics at matrix creation:
//  * stream : a block owns a tile of R consecutive rows.  All 256 lanes read
//             the tile's column and value streams contiguously (non-temporal,
//             so x stays in cache), gather x, and stage the products in LDS;
//             then one lane per row sums its products in order.  Every lane is
//             busy during the loads even for 5..27-entry rows.
//  * vector : L lanes per row (L = 64 is one row per wavefront), lane-strided
//             FMA partial sums, butterfly shuffle reduction inside the group.
//  * merge  : merge-path over the sequence of (row ends + nonzeros), split into
//             equal tiles of 2048 items; each lane walks 8 items, a segmented
//             scan in LDS combines rows split across lanes, and a fix-up pass
//             adds rows split across tiles in tile order (no atomics, so the
//             result is reproducible bit for bit).
#pragma once

#include <type_traits>

#include "common.hpp"

namespace spk {

enum { kGateNone = 0, kGateInner64 = 1, kGateInner32 = 2, kGateResid = 3 };

// The state fields that decide whether a solver kernel runs.  Kernels load
// them together with their first operands (one memory round trip) and test
// them afterwards.
struct Gate {
    int32_t status, phase, mixed;
};

__device__ __forceinline__ Gate load_gate(const SysState *st)
{
    return Gate{st->status, st->phase, st->mixed};
}

// Whether a solver kernel launched inside a captured graph should run.
__device__ __forceinline__ bool gate_ok(const Gate &g, int mode)
{
    switch (mode) {
    case kGateNone: return true;
    case kGateInner64:
        return g.status == SPK_RUNNING && g.phase == kPhaseInner && g.mixed == 0;
    case kGateInner32:
        return g.status == SPK_RUNNING && g.phase == kPhaseInner && g.mixed == 1;
    case kGateResid:
        return g.status == SPK_RUNNING && g.mixed == 1 &&
               (g.phase == kPhaseResid || g.phase == kPhaseUpdate);
    }
    return false;
}

__device__ __forceinline__ bool gate_open(const SysState *st, int mode)
{
    return mode == kGateNone || gate_ok(load_gate(st), mode);
}

// sum over k = k0, k0 + L, ... below e of val[k] x[col[k]] in that order
// (FMA), four entries per round with their gathers issued together.
template <class V, int L>
__device__ __forceinline__ V strided_dot(int k0, int e, const int32_t *__restrict__ col,
                                         const V *__restrict__ val, const V *__restrict__ x)
{
    constexpr int U = 4;
    V s = V(0);
    for (int kb = k0; kb < e; kb += L * U) {
        int c[U];
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kb + u * L < e ? kb + u * L : e - 1;
            c[u] = ld_stream(col + k);
            v[u] = ld_stream(val + k);
        }
        V xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (kb + u * L < e) s = fma(v[u], xv[u], s);
    }
    return s;
}

template <class V>
struct TileLds {
    static constexpr int kCap = kTileBytes / (int)sizeof(V);
    V prod[kCap];
    int32_t rp[kBlock + 1];
    V red[kBlock / kWave];
};

// One tile of rows [r0, r1) (r1 - r0 <= kBlock).  fn(row, value) is called
// once per row, by the lane that owns it.  Products are rounded to V and
// summed in V in column order.  Tiles with more than kCap nonzeros take the
// block-per-row path (block-wide FMA partials and a fixed-order block sum).
template <class V, class Fn>
__device__ __forceinline__ void stream_tile(int r0, int r1, const int32_t *__restrict__ rowptr,
                                            const int32_t *__restrict__ col,
                                            const V *__restrict__ val, const V *__restrict__ x,
                                            TileLds<V> &sm, Fn &&fn)
{
    const int nr = r1 - r0;
    for (int i = threadIdx.x; i <= nr; i += kBlock) sm.rp[i] = rowptr[r0 + i];
    __syncthreads();
    const int k0 = sm.rp[0];
    const int k1 = sm.rp[nr];
    if (k1 - k0 <= TileLds<V>::kCap) {
        constexpr int U = 4;
        for (int kb = k0 + (int)threadIdx.x; kb < k1; kb += kBlock * U) {
            int c[U];
            V v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u * kBlock;
                const int kc = k < k1 ? k : k1 - 1;
                c[u] = ld_stream(col + kc);
                v[u] = ld_stream(val + kc);
            }
            // all gathers before the first store: one latency per round
            V xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u * kBlock;
                if (k < k1) sm.prod[k - k0] = v[u] * xv[u];
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < nr) {
            const int a = sm.rp[threadIdx.x] - k0;
            const int e = sm.rp[threadIdx.x + 1] - k0;
            V s = V(0);
            for (int k = a; k < e; ++k) s += sm.prod[k];
            fn(r0 + (int)threadIdx.x, s);
        }
    } else {
        for (int i = 0; i < nr; ++i) {
            const int a = sm.rp[i];
            const int e = sm.rp[i + 1];
            const V s = block_sum(strided_dot<V, kBlock>(a + (int)threadIdx.x, e, col, val, x), sm.red);
            if (threadIdx.x == 0) fn(r0 + i, s);
            __syncthreads();
        }
    }
    __syncthreads();
}

// Standalone stream SpMV: grid = nblk logical blocks, each a contiguous chunk
// of tiles (XCD-aware).
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(int n, int R, int ntiles, int nblk,
                                                        const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const V *__restrict__ val,
                                                        const V *__restrict__ x, V *__restrict__ y)
{
    __shared__ TileLds<V> sm;
    const int j = xcd_remap(blockIdx.x, nblk);
    int t0, t1;
    block_tiles(j, nblk, ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * R;
        const int r1 = min(r0 + R, n);
        stream_tile<V>(r0, r1, rowptr, col, val, x, sm, [&](int i, V s) { y[i] = s; });
    }
}

// Vector CSR: L lanes per row, rows of a block contiguous (XCD-aware chunks).
template <class V, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_vector(int n, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const V *__restrict__ val,
                                                        const V *__restrict__ x, V *__restrict__ y,
                                                        const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    const int nb = gridDim.x;
    const int j = xcd_remap(blockIdx.x, nb);
    constexpr int RPB = kBlock / L;  // rows per block pass
    const int64_t rows_per_blk = (((int64_t)n + nb - 1) / nb + RPB - 1) / RPB * RPB;
    const int rb = (int)min((int64_t)n, (int64_t)j * rows_per_blk);
    const int re = (int)min((int64_t)n, (int64_t)(j + 1) * rows_per_blk);
    const int lane = threadIdx.x % L;
    for (int row = rb + (int)threadIdx.x / L; row < re; row += RPB) {
        const int a = rowptr[row];
        const int e = rowptr[row + 1];
        V s = strided_dot<V, L>(a + lane, e, col, val, x);
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (lane == 0) y[row] = s;
    }
}

// ------------------------------------------------------------------ SELL-64
// Sliced ELLPACK with one slice of 64 consecutive rows per wavefront: entry j
// of the slice's rows is stored contiguously (column-major inside the slice),
// so lane l streams row (64 s + l) with fully coalesced loads and no LDS, no
// barrier and no cross-lane reduction.  Columns are stored as offsets from the
// row (int16 when every |col - row| < 2^15, which holds for stencils), so an
// FP64 nonzero costs 10 bytes instead of CSR's 12 (FP32: 6 instead of 8);
// this is the index compression Challenge A7 points to.  Rows shorter than
// their slice are padded; padding is never multiplied (per-row length test).
constexpr int kSell = 64;

struct SellView {
    const int32_t *ptr;    // element offset of each slice (nslices + 1)
    const void *col;       // int16 or int32 row-relative column offsets
    const uint8_t *len;    // row lengths
    int plain;             // load policy of offsets and values, see kSellPlain64/32
};

// Load policy of the SELL entries.  A matrix whose stored entries fit well
// inside the 256 MB Infinity Cache is read with ordinary loads, so that it
// stays resident from one SpMV (or Krylov iteration) to the next; a larger
// one is streamed with nontemporal loads, which keep it from evicting the
// vectors that do fit.  One bit per value precision (FP64 / FP32 kernels).
constexpr int kSellPlain64 = 1, kSellPlain32 = 2;

// Row sum of lane `lane` of the slice starting at element b with slen
// entries per row; the row has rlen of them.  Entries in column order, FMA.
// U entries per round: the round's offsets and values are loaded together,
// then all U gathers of x are issued before the first FMA, so a round costs
// one memory latency, not U.  Entries past the slice width repeat its last
// entry and padding has offset 0, so every gather reads a valid element of
// x; only the row's own entries are multiplied.  U is chosen per matrix from
// the widest slice (7 for a 7-point stencil: no wasted load).
template <class V, class CI, int U, bool NT>
__device__ __forceinline__ V sell_row(const SellView &sv, const V *__restrict__ val,
                                      const V *__restrict__ x, int32_t b, int slen, int rlen,
                                      int lane, int row)
{
    const CI *__restrict__ col = reinterpret_cast<const CI *>(sv.col) + b + lane;
    const V *__restrict__ v = val + b + lane;
    V acc = V(0);
    for (int j0 = 0; j0 < slen; j0 += U) {
        CI c[U];
        V a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u < slen ? j0 + u : slen - 1;
            c[u] = NT ? ld_stream(col + (size_t)j * kSell) : col[(size_t)j * kSell];
            a[u] = NT ? ld_stream(v + (size_t)j * kSell) : v[(size_t)j * kSell];
        }
        V xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[row + (int)c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < rlen) acc = fma(a[u], xv[u], acc);
    }
    return acc;
}

// Slices s, s + stride, ... below ceil(n/64), one per wavefront at a time;
// fn(row, y) is called by the lane that owns row (< n).  Callers pass
// s = 4 * (physical block) + wave and stride = 4 * (blocks), so the slices in
// flight at any moment are adjacent in memory (one DRAM stream front rather
// than one per block).  The first slice's header is loaded before go() is
// asked whether to run (go holds no barrier: waves may own different counts).
template <class V, class CI, int U, bool NT, class Go, class Fn>
__device__ __forceinline__ void sell_slices_run(int n, int s, int stride, const SellView &sv,
                                                const V *__restrict__ val, const V *__restrict__ x,
                                                Go &&go, Fn &&fn)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int ns = (n + kSell - 1) / kSell;
    int32_t b = 0, e = 0;
    int rlen = 0;
    if (s < ns) {
        b = sv.ptr[s];
        e = sv.ptr[s + 1];
        const int row = s * kSell + lane;
        rlen = row < n ? sv.len[row] : 0;
    }
    if (!go()) return;
    while (s < ns) {
        const int row = s * kSell + lane;
        const int slen = (e - b) / kSell;
        if (row < n) fn(row, sell_row<V, CI, U, NT>(sv, val, x, b, slen, rlen, lane, row));
        s += stride;
        if (s >= ns) break;
        b = sv.ptr[s];
        e = sv.ptr[s + 1];
        const int nrow = s * kSell + lane;
        rlen = nrow < n ? sv.len[nrow] : 0;
    }
}

// The load policy is chosen here, around the whole slice loop, so that the
// two variants stay separate code (a branch inside the round lets the
// compiler merge the loads and drop the nontemporal hint).
template <class V, class CI, int U, class Go, class Fn>
__device__ __forceinline__ void sell_slices(int n, int s, int stride, const SellView &sv,
                                            const V *__restrict__ val, const V *__restrict__ x,
                                            Go &&go, Fn &&fn)
{
    if (sv.plain & (sizeof(V) == 4 ? kSellPlain32 : kSellPlain64))
        sell_slices_run<V, CI, U, false>(n, s, stride, sv, val, x, go, fn);
    else
        sell_slices_run<V, CI, U, true>(n, s, stride, sv, val, x, go, fn);
}

// Standalone SELL SpMV; the grid has up to one wavefront per slice.
template <class V, class CI, int U>
__global__ __launch_bounds__(kBlock) void k_spmv_sell(int n, SellView sv, const V *__restrict__ val,
                                                      const V *__restrict__ x, V *__restrict__ y)
{
    sell_slices<V, CI, U>(n, blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave,
                          gridDim.x * (kBlock / kWave), sv, val, x, [] { return true; },
                          [&](int i, V s) { y[i] = s; });
}

// Widths U the SELL kernels are built for, and the launch helper: calls
// f(std::integral_constant<int, U>) for the handle's U.
constexpr int kSellUMin = 4, kSellUMax = 9;

template <class F>
inline void with_sell_u(int u, F &&f)
{
    switch (u) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
    }
}

// U for a matrix whose widest slice has w entries per row: w itself up to 9
// (at least 4), else the U in [5, 9] that wastes the fewest loads.
inline int pick_sell_u(int w)
{
    if (w <= kSellUMax) return w < kSellUMin ? kSellUMin : w;
    int best = 8, waste = 1 << 30;
    for (int u = kSellUMax; u >= 5; --u) {
        const int wst = (w + u - 1) / u * u - w;
        if (wst < waste) { waste = wst; best = u; }
    }
    return best;
}

// Layout fill: one lane per row writes its entries and the slice padding.
template <class CI>
__global__ void k_sell_fill(int n, const int32_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, const double *__restrict__ val,
                            const int32_t *__restrict__ sptr, CI *__restrict__ scol,
                            double *__restrict__ sval, uint8_t *__restrict__ slen)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = i / kSell, lane = i % kSell;
        const int b = sptr[s];
        const int len = (sptr[s + 1] - b) / kSell;
        const int a = rowptr[i], e = rowptr[i + 1];
        slen[i] = (uint8_t)(e - a);
        for (int j = 0; j < len; ++j) {
            const size_t d = (size_t)b + (size_t)j * kSell + lane;
            const bool real = a + j < e;
            scol[d] = real ? (CI)(col[a + j] - i) : (CI)0;
            sval[d] = real ? val[a + j] : 0.0;
        }
    }
}

// ------------------------------------------------------------------ merge path
// Split point of diagonal d on the merge of row ends (rowptr[i+1]) with
// nonzero indices: (i, d - i) with i the number of completed rows.
static __global__ void k_merge_partition(int n, int nnz, const int32_t *__restrict__ rowptr, int ntiles,
                                  int32_t *__restrict__ tile_row, int32_t *__restrict__ tile_k)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    const int64_t total = (int64_t)n + nnz;
    const int64_t d64 = min((int64_t)t * kMergeItems, total);
    const int d = (int)d64;
    int lo = d > nnz ? d - nnz : 0;
    int hi = d < n ? d : n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowptr[mid + 1] <= d - mid - 1) lo = mid + 1; else hi = mid;
    }
    tile_row[t] = lo;
    tile_k[t] = d - lo;
}

template <class V>
struct MergeLds {
    V prod[kMergeItems];
    int32_t rend[kMergeItems + 1];
    V sv[2][kBlock];
    int32_t sk[kBlock];
};

// Merge-path tile t, computed by one block.  Rows that end inside the tile
// are written (complete rows directly, rows split across lanes after a
// segmented scan); the partial of the row still open at the tile end goes to
// carry_{row,val}.
template <class V>
__device__ __forceinline__ void merge_tile(int t, int n, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, const V *__restrict__ val,
                                           const V *__restrict__ x, V *__restrict__ y,
                                           const int32_t *__restrict__ tile_row,
                                           const int32_t *__restrict__ tile_k, int32_t *__restrict__ carry_row,
                                           V *__restrict__ carry_val, MergeLds<V> &sm)
{
    const int i0 = tile_row[t], k0 = tile_k[t];
    const int i1 = tile_row[t + 1], k1 = tile_k[t + 1];
    const int nrows = i1 - i0;   // row ends inside the tile
    const int nk = k1 - k0;      // nonzeros inside the tile
    for (int r = threadIdx.x; r <= nrows; r += kBlock)
        sm.rend[r] = (i0 + r < n) ? rowptr[i0 + r + 1] - k0 : nk;
    {
        constexpr int U = 4;
        for (int kb = k0 + (int)threadIdx.x; kb < k1; kb += kBlock * U) {
            int c[U];
            V v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u * kBlock;
                const int kc = k < k1 ? k : k1 - 1;
                c[u] = ld_stream(col + kc);
                v[u] = ld_stream(val + kc);
            }
            V xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u * kBlock;
                if (k < k1) sm.prod[k - k0] = v[u] * xv[u];
            }
        }
    }
    __syncthreads();
    // this lane's start on the tile-local merge path
    const int total = nrows + nk;
    const int dd = min((int)threadIdx.x * kMergeIpt, total);
    int lo = dd > nk ? dd - nk : 0;
    int hi = dd < nrows ? dd : nrows;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sm.rend[mid] <= dd - mid - 1) lo = mid + 1; else hi = mid;
    }
    int r = lo;
    int kk = dd - lo;
    const int items = min(kMergeIpt, total - dd);
    V acc = V(0);
    V head = V(0);
    int head_row = -1;
    for (int it = 0; it < items; ++it) {
        if (kk < nk && kk < sm.rend[r]) {
            acc += sm.prod[kk];
            ++kk;
        } else {
            if (r >= nrows || i0 + r >= n) break;  // never taken on a consistent path
            if (head_row < 0) { head = acc; head_row = r; }
            else y[i0 + r] = acc;
            acc = V(0);
            ++r;
        }
    }
    // inclusive segmented scan of (carry row, carry value) over the lanes
    sm.sk[threadIdx.x] = r;
    sm.sv[0][threadIdx.x] = acc;
    __syncthreads();
    int cur = 0;
#pragma unroll
    for (int off = 1; off < kBlock; off <<= 1) {
        V v = sm.sv[cur][threadIdx.x];
        if ((int)threadIdx.x >= off && sm.sk[threadIdx.x - off] == r)
            v = sm.sv[cur][threadIdx.x - off] + v;
        sm.sv[cur ^ 1][threadIdx.x] = v;
        cur ^= 1;
        __syncthreads();
    }
    if (head_row >= 0) {
        const V cin = threadIdx.x > 0 ? sm.sv[cur][threadIdx.x - 1] : V(0);
        y[i0 + head_row] = cin + head;
    }
    if (threadIdx.x == kBlock - 1) {
        carry_row[t] = i0 + r;
        carry_val[t] = sm.sv[cur][threadIdx.x];
    }
}

// One merge-path tile per block.
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_merge(int n, int nnz,
                                                       const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col,
                                                       const V *__restrict__ val,
                                                       const V *__restrict__ x, V *__restrict__ y,
                                                       const int32_t *__restrict__ tile_row,
                                                       const int32_t *__restrict__ tile_k,
                                                       int32_t *__restrict__ carry_row,
                                                       V *__restrict__ carry_val,
                                                       const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    (void)nnz;
    __shared__ MergeLds<V> sm;
    merge_tile<V>(blockIdx.x, n, rowptr, col, val, x, y, tile_row, tile_k, carry_row, carry_val, sm);
}

// Adds the carries of rows that span tiles, in tile order; one lane per chain.
template <class V>
__global__ void k_merge_fixup(int n, int ntiles, const int32_t *__restrict__ carry_row,
                              const V *__restrict__ carry_val, V *__restrict__ y,
                              const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int c = carry_row[t];
    if (c >= n) return;
    if (t > 0 && carry_row[t - 1] == c) return;
    V s = carry_val[t];
    for (int u = t + 1; u < ntiles && carry_row[u] == c; ++u) s += carry_val[u];
    y[c] += s;
}

}  // namespace spk
