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
// Sliced ELLPACK with one slice of 64 consecutive rows per wavefront: lane l
// streams row (64 s + l) with coalesced loads and no LDS, no barrier and no
// cross-lane reduction.  Inside a slice of width w (its longest row) the
// entries are stored in pairs: entries 2p and 2p + 1 of lane l sit next to
// each other at element 128 p + 2 l, so one 8- or 16-byte load per lane
// fetches two entries (a wavefront load moves 512 B / 1 KB instead of
// 128 B / 512 B: fewer memory instructions per byte, 11 % faster on the
// 27-point 160^3 product), and the last entry of an odd width sits at
// 128 (w / 2) + l.  Columns are stored as offsets from the row (int16 when
// every |col - row| < 2^15, which holds for stencils), so an FP64 nonzero
// costs 10 bytes instead of CSR's 12 (FP32: 6 instead of 8); this is the
// index compression Challenge A7 points to.  Rows shorter than their slice
// are padded; padding is never multiplied (per-row length test).
//
// Shared offsets (stencil-like matrices): when the rows of every slice use
// between them at most 32 distinct column offsets, each slice stores its
// sorted offset list once (int32, one per position) and each row a 32-bit
// mask of the positions it occupies, the other positions holding zeros.
// An FP64 nonzero then costs 8 bytes plus 4 per row and 4 per slice
// position (FP32: 4), a row's entries still sit in column order and only
// masked positions are multiplied, so the sums are the same as with
// per-lane offsets.  Gathers of unmasked positions read a clamped valid
// element of x and are discarded.
constexpr int kSell = 64;
constexpr int kSellSharedMax = 32;

// Element of entry k of lane `lane` in a slice of w entries per row,
// relative to the slice's first element.
__host__ __device__ __forceinline__ size_t sell_pos(int k, int w, int lane)
{
    return k < (w & ~1) ? (size_t)(k >> 1) * (2 * kSell) + 2 * lane + (k & 1)
                        : (size_t)(w >> 1) * (2 * kSell) + lane;
}

// Two-element vectors for the paired loads.
template <class T> struct Pair2;
template <> struct Pair2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Pair2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Pair2<int16_t> { typedef short type __attribute__((ext_vector_type(2))); };
template <> struct Pair2<int32_t> { typedef int type __attribute__((ext_vector_type(2))); };

struct SellView {
    const int32_t *ptr;    // element offset of each slice (nslices + 1)
    const void *col;       // int16 or int32 row-relative column offsets (per entry, or
                           // per slice position with shared offsets)
    const uint8_t *len;    // row lengths (rows of at most 255 entries), or null
    int plain;             // load policy of offsets and values, see kSellPlain64/32
    const uint16_t *len16; // row lengths when some row has more than 255 entries
    const int32_t *perm;   // SELL-C-sigma: matrix row of each sorted position, or null
    const uint32_t *mask;  // shared offsets: per-row position masks (col then holds
                           // each slice's int32 offsets at element ptr[s] / 64), or null
};

// Load policy of the SELL entries.  A matrix whose stored entries fit well
// inside the 256 MB Infinity Cache is read with ordinary loads, so that it
// stays resident from one SpMV (or Krylov iteration) to the next; a larger
// one is streamed with nontemporal loads, which keep it from evicting the
// vectors that do fit.  One bit per value precision (FP64 / FP32 kernels).
constexpr int kSellPlain64 = 1, kSellPlain32 = 2;

template <bool NT, class T>
__device__ __forceinline__ T sell_ld(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Row sum of lane `lane` of the slice starting at element b with slen
// entries per row; the row has rlen of them.  Entries in column order, FMA.
// UP pairs per round: the round's offset and value pairs are loaded
// together, then all 2 UP gathers of x are issued before the first FMA, so
// a round costs one memory latency.  Pairs past the slice width repeat its
// last pair and padding has offset 0, so every gather reads a valid element
// of x; only the row's own entries are multiplied.  UP is chosen per matrix
// from the widest slice (3 for a 7-point stencil: one round and the tail).
// gat(j) is the gathered operand at column j: x[j] for a plain product; the
// fused PCG kernels form p = z + beta p there.
//
// SH (shared offsets, CI = int32): the offsets come from the slice's list
// (wave-uniform, scalar loads), rlen is the row's position mask, and gathered
// columns are clamped into [0, n) for the positions the row does not use.
template <class V, class CI, int UP, bool NT, bool SH, class G>
__device__ __forceinline__ V sell_row(const SellView &sv, const V *__restrict__ val, G &&gat,
                                      int32_t b, int slen, int rlen, int lane, int row, int n)
{
    static_assert(!SH || std::is_same<CI, int32_t>::value, "shared offsets are int32");
    using CP = typename Pair2<CI>::type;
    using VP = typename Pair2<V>::type;
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
            return sell_ld<NT>(cp + (size_t)p * kSell);
        }
    };
    auto column = [&](int off) -> int {
        if constexpr (SH) return min(max(row + off, 0), n - 1);
        else return row + off;
    };
    auto real = [&](int k) -> bool {
        if constexpr (SH) return ((unsigned)rlen >> k) & 1u;
        else return k < rlen;
    };
    const int np = slen >> 1;
    // the odd last entry is loaded first and gathered with the first round,
    // so an odd width costs no extra memory round trip; it is added last
    const bool odd = slen & 1;
    CI ct = CI(0);
    V at = V(0), xt = V(0);
    if (odd) {
        const size_t t = (size_t)b + (size_t)np * (2 * kSell) + lane;
        if constexpr (SH) ct = ou[2 * np];
        else ct = sell_ld<NT>(reinterpret_cast<const CI *>(sv.col) + t);
        at = sell_ld<NT>(val + t);
    }
    V acc = V(0);
    for (int p0 = 0; p0 < np; p0 += UP) {
        CP c[UP];
        VP a[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int p = p0 + u < np ? p0 + u : np - 1;
            c[u] = offsets(p);
            a[u] = sell_ld<NT>(vp + (size_t)p * kSell);
        }
        V xv[2 * UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            xv[2 * u] = gat(column((int)c[u].x));
            xv[2 * u + 1] = gat(column((int)c[u].y));
        }
        if (p0 == 0 && odd) xt = gat(column((int)ct));
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int k = 2 * (p0 + u);
            if (p0 + u < np) {
                if (real(k)) acc = fma(a[u].x, xv[2 * u], acc);
                if (real(k + 1)) acc = fma(a[u].y, xv[2 * u + 1], acc);
            }
        }
    }
    if (odd) {
        if (np == 0) xt = gat(column((int)ct));
        if (real(slen - 1)) acc = fma(at, xt, acc);
    }
    return acc;
}

// Slices s, s + stride, ... below ceil(n/64), one per wavefront at a time;
// fn(row, y) is called by the lane that owns row (< n).  Callers pass
// s = 4 * (physical block) + wave and stride = 4 * (blocks), so the slices in
// flight at any moment are adjacent in memory (one DRAM stream front rather
// than one per block).  The first slice's header is loaded before go() is
// asked whether to run (go holds no barrier: waves may own different counts).
template <class V, class CI, int U, bool NT, bool SH, class G, class Go, class Fn>
__device__ __forceinline__ void sell_slices_run(int n, int s, int stride, const SellView &sv,
                                                const V *__restrict__ val, G &&gat, Go &&go, Fn &&fn)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int ns = (n + kSell - 1) / kSell;
    // position j = 64 s + lane of the layout holds matrix row perm[j]
    // (SELL-C-sigma) or row j; its length is in len or len16 (its position
    // mask in mask with shared offsets)
    auto head = [&](int j, int &rlen, int &row) {
        if constexpr (SH) rlen = j < n ? (int)sv.mask[j] : 0;
        else rlen = j < n ? (sv.len16 ? (int)sv.len16[j] : (int)sv.len[j]) : 0;
        row = j < n && sv.perm ? sv.perm[j] : j;
    };
    int32_t b = 0, e = 0;
    int rlen = 0, row = 0;
    if (s < ns) {
        b = sv.ptr[s];
        e = sv.ptr[s + 1];
        head(s * kSell + lane, rlen, row);
    }
    if (!go()) return;
    while (s < ns) {
        const int slen = (e - b) / kSell;
        if (s * kSell + lane < n) fn(row, sell_row<V, CI, U, NT, SH>(sv, val, gat, b, slen, rlen, lane, row, n));
        s += stride;
        if (s >= ns) break;
        b = sv.ptr[s];
        e = sv.ptr[s + 1];
        head(s * kSell + lane, rlen, row);
    }
}

// The load policy is chosen here, around the whole slice loop, so that the
// two variants stay separate code (a branch inside the round lets the
// compiler merge the loads and drop the nontemporal hint).
template <class V, class CI, int U, class G, class Go, class Fn>
__device__ __forceinline__ void sell_slices_g(int n, int s, int stride, const SellView &sv,
                                              const V *__restrict__ val, G &&gat, Go &&go, Fn &&fn)
{
    const bool plain = sv.plain & (sizeof(V) == 4 ? kSellPlain32 : kSellPlain64);
    if constexpr (std::is_same<CI, int32_t>::value) {
        if (sv.mask) {
            if (plain) sell_slices_run<V, CI, U, false, true>(n, s, stride, sv, val, gat, go, fn);
            else sell_slices_run<V, CI, U, true, true>(n, s, stride, sv, val, gat, go, fn);
            return;
        }
    }
    if (plain) sell_slices_run<V, CI, U, false, false>(n, s, stride, sv, val, gat, go, fn);
    else sell_slices_run<V, CI, U, true, false>(n, s, stride, sv, val, gat, go, fn);
}

// The plain product: the gathered operand is x.
template <class V, class CI, int U, class Go, class Fn>
__device__ __forceinline__ void sell_slices(int n, int s, int stride, const SellView &sv,
                                            const V *__restrict__ val, const V *__restrict__ x,
                                            Go &&go, Fn &&fn)
{
    sell_slices_g<V, CI, U>(n, s, stride, sv, val, [x](int j) { return x[j]; }, go, fn);
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

// Pairs per round UP the SELL kernels are built for, and the launch
// helper: calls f(std::integral_constant<int, UP>) for the handle's UP.
template <class F>
inline void with_sell_u(int u, F &&f)
{
    switch (u) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 13: f(std::integral_constant<int, 13>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
    }
}

// UP for a matrix whose widest slice has w entries per row: the fewest
// rounds, then the fewest repeated pairs, among the built values (2 below 3
// pairs).  One round beats register room: the 27-point rows (13 pairs) in
// one round of 13 (FP64 140 VGPRs, 3 wavefronts per SIMD) took the 160^3
// PCG product from 225.7 to 216.3 us against two rounds of 7 (95 VGPRs,
// 5 per SIMD); rounds of 5 and 4 (6 and 7 per SIMD) took 231.7 and 233.1.
inline int pick_sell_u(int w)
{
    const int np = w >> 1;
    if (np <= 2) return 2;
    constexpr int kBuilt[] = {3, 4, 5, 6, 7, 9, 13};
    int best = 13, rounds = 1 << 30, waste = 1 << 30;
    for (const int u : kBuilt) {
        const int r = (np + u - 1) / u, wst = r * u - np;
        if (r < rounds || (r == rounds && wst < waste)) { best = u; rounds = r; waste = wst; }
    }
    return best;
}

// Layout fill: one lane per layout position j writes the entries of its
// matrix row (perm[j], or j) and the slice padding; the row's length goes to
// slen (one byte) or, for rows longer than 255 entries, to slen16.
template <class CI>
__global__ void k_sell_fill(int n, const int32_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, const double *__restrict__ val,
                            const int32_t *__restrict__ sptr, const int32_t *__restrict__ perm,
                            CI *__restrict__ scol, double *__restrict__ sval, uint8_t *__restrict__ slen,
                            uint16_t *__restrict__ slen16)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = i / kSell, lane = i % kSell;
        const int r = perm ? perm[i] : i;
        const int b = sptr[s];
        const int len = (sptr[s + 1] - b) / kSell;
        const int a = rowptr[r], e = rowptr[r + 1];
        if (slen16) slen16[i] = (uint16_t)(e - a);
        else slen[i] = (uint8_t)(e - a);
        for (int j = 0; j < len; ++j) {
            const size_t d = (size_t)b + sell_pos(j, len, lane);
            const bool real = a + j < e;
            scol[d] = real ? (CI)(col[a + j] - r) : (CI)0;
            sval[d] = real ? val[a + j] : 0.0;
        }
    }
}

// Shared-offset fill: row i (no permutation) has the positions of the set
// bits of mask[i] in its slice's offset list, in column order; its k-th
// entry goes to the position of the k-th set bit, the other positions get
// zeros.
static __global__ void k_sell_fill_shared(int n, const int32_t *__restrict__ rowptr,
                                          const double *__restrict__ val, const int32_t *__restrict__ sptr,
                                          const uint32_t *__restrict__ mask, double *__restrict__ sval)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = i / kSell, lane = i % kSell;
        const int b = sptr[s];
        const int w = (sptr[s + 1] - b) / kSell;
        const uint32_t m = mask[i];
        int k = rowptr[i];
        for (int j = 0; j < w; ++j) {
            const bool real = (m >> j) & 1u;
            sval[(size_t)b + sell_pos(j, w, lane)] = real ? val[k] : 0.0;
            k += real;
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
