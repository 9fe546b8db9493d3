// Column-sliced CSR SpMV for matrices whose columns scatter over a vector
// larger than one XCD's L2 (the C4-type power-law matrices: x of 32 MB,
// uniform random columns).
//
// The columns are split into kSlices = 8 equal ranges.  The entries of row i
// whose columns fall in range s form row s*n + i of a CSR matrix with
// kSlices*n rows (entries keep their global column and their order).  One
// launch computes all kSlices partial products: block b takes slice b % 8,
// and the dispatcher places block b on XCD b % 8, so each XCD gathers only
// its 4 MB eighth of x, which stays in that XCD's 4 MB L2 instead of being
// fetched line by line from the Infinity Cache (the unsliced kernels fetch a
// 128-byte line per 8-byte gather).  A second pass sums the eight partial
// products of each row in slice order, so the result is reproducible bit for
// bit.
#pragma once

#include "spmv.hpp"

namespace spk {

constexpr int kSlices = kXcd;

__device__ __forceinline__ int slice_of(int c, int n) { return (int)(((int64_t)c * kSlices) / n); }

// cnt[s * n + i] = entries of row i in column range s.  Rows need not be
// sorted: every entry is counted where its column falls.
static __global__ void k_xs_count(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                  int32_t *__restrict__ cnt)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c[kSlices] = {};
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int s = slice_of(col[k], n);
#pragma unroll
            for (int t = 0; t < kSlices; ++t) c[t] += t == s;
        }
#pragma unroll
        for (int s = 0; s < kSlices; ++s) cnt[(size_t)s * n + i] = c[s];
    }
}

// Scatter each row's entries to its slices' rows (xptr: exclusive scan of
// cnt), keeping their order within the row.
static __global__ void k_xs_fill(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                 const double *__restrict__ val, const int32_t *__restrict__ xptr,
                                 int32_t *__restrict__ xcol, double *__restrict__ xval)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int d[kSlices];
#pragma unroll
        for (int s = 0; s < kSlices; ++s) d[s] = xptr[(size_t)s * n + i];
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int c = col[k];
            const int s = slice_of(c, n);
            int pos = 0;
#pragma unroll
            for (int t = 0; t < kSlices; ++t)
                if (t == s) pos = d[t]++;
            xcol[pos] = c;
            xval[pos] = val[k];
        }
    }
}

// part[s * n + i] = (A_s x)_i with L lanes per row; the grid is a multiple of
// kSlices and block b serves slice b % kSlices.
template <class V, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_xs(int n, const int32_t *__restrict__ xptr,
                                                    const int32_t *__restrict__ xcol, const V *__restrict__ xval,
                                                    const V *__restrict__ x, V *__restrict__ part,
                                                    const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    const int s = blockIdx.x % kSlices;
    const int nb = gridDim.x / kSlices;
    const int g = blockIdx.x / kSlices;
    constexpr int RPB = kBlock / L;
    const int64_t rows_per_blk = (((int64_t)n + nb - 1) / nb + RPB - 1) / RPB * RPB;
    const int rb = (int)min((int64_t)n, (int64_t)g * rows_per_blk);
    const int re = (int)min((int64_t)n, (int64_t)(g + 1) * rows_per_blk);
    const int32_t *rp = xptr + (size_t)s * n;
    V *y = part + (size_t)s * n;
    const int lane = threadIdx.x % L;
    for (int row = rb + (int)threadIdx.x / L; row < re; row += RPB) {
        V acc = strided_dot<V, L>(rp[row] + lane, rp[row + 1], xcol, xval, x);
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
        if (lane == 0) y[row] = acc;
    }
}

// The stacked slices as one merge path (for skewed rows, whose long slice
// rows leave lane-per-row groups unbalanced): the tiles whose start lies in
// slice s are tiles slice_tile[s] .. slice_tile[s+1]-1, and block b takes the
// (b / 8)-th of them for s = b % 8, so a slice's tiles stay on its XCD.
template <class V>
__global__ __launch_bounds__(kBlock) void k_spmv_xs_merge(int rows, const int32_t *__restrict__ xptr,
                                                          const int32_t *__restrict__ xcol,
                                                          const V *__restrict__ xval, const V *__restrict__ x,
                                                          V *__restrict__ part, const int32_t *__restrict__ tile_row,
                                                          const int32_t *__restrict__ tile_k,
                                                          int32_t *__restrict__ carry_row, V *__restrict__ carry_val,
                                                          const int32_t *__restrict__ slice_tile,
                                                          const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    const int s = blockIdx.x % kSlices;
    const int t = slice_tile[s] + (int)blockIdx.x / kSlices;
    if (t >= slice_tile[s + 1]) return;
    __shared__ MergeLds<V> sm;
    merge_tile<V>(t, rows, xptr, xcol, xval, x, part, tile_row, tile_k, carry_row, carry_val, sm);
}

// y_i = sum over s = 0..7 of part[s * n + i], in that order.
template <class V>
__global__ __launch_bounds__(kBlock) void k_xs_reduce(int n, const V *__restrict__ part, V *__restrict__ y,
                                                      const SysState *gate_st, int gate_mode)
{
    if (gate_st && !gate_open(gate_st, gate_mode)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        V v[kSlices];
#pragma unroll
        for (int s = 0; s < kSlices; ++s) v[s] = ld_stream(part + (size_t)s * n + i);
        V t = v[0];
#pragma unroll
        for (int s = 1; s < kSlices; ++s) t += v[s];
        y[i] = t;
    }
}

}  // namespace spk
