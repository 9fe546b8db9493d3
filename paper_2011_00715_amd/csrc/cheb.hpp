// Jacobi-preconditioned Chebyshev smoother kernels (the multigrid smoother of
// Sec. 5.3).  The three-term recurrence has coefficients known before the
// first step, so each step is one pass with no inner product:
//   x += d_k;  r -= A d_k;  d_{k+1} = c1 d_k + c2 D^-1 r
// For the SELL and stream families that pass is a single kernel (the update
// runs in the SpMV's row epilogue); d is double-buffered because every block
// gathers d_k while it writes d_{k+1} for its own rows.
#pragma once

#include "spmv.hpp"

namespace spk {

template <class V>
struct ChebStep {
    const V *dk;  // d_k (gathered)
    V *dn;        // d_{k+1}, or null on the last step
    V *r;
    V *x;
    const V *dinv;
    V c1, c2;
    const SysState *gate = nullptr;  // inside a captured solve: run only while it iterates
};

__device__ __forceinline__ bool cheb_go(const SysState *gate)
{
    return !gate || gate_open(gate, kGateInner64);
}

template <class V>
__device__ __forceinline__ void cheb_row(const ChebStep<V> &c, int i, V y)
{
    const V ri = c.r[i] - y;
    c.r[i] = ri;
    const V di = c.dk[i];
    c.x[i] = c.x[i] + di;
    if (c.dn) c.dn[i] = fma(c.c1, di, c.c2 * (c.dinv[i] * ri));
}

template <class V, class CI, int U>
__global__ __launch_bounds__(kBlock) void k_cheb_sell(int n, SellView sv, const V *__restrict__ val,
                                                      ChebStep<V> c)
{
    sell_slices<V, CI, U>(n, blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave,
                          gridDim.x * (kBlock / kWave), sv, val, c.dk, [&] { return cheb_go(c.gate); },
                          [&](int i, V y) { cheb_row(c, i, y); });
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_cheb_stream(int n, int R, int ntiles, int nblk,
                                                        const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const V *__restrict__ val, ChebStep<V> c)
{
    if (!cheb_go(c.gate)) return;
    __shared__ TileLds<V> sm;
    const int j = xcd_remap(blockIdx.x, nblk);
    int t0, t1;
    block_tiles(j, nblk, ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const int r0 = t * R;
        const int r1 = min(r0 + R, n);
        stream_tile<V>(r0, r1, rowptr, col, val, c.dk, sm, [&](int i, V y) { cheb_row(c, i, y); });
    }
}

// Other families: y = A d_k was written by the standalone SpMV.
template <class V>
__global__ void k_cheb_update(int n, const V *__restrict__ y, ChebStep<V> c)
{
    if (!cheb_go(c.gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        cheb_row(c, i, y[i]);
}

// r = b - A x (ax holds A x; null for x = 0, which is then stored), and
// d_0 = D^-1 r / theta.  B is the right-hand side's type: a double b with
// float vectors also stores the rounded b into bcopy (the FP32 cycle of a
// multigrid preconditioner inside FP64 CG).
template <class V, class B>
__global__ void k_cheb_init(int n, const B *__restrict__ b, const V *__restrict__ ax, V *__restrict__ x,
                            V *__restrict__ r, V *__restrict__ d0, const V *__restrict__ dinv, V inv_theta,
                            const SysState *gate, V *__restrict__ bcopy)
{
    if (!cheb_go(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const V bi = (V)b[i];
        if (bcopy) bcopy[i] = bi;
        V ri;
        if (ax) ri = bi - ax[i];
        else {
            ri = bi;
            x[i] = V(0);
        }
        r[i] = ri;
        d0[i] = dinv[i] * ri * inv_theta;
    }
}

// The last step without a residual: x += d.
template <class V>
__global__ void k_cheb_last(int n, const V *__restrict__ d, V *__restrict__ x, const SysState *gate)
{
    if (!cheb_go(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = x[i] + d[i];
}

}  // namespace spk
