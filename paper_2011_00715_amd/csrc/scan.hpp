// Exclusive prefix sum of int32 counts into int32 offsets out[0..n], with
// out[n] the total (setup work: building row pointers of derived layouts).
// Three launches on the caller's stream: every block sums a contiguous chunk
// of the counts, one block scans the chunk sums, then every block scans its
// chunk again from its offset, a tile of kBlock * kScanIpt counts at a time.
// The total must fit int32 (callers check it: the layouts index int32).
#pragma once

#include "common.hpp"

namespace spk {

constexpr int kScanMaxBlocks = 1024;
constexpr int kScanIpt = 4;  // consecutive counts per thread in a tile
constexpr int kScanTile = kBlock * kScanIpt;

// Exclusive scan of one value per thread over the block (thread order);
// `total` receives the block's sum.  sh holds kBlock / kWave values.
__device__ __forceinline__ long long block_excl_scan(long long v, long long *sh, long long &total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    long long x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const long long y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) sh[w] = x;
    __syncthreads();
    long long before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        if (i < w) before += sh[i];
        all += sh[i];
    }
    total = all;
    return before + x - v;
}

// Chunk of block j: [j * chunk, min(n, (j + 1) * chunk)).
static __global__ __launch_bounds__(kBlock) void k_scan_sums(int64_t n, int64_t chunk,
                                                             const int32_t *__restrict__ cnt,
                                                             long long *__restrict__ bsum)
{
    __shared__ long long sh[kBlock / kWave];
    const int64_t b = (int64_t)blockIdx.x * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    long long s = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) s += cnt[i];
    long long total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// bsum[0..g) -> exclusive offsets, bsum[g] = total (one block).
static __global__ __launch_bounds__(kBlock) void k_scan_top(int g, long long *__restrict__ bsum)
{
    __shared__ long long sh[kBlock / kWave];
    const int per = (g + kBlock - 1) / kBlock;
    const int b = min(g, (int)threadIdx.x * per), e = min(g, b + per);
    long long s = 0;
    for (int i = b; i < e; ++i) s += bsum[i];
    long long total;
    long long run = block_excl_scan(s, sh, total);
    __syncthreads();
    for (int i = b; i < e; ++i) {
        const long long v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) bsum[g] = total;
}

static __global__ __launch_bounds__(kBlock) void k_scan_apply(int64_t n, int64_t chunk, int g,
                                                              const int32_t *__restrict__ cnt,
                                                              const long long *__restrict__ bsum,
                                                              int32_t *__restrict__ out)
{
    __shared__ long long sh[kBlock / kWave];
    const int64_t b = (int64_t)blockIdx.x * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    long long carry = bsum[blockIdx.x];
    for (int64_t t = b; t < e; t += kScanTile) {
        const int64_t i0 = t + (int64_t)threadIdx.x * kScanIpt;
        int32_t v[kScanIpt];
        long long s = 0;
#pragma unroll
        for (int u = 0; u < kScanIpt; ++u) {
            v[u] = i0 + u < e ? cnt[i0 + u] : 0;
            s += v[u];
        }
        long long total;
        long long run = carry + block_excl_scan(s, sh, total);
#pragma unroll
        for (int u = 0; u < kScanIpt; ++u) {
            if (i0 + u < e) out[i0 + u] = (int32_t)run;
            run += v[u];
        }
        carry += total;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int32_t)bsum[g];
}

// Blocks of a scan over n counts; `bsum` needs scan_blocks(n) + 1 entries.
inline int scan_blocks(int64_t n)
{
    int64_t g = (n + kScanTile - 1) / kScanTile;
    if (g > kScanMaxBlocks) g = kScanMaxBlocks;
    return (int)(g < 1 ? 1 : g);
}

inline hipError_t scan_exclusive(int64_t n, const int32_t *cnt, int32_t *out, long long *bsum, hipStream_t s)
{
    const int g = scan_blocks(n);
    const int64_t chunk = (n + g - 1) / g;
    hipLaunchKernelGGL(k_scan_sums, dim3(g), dim3(kBlock), 0, s, n, chunk, cnt, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, g, bsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(g), dim3(kBlock), 0, s, n, chunk, g, cnt, (const long long *)bsum, out);
    return hipGetLastError();
}

}  // namespace spk
