// Internal definitions shared by the HIP translation units of libspk.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "spk.h"

namespace spk {

// ------------------------------------------------------------------ launch shape
constexpr int kBlock = 256;              // threads per block (4 wavefronts of 64)
constexpr int kWave = 64;
constexpr int kXcd = 8;                  // MI355X: 8 accelerator complex dies
constexpr int kMaxBlocksSingle = 2048;   // 256 CUs x 8 resident blocks
constexpr int kTileBytes = 16384;        // LDS bytes for one tile of products
constexpr int kMergeItems = 2048;        // merge-path items per tile (256 x 8)
constexpr int kMergeIpt = kMergeItems / kBlock;

// ------------------------------------------------------------------ solver state
// Phase of a system inside a solve (FP64 solves stay in kPhaseInner).
enum : int32_t {
    kPhaseInner = 0,   // Krylov iterations (FP64, or FP32 inner for mixed)
    kPhaseResid = 1,   // mixed: form r = b - A x in FP64
    kPhaseSetup = 2,   // mixed: scale/cast r, start the FP32 inner solve
    kPhaseUpdate = 3,  // mixed: x += s d, then kPhaseResid
};

// Slots of the per-block partial sums (each B doubles).
enum { kPartPq = 0, kPartRz = 1, kPartRr = 2, kPartBb = 3, kNumPart = 4 };

// Device-resident scalars of one system.  Written by one block only: the
// one-block finalize kernels, the one-thread init kernel, block 0 of the
// PCG update pass (the snap_* fields) and block 0 of the p/x pass (the rest);
// no kernel's blocks read a field that a block of the same kernel writes.
// Every later kernel turns into a no-op once `status` is no longer
// SPK_RUNNING.
struct SysState {
    int32_t status;       // SPK_RUNNING or a reason
    int32_t phase;        // kPhase*
    int32_t iter;         // Krylov iterations done (inner ones for mixed)
    int32_t inner_iter;   // iterations of the current inner solve
    int32_t outer;        // mixed: refinement steps done
    int32_t cmode;        // next x/p update: 2 both, 1 x only (last), 0 none
    int32_t maxit;
    int32_t inner_maxit;
    int32_t max_outer;
    int32_t stagnant;     // mixed: consecutive weak outer reductions
    int32_t mixed;        // 1: mixed-precision solve
    int32_t hist_len;
    int32_t ru;           // mixed: 1 keeps p across refinements (reliable updates)
    int32_t fresh_p;      // mixed: the next refinement starts p from z
    // the scalars of the current iteration as the update pass saw them: the
    // p/x pass decides from these while its block 0 rewrites the live ones
    int32_t snap_status, snap_phase, snap_iter, snap_inner_iter;
    // fused p/x + product kernel (F): p lives in one of two buffers, pbuf
    // (written by F's block 0) naming the current one; snap_pbuf is the
    // copy F's blocks read.  snap_mode says what the next F does: 1 take the
    // decision recorded by the update pass, then (while iterating) the
    // product with p = z + beta p; 0 start: p = z; 3 continue after a
    // reliable update: p = z + beta p with beta from the refinement
    int32_t pbuf, snap_pbuf, snap_mode, pad_f;
    double scale;         // mixed: r32 = r / scale, x += scale d
    double rho, alpha, beta, eta;
    double rnorm, rnorm0, bnorm, thresh, rtol, atol;
    double inner_rtol, inner_thresh;
    double s;             // mixed: ||r|| of the current outer residual
    double s_prev;        // mixed: previous outer ||r||
    double rnorm_true;    // result of the last true-residual kernel
    double snap_rho, snap_eta;
};

// One linear system as seen by the batched kernels.
struct SysDesc {
    int32_t n;
    int32_t R;            // rows per tile
    int32_t ntiles;
    int32_t nblk;         // logical blocks (a multiple of kXcd when >= kXcd)
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const float *val32;
    const double *dinv;
    const float *dinv32;
    const double *b;
    double *x;
    double *r, *z, *p, *q;            // FP64 Krylov vectors
    float *r32, *z32, *p32, *q32, *d32;  // FP32 inner vectors (mixed)
    double *p2;                       // second p buffer of the fused kernels
    float *p2_32;                     //   (null: the three-kernel iteration)
    double *partials;                 // kNumPart * nblk
    SysState *st;
    double *hist;                     // device history (hist_len) or null
    // SELL-64 copy of the matrix (used when `sell_cw` is nonzero)
    int32_t sell_cw;
    int32_t sell_plain;  // kSellPlain64/32 load-policy bits
    const int32_t *sell_ptr;
    const void *sell_col;
    const uint8_t *sell_len;
    const double *sell_val;
    const float *sell_val32;
    const uint16_t *sell_len16;  // row lengths when some row has more than 255 entries
    const int32_t *sell_perm;    // SELL-C-sigma: matrix row of each sorted position
    const uint32_t *sell_mask;   // shared offsets: per-row position masks, or null
};

// ------------------------------------------------------------------ host helpers
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what, const char *file, int line);

#define SPK_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return ::spk::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Logical blocks for a system of `ntiles` tiles, at most `maxb`: a multiple of
// kXcd when there are at least kXcd tiles, so that the XCD-aware remap below
// is a bijection.
inline int pick_nblk(int ntiles, int maxb)
{
    if (ntiles <= 0) return 0;
    if (ntiles < kXcd) return ntiles;
    int b = ntiles < maxb ? ntiles : maxb;
    return b - b % kXcd;
}

// ------------------------------------------------------------------ device helpers
// Workgroups are dispatched round-robin over the 8 XCDs.  Physical block `l`
// of a system therefore runs on XCD l % 8; give XCD x the contiguous logical
// range [x*B/8, (x+1)*B/8) so each XCD's L2 sees a contiguous band of rows
// (and of the gathered x window of banded matrices).
__device__ __forceinline__ int xcd_remap(int l, int nblk)
{
    if (nblk < kXcd || (nblk % kXcd) != 0) return l;
    return (l % kXcd) * (nblk / kXcd) + l / kXcd;
}

// Tiles handled by logical block j of nblk: a balanced contiguous chunk.
__device__ __forceinline__ void block_tiles(int j, int nblk, int ntiles, int &t0, int &t1)
{
    t0 = (int)(((int64_t)j * ntiles) / nblk);
    t1 = (int)(((int64_t)(j + 1) * ntiles) / nblk);
}

// Find the system of physical block b: blk_start is ascending, nsys+1 entries.
__device__ __forceinline__ int find_sys(const int32_t *blk_start, int nsys, int b)
{
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (blk_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Butterfly sum over a wavefront; every lane ends with the same bits
// (each level adds two values whose sum is commutative, hence identical).
template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Deterministic block sum: wave butterflies, then wave 0..3 in order.
// Result valid in every thread.  `sh` holds kBlock/kWave values.
template <class T>
__device__ __forceinline__ T block_sum(T v, T *sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    T s = sh[0];
#pragma unroll
    for (int i = 1; i < kBlock / kWave; ++i) s += sh[i];
    return s;
}

// Fixed-order sum of nblk partials by one block (all threads get the result).
// Each lane sums part[tid], part[tid + 256], ... in that order; the loads of a
// chunk are issued together so the reduction costs one memory latency.
__device__ __forceinline__ double reduce_partials(const double *part, int nblk, double *sh)
{
    constexpr int U = 8;
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < nblk; i0 += kBlock * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            v[u] = i < nblk ? part[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    return block_sum(s, sh);
}

// Three partial arrays reduced together (same order as reduce_partials); all
// loads of a chunk are in flight at once.
__device__ __forceinline__ void reduce_partials3(const double *pa, const double *pb,
                                                 const double *pc, int nblk, double *sh,
                                                 double &A, double &B, double &C)
{
    constexpr int U = 8;
    double s = 0.0, t = 0.0, w = 0.0;
    for (int i0 = threadIdx.x; i0 < nblk; i0 += kBlock * U) {
        double u0[U], u1[U], u2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            u0[u] = i < nblk ? pa[i] : 0.0;
            u1[u] = i < nblk ? pb[i] : 0.0;
            u2[u] = i < nblk ? pc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s += u0[u];
            t += u1[u];
            w += u2[u];
        }
    }
    A = block_sum(s, sh);
    B = block_sum(t, sh);
    C = block_sum(w, sh);
}

// Two partial arrays reduced together (same order as reduce_partials).
__device__ __forceinline__ void reduce_partials2(const double *pa, const double *pb, int nblk,
                                                 double *sh, double &A, double &B)
{
    constexpr int U = 8;
    double s = 0.0, t = 0.0;
    for (int i0 = threadIdx.x; i0 < nblk; i0 += kBlock * U) {
        double v[U], w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kBlock;
            v[u] = i < nblk ? pa[i] : 0.0;
            w[u] = i < nblk ? pb[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s += v[u];
            t += w[u];
        }
    }
    A = block_sum(s, sh);
    B = block_sum(t, sh);
}

template <class T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

}  // namespace spk
