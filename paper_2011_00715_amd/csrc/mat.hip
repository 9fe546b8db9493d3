// Matrix handle, SpMV dispatch, vector kernels and utilities of libspk.so.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "runtime.hpp"
#include "spmv.hpp"

namespace spk {

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what, const char *file, int line)
{
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return e == hipErrorOutOfMemory ? SPK_ENOMEM : SPK_EHIP;
}

// ------------------------------------------------------------------ analysis kernels
__global__ void k_row_stats(int n, int64_t nnz, const int32_t *__restrict__ rowptr,
                            RowStats *__restrict__ out)
{
    __shared__ int32_t hist[33];
    __shared__ unsigned long long s1, s2;
    __shared__ int32_t mx, mn, bad, tmax[6];
    if (threadIdx.x < 33) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s1 = 0; s2 = 0; mx = 0; mn = 0x7fffffff; bad = 0; }
    if (threadIdx.x < 6) tmax[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long a1 = 0, a2 = 0;
    int amx = 0, amn = 0x7fffffff, abad = 0;
    int at[6] = {0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int64_t a = rowptr[i], e = rowptr[i + 1];
        if (e < a || a < 0 || e > nnz || (i == 0 && a != 0) || (i == n - 1 && e != nnz)) {
            ++abad;
            continue;
        }
        const int len = (int)(e - a);
        a1 += (unsigned long long)len;
        a2 += (unsigned long long)len * (unsigned long long)len;
        amx = max(amx, len);
        amn = min(amn, len);
        const int bin = len == 0 ? 0 : 32 - __clz(len);
        atomicAdd(&hist[bin], 1);
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int R = t == 0 ? 256 : (t == 1 ? 128 : (t == 2 ? 64 : (t == 3 ? 32 : (t == 4 ? 16 : 8))));
            if (i % R == 0) {
                const int ie = min(i + R, n);
                const int64_t te = rowptr[ie];
                if (te >= a && te <= nnz) at[t] = max(at[t], (int)(te - a));
            }
        }
    }
    atomicAdd(&s1, a1);
    atomicAdd(&s2, a2);
    atomicMax(&mx, amx);
    atomicMin(&mn, amn);
    atomicAdd(&bad, abad);
#pragma unroll
    for (int t = 0; t < 6; ++t) atomicMax(&tmax[t], at[t]);
    __syncthreads();
    if (threadIdx.x < 33 && hist[threadIdx.x]) atomicAdd(&out->hist[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x < 6) atomicMax(&out->tile_max[threadIdx.x], tmax[threadIdx.x]);
    if (threadIdx.x == 0) {
        atomicAdd(&out->sum_len, s1);
        atomicAdd(&out->sum_len2, s2);
        atomicMax(&out->max_len, mx);
        atomicMin(&out->min_len, mn);
        atomicAdd(&out->bad_rowptr, bad);
    }
}

// Column range and (optionally) strict ascending order; needs a valid rowptr.
// Entries of a SELL-64 layout: one thread per slice of 64 rows adds 64 x the
// slice's longest row (rowptr already validated).
__global__ void k_slice_pad(int n, const int32_t *__restrict__ rowptr, RowStats *__restrict__ out)
{
    const int ns = (n + 63) / 64;
    unsigned long long acc = 0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += gridDim.x * blockDim.x) {
        const int r0 = s * 64, r1 = min(r0 + 64, n);
        int mx = 0;
        int prev = rowptr[r0];
        for (int i = r0; i < r1; ++i) {
            const int e = rowptr[i + 1];
            mx = max(mx, e - prev);
            prev = e;
        }
        acc += 64ULL * (unsigned long long)mx;
    }
    if (acc) atomicAdd(&out->sell_padded, acc);
}

__global__ void k_check_cols(int n, const int32_t *__restrict__ rowptr,
                             const int32_t *__restrict__ col, int check_sorted,
                             RowStats *__restrict__ out)
{
    int badc = 0, uns = 0, md = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int prev = -1;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int c = col[k];
            if (c < 0 || c >= n) ++badc;
            if (check_sorted && c <= prev) ++uns;
            prev = c;
            md = max(md, abs(c - i));
        }
    }
    if (badc) atomicAdd(&out->bad_col, badc);
    if (uns) atomicAdd(&out->unsorted, uns);
    if (md) atomicMax(&out->max_delta, md);
}

// dinv_i = 1 / a_ii (duplicates of the diagonal are summed).
__global__ void k_diag_inv(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ dinv,
                           RowStats *__restrict__ out)
{
    int bad = 0;
    double gmax = 0.0;  // Gershgorin bound of D^-1 A: max_i sum_j |a_ij| / |a_ii|
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double d = 0.0, sabs = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const double v = val[k];
            sabs += fabs(v);
            if (col[k] == i) d += v;
        }
        if (d == 0.0) { ++bad; dinv[i] = 0.0; }
        else {
            dinv[i] = 1.0 / d;
            gmax = fmax(gmax, sabs / fabs(d));
        }
    }
    if (bad) atomicAdd(&out->zero_diag, bad);
    // non-negative doubles order like their bit patterns: one atomic per wave
    gmax = fmax(gmax, 0.0);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && gmax > 0.0)
        atomicMax(&out->gersh_bits, (unsigned long long)__double_as_longlong(gmax));
}

__global__ void k_to_f32(int64_t m, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// ------------------------------------------------------------------ vector kernels
__global__ void k_fill0(int64_t m, double *__restrict__ a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

__global__ void k_axpy(int n, double alpha, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fma(alpha, x[i], y[i]);
}

__global__ void k_aypx(int n, double beta, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fma(beta, y[i], x[i]);
}

__global__ void k_pmul(int n, const double *__restrict__ d, const double *__restrict__ r,
                       double *__restrict__ z)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = d[i] * r[i];
}

// Single-pass dots: per-block partials of x.y (and x.w) over a contiguous
// chunk per block; k_dot_fin sums them in a fixed order.
__global__ __launch_bounds__(kBlock) void k_dot(int n, const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ w,
                                                double *__restrict__ part)
{
    __shared__ double red[kBlock / kWave];
    const int nb = gridDim.x;
    const int j = xcd_remap(blockIdx.x, nb);
    const int64_t chunk = ((int64_t)n + nb - 1) / nb;
    const int rb = (int)min((int64_t)n, j * chunk);
    const int re = (int)min((int64_t)n, (j + 1) * chunk);
    double a = 0.0, b = 0.0;
    for (int i = rb + (int)threadIdx.x; i < re; i += kBlock) {
        const double xi = x[i];
        a = fma(xi, y[i], a);
        if (w) b = fma(xi, w[i], b);
    }
    a = block_sum(a, red);
    if (w) b = block_sum(b, red);
    if (threadIdx.x == 0) { part[j] = a; part[nb + j] = b; }
}

// result[0] = x.y, result[1] = x.w (if two), or ||x|| (mode 2).
__global__ __launch_bounds__(kBlock) void k_dot_fin(int nb, int two, int mode,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ result)
{
    __shared__ double red[kBlock / kWave];
    const double A = reduce_partials(part, nb, red);
    const double B = two ? reduce_partials(part + nb, nb, red) : 0.0;
    if (threadIdx.x == 0) {
        if (mode == 2) result[0] = sqrt(A);
        else {
            result[0] = A;
            if (two) result[1] = B;
        }
    }
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Bandwidth calibration: plain stream copy (2 accesses per entry, Sec. 5.1),
// one 16-byte pair per thread, launched with grid_stream.
__global__ __launch_bounds__(kBlock) void k_copy(int64_t m, const dvec2 *__restrict__ a,
                                                 dvec2 *__restrict__ b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// Cache eviction by reading: the Infinity Cache ends up holding clean lines
// of the scratch buffer, so the next kernel finds none of its data cached and
// pays no write-back of dirty lines left by the eviction itself.  The store
// only happens for a sum no real buffer of finite values produces; it keeps
// the loads from being optimised away.
__global__ __launch_bounds__(kBlock) void k_evict(int64_t m, dvec2 *__restrict__ b)
{
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const dvec2 v = b[i];
        s += v.x + v.y;
    }
    if (s == -1.0e308) b[0] = dvec2{s, s};
}

// ------------------------------------------------------------------ SpMV dispatch
template <class V, int L>
static void launch_vector_l(const spk_mat *A, const V *val, const V *x, V *y, hipStream_t s,
                            const SysState *gst, int gmode)
{
    constexpr int rpb = kBlock / L;
    int grid = ceil_div(A->n, rpb);
    if (grid > kMaxBlocksSingle) grid = kMaxBlocksSingle;
    if (grid >= kXcd) grid -= grid % kXcd;
    hipLaunchKernelGGL((k_spmv_vector<V, L>), dim3(grid), dim3(kBlock), 0, s, A->n, A->rowptr,
                       A->col, val, x, y, gst, gmode);
}

template <class V>
int launch_spmv(const spk_mat *A, const V *val, const V *x, V *y, hipStream_t s,
                const SysState *gst, int gmode)
{
    if (A->n == 0) return SPK_OK;
    switch (A->kernel) {
    case SPK_KERNEL_STREAM:
        if (gst) {
            set_error("internal: gated stream SpMV");
            return SPK_EINVAL;
        }
        hipLaunchKernelGGL((k_spmv_stream<V>), dim3(A->nblk), dim3(kBlock), 0, s, A->n, A->R,
                           A->ntiles, A->nblk, A->rowptr, A->col, val, x, y);
        break;
    case SPK_KERNEL_VECTOR:
        switch (A->lanes) {
        case 1: launch_vector_l<V, 1>(A, val, x, y, s, gst, gmode); break;
        case 2: launch_vector_l<V, 2>(A, val, x, y, s, gst, gmode); break;
        case 4: launch_vector_l<V, 4>(A, val, x, y, s, gst, gmode); break;
        case 8: launch_vector_l<V, 8>(A, val, x, y, s, gst, gmode); break;
        case 16: launch_vector_l<V, 16>(A, val, x, y, s, gst, gmode); break;
        case 32: launch_vector_l<V, 32>(A, val, x, y, s, gst, gmode); break;
        default: launch_vector_l<V, 64>(A, val, x, y, s, gst, gmode); break;
        }
        break;
    case SPK_KERNEL_SELL: {
        if (gst || !A->sell_cw) {
            set_error("internal: gated SELL SpMV or no SELL layout");
            return SPK_EINVAL;
        }
        const SellView sv{A->sell_ptr, A->sell_col, A->sell_len, A->sell_plain_spmv, A->sell_len16, A->sell_perm,
                          A->sell_mask};
        const V *sval = std::is_same<V, double>::value ? (const V *)A->sell_val : (const V *)A->sell_val32;
        (void)val;
        // up to one wavefront per slice
        const dim3 grid(std::max(1, std::min(ceil_div(ceil_div(A->n, kSell), kBlock / kWave), 16384)));
        const int n = A->n;
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2)
                hipLaunchKernelGGL((k_spmv_sell<V, int16_t, U>), grid, dim3(kBlock), 0, s, n, sv, sval, x, y);
            else
                hipLaunchKernelGGL((k_spmv_sell<V, int32_t, U>), grid, dim3(kBlock), 0, s, n, sv, sval, x, y);
        });
        break;
    }
    case SPK_KERNEL_SLICED:
        return launch_sliced<V>(A, x, y, s, gst, gmode);
    case SPK_KERNEL_MERGE: {
        V *cv = reinterpret_cast<V *>(A->carry_val);
        hipLaunchKernelGGL((k_spmv_merge<V>), dim3(A->mtiles), dim3(kBlock), 0, s, A->n,
                           (int)A->nnz, A->rowptr, A->col, val, x, y, A->tile_row, A->tile_k,
                           A->carry_row, cv, gst, gmode);
        hipLaunchKernelGGL((k_merge_fixup<V>), dim3(ceil_div(A->mtiles, kBlock)), dim3(kBlock), 0,
                           s, A->n, A->mtiles, A->carry_row, (const V *)cv, y, gst, gmode);
        break;
    }
    default:
        set_error("internal: unknown kernel %d", A->kernel);
        return SPK_EINVAL;
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

template int launch_spmv<double>(const spk_mat *, const double *, const double *, double *,
                                 hipStream_t, const SysState *, int);
template int launch_spmv<float>(const spk_mat *, const float *, const float *, float *,
                                hipStream_t, const SysState *, int);

// Elementwise kernels: one element per thread and one block per 256 of them
// (up to 2^22 blocks, grid-stride beyond).  On gfx950 a launch of many
// short blocks streams faster than a grid-stride loop over a resident grid
// (2 GiB copy: 6.6 against 5.0 TB/s with 8192 blocks).
static int grid_stream(int64_t m)
{
    int64_t g = (m + kBlock - 1) / kBlock;
    if (g > (1 << 22)) g = 1 << 22;
    if (g < 1) g = 1;
    return (int)g;
}

static int grid_for(int64_t m)
{
    int64_t g = (m + kBlock - 1) / kBlock;
    if (g > kMaxBlocksSingle) g = kMaxBlocksSingle;
    if (g < 1) g = 1;
    return (int)g;
}

void update_info(spk_mat *A)
{
    spk_mat_info &I = A->info;
    const RowStats &S = A->stats;
    I.n = A->n;
    I.nnz = A->nnz;
    I.kernel = A->kernel == SPK_KERNEL_SELL && A->sell_sigma ? SPK_KERNEL_SELL_SIGMA : A->kernel;
    I.sell_sigma = A->kernel == SPK_KERNEL_SELL ? A->sell_sigma : 0;
    I.lanes = A->kernel == SPK_KERNEL_SLICED ? (A->xs_merge ? kMergeItems : A->lanes)
              : A->kernel == SPK_KERNEL_VECTOR ? A->lanes
              : A->kernel == SPK_KERNEL_STREAM ? A->R
              : A->kernel == SPK_KERNEL_SELL ? (A->sell_mask ? 0 : 8 * A->sell_cw) : kMergeItems;
    I.has_f32 = A->val32 != nullptr;
    I.row_min = A->n ? S.min_len : 0;
    I.row_max = S.max_len;
    const double n = A->n > 0 ? (double)A->n : 1.0;
    I.row_mean = (double)S.sum_len / n;
    const double var = (double)S.sum_len2 / n - I.row_mean * I.row_mean;
    I.row_cv = I.row_mean > 0 ? sqrt(var > 0 ? var : 0) / I.row_mean : 0.0;
    // percentiles: upper bound of the log2 bin holding the 50% / 99% rank
    int64_t acc = 0;
    I.row_p50 = I.row_p99 = 0;
    bool got50 = false;
    for (int b = 0; b < 33; ++b) {
        acc += S.hist[b];
        const int ub = b == 0 ? 0 : (int)((1ll << b) - 1);
        if (!got50 && acc * 2 >= A->n) { I.row_p50 = std::min(ub, S.max_len); got50 = true; }
        if (acc * 100 >= (int64_t)A->n * 99) { I.row_p99 = std::min(ub, S.max_len); break; }
    }
    const int64_t nn = A->n, nz = A->nnz;
    I.bytes_spmv_f64 = 12 * nz + 4 * (nn + 1) + 16 * nn;
    I.bytes_spmv_f32 = 8 * nz + 4 * (nn + 1) + 8 * nn;
    I.bytes_pcg_iter_f64 = 12 * nz + 4 * (nn + 1) + 88 * nn;
    I.bytes_pcg_iter_f32 = 8 * nz + 4 * (nn + 1) + 44 * nn;
    I.device_bytes = A->bytes + (A->ws ? A->ws->bytes : 0);
    I.zero_diag_rows = S.zero_diag;
    I.cached_loads = A->kernel == SPK_KERNEL_SELL ? A->sell_plain | A->sell_plain_spmv << 2 : 0;
    double g = 0.0;
    memcpy(&g, &S.gersh_bits, sizeof g);  // bits of a non-negative double
    I.gershgorin = S.zero_diag ? 0.0 : g;
    if (A->kernel == SPK_KERNEL_SELL && A->sell_cw) {
        const int64_t ns = (nn + kSell - 1) / kSell;
        I.stored_nnz = A->sell_nnz;
        // offsets and row lengths (or shared offsets and row masks), plus the
        // row permutation of SELL-C-sigma
        const int64_t extra = A->sell_idx_bytes + (A->sell_perm ? 4 * nn : 0);
        I.format_bytes_spmv_f64 = 8 * A->sell_nnz + 4 * (ns + 1) + 16 * nn + extra;
        I.format_bytes_spmv_f32 = 4 * A->sell_nnz + 4 * (ns + 1) + 8 * nn + extra;
    } else if (A->kernel == SPK_KERNEL_SLICED && A->xs_ptr) {
        // stacked slices: 8n + 1 row pointers; the 8n partial products are
        // written once and read once by the summing pass
        I.stored_nnz = nz;
        I.format_bytes_spmv_f64 = 12 * nz + 4 * (8 * nn + 1) + 8 * nn + 2 * 8 * 8 * nn + 8 * nn;
        I.format_bytes_spmv_f32 = 8 * nz + 4 * (8 * nn + 1) + 4 * nn + 2 * 4 * 8 * nn + 4 * nn;
    } else {
        I.stored_nnz = nz;
        I.format_bytes_spmv_f64 = I.bytes_spmv_f64;
        I.format_bytes_spmv_f32 = I.bytes_spmv_f32;
    }
}

int ensure_f32(spk_mat *A, hipStream_t s)
{
    if (A->sell_cw && !A->sell_val32 && A->sell_nnz > 0) {
        SPK_HIP(hipMalloc(&A->sell_val32, sizeof(float) * A->sell_nnz));
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(A->sell_nnz)), dim3(kBlock), 0, s, A->sell_nnz,
                           A->sell_val, A->sell_val32);
        SPK_HIP(hipGetLastError());
        A->bytes += 4 * A->sell_nnz;
    }
    if (A->xs_ptr) {
        const int rc = ensure_sliced_f32(A, s);
        if (rc) return rc;
    }
    if (A->val32 || A->n == 0) return SPK_OK;
    SPK_HIP(hipMalloc(&A->val32, sizeof(float) * (A->nnz > 0 ? A->nnz : 1)));
    SPK_HIP(hipMalloc(&A->dinv32, sizeof(float) * A->n));
    A->bytes += 4 * A->nnz + 4 * (int64_t)A->n;
    if (A->nnz > 0)
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(A->nnz)), dim3(kBlock), 0, s, A->nnz, A->val,
                           A->val32);
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(A->n)), dim3(kBlock), 0, s, (int64_t)A->n, A->dinv,
                       A->dinv32);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int pow2_ceil(double v)
{
    int L = 1;
    while (L < v && L < 64) L <<= 1;
    return L;
}

// Merge-path diagonals are int32: n + nnz must stay below 2^31.
static bool merge_fits(const spk_mat *A) { return (int64_t)A->n + A->nnz < 0x7fff0000LL; }

// Row-length statistics -> kernel family (stream for short, even rows; vector
// for long, even rows; merge-path for skewed lengths).
// The sliced layout pays when x does not fit one XCD's 4 MB L2 and rows
// reach across it (scattered columns).  With the merge path over the slices:
// 1.15 ms against 2.02 ms (SELL) and 2.13 ms (merge) for 4M rows of 32
// uniform random columns, 1.16 against 1.94 ms (merge) for the skewed
// power-law C4 rows; lanes per slice row take 1.44 and 1.95 ms.  Banded
// matrices keep their x window in L2 anyway.
static bool sliced_wanted(const spk_mat *A)
{
    const double mean = A->n ? (double)A->stats.sum_len / A->n : 0.0;
    return sliced_fits(A) && A->n >= (1 << 19) && mean >= 8.0 &&
           (int64_t)A->stats.max_delta * kXcd >= A->n && (!sliced_skewed(A) || sliced_merge_fits(A));
}

static void choose_kernel(spk_mat *A, bool allow_sell = true, bool allow_sliced = true)
{
    const RowStats &S = A->stats;
    const double mean = A->n ? (double)S.sum_len / A->n : 0.0;
    const int cap = TileLds<double>::kCap;
    int R = 0;
    for (int t = 0; t < 6; ++t)
        if (S.tile_max[t] <= cap) { R = kTileRs[t]; break; }
    // SELL-64: short rows of similar length within each slice (stencils).
    // No LDS staging; column offsets shared per slice where the slices' rows
    // use at most 32 of them (8 bytes per FP64 nonzero and 4 per row instead
    // of CSR's 12), else int16 offsets per entry in a band of +-32767 (10
    // bytes; wider bands keep int32 offsets and still beat the stream
    // kernel: 171 against 195 us on a 200^3 7-point stencil)
    const bool sell_ok = allow_sell && A->n >= kSell && S.max_len <= 64 &&
                         (double)S.sell_padded <= 1.15 * (double)A->nnz &&
                         S.sell_padded < 0x7fff0000ULL;
    if (sell_ok) {
        A->kernel = SPK_KERNEL_SELL;
        A->R = 256;
    } else if (S.max_len <= 64 && R >= 32) {
        A->kernel = SPK_KERNEL_STREAM;
        A->R = R;
    } else if ((mean >= 8 && S.max_len <= 8 * mean + 8) || !merge_fits(A)) {
        A->kernel = SPK_KERNEL_VECTOR;
        A->lanes = pow2_ceil(mean < 2 ? 2 : mean);
        A->R = 256;
    } else {
        A->kernel = SPK_KERNEL_MERGE;
        A->R = 256;
    }
    if (allow_sliced && sliced_wanted(A)) {
        A->kernel = SPK_KERNEL_SLICED;
        A->lanes = sliced_lanes(A);
        A->xs_merge = sliced_merge_fits(A) ? 1 : 0;
        A->R = 256;
    }
}

// Blocks of the PCG kernels of one SELL system (product with its p.q
// partials, update, p/x pass).  Every block of the update and p/x passes
// sums all blocks' partials, so fewer, larger blocks cut that L2 traffic;
// measured on the 7-point 128^3 / 27-point 160^3 systems against caps of
// 512, 1536 and 2048 (same box, two rounds each): 1024 gave the fastest FP64
// and FP32 iterations overall (FP64 66.3 -> 64.4 us and 288.4 -> 286.0 us
// per iteration against 2048).  The other families keep 2048: their
// products use the block count too, and the stream-tile SpMV of the
// power-law matrix took 2693 us on 1024 blocks against 2138 us on 2048.
constexpr int kPcgBlocksSell = 1024;

static int apply_partition(spk_mat *A)
{
    A->ntiles = ceil_div(A->n, A->R);
    A->nblk = pick_nblk(A->ntiles, A->kernel == SPK_KERNEL_SELL ? kPcgBlocksSell : kMaxBlocksSingle);
    return SPK_OK;
}

static int setup_merge(spk_mat *A, hipStream_t s)
{
    if (A->tile_row) return SPK_OK;
    const int64_t items = (int64_t)A->n + A->nnz;
    A->mtiles = (int)((items + kMergeItems - 1) / kMergeItems);
    const int mt = A->mtiles > 0 ? A->mtiles : 1;
    SPK_HIP(hipMalloc(&A->tile_row, sizeof(int32_t) * (mt + 1)));
    SPK_HIP(hipMalloc(&A->tile_k, sizeof(int32_t) * (mt + 1)));
    SPK_HIP(hipMalloc(&A->carry_row, sizeof(int32_t) * mt));
    SPK_HIP(hipMalloc(&A->carry_val, sizeof(double) * mt));
    A->bytes += (int64_t)mt * 20 + 8;
    hipLaunchKernelGGL(k_merge_partition, dim3(ceil_div(A->mtiles + 1, kBlock)), dim3(kBlock), 0, s,
                       A->n, (int)A->nnz, A->rowptr, A->mtiles, A->tile_row, A->tile_k);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

void free_workspace(spk_mat *A);

static void free_sell(spk_mat *A)
{
    if (A->sell_cw) {
        const int64_t ns = (A->n + kSell - 1) / kSell;
        A->bytes -= 4 * (ns + 1) + 8 * A->sell_nnz + A->sell_idx_bytes;
        if (A->sell_perm) A->bytes -= 4ll * A->n;
        if (A->sell_val32) A->bytes -= 4 * A->sell_nnz;
    }
    hipFree(A->sell_mask);
    A->sell_mask = nullptr;
    A->sell_idx_bytes = 0;
    A->sell_req = -1;
    hipFree(A->sell_ptr);
    hipFree(A->sell_col);
    hipFree(A->sell_len);
    hipFree(A->sell_len16);
    hipFree(A->sell_perm);
    hipFree(A->sell_val);
    hipFree(A->sell_val32);
    A->sell_ptr = nullptr;
    A->sell_col = nullptr;
    A->sell_len = nullptr;
    A->sell_len16 = nullptr;
    A->sell_perm = nullptr;
    A->sell_val = nullptr;
    A->sell_val32 = nullptr;
    A->sell_cw = 0;
    A->sell_sigma = 0;
    A->sell_nnz = 0;
    A->sell_plain = 0;
    A->sell_plain_spmv = 0;
}


// Shared offsets for a SELL-64 layout of rows in matrix order: every slice's
// rows must have strictly increasing columns and use between them at most
// kSellSharedMax distinct offsets, and the padding may grow by at most 1/16
// over the per-lane layout.  On success: slice widths u (the list sizes),
// the concatenated offset lists and each row's position mask.
static bool shared_offsets(const std::vector<int32_t> &rp, const std::vector<int32_t> &cl, int n,
                           std::vector<int32_t> &u, std::vector<int32_t> &offs, std::vector<uint32_t> &mask)
{
    const int ns = ceil_div(n, kSell);
    u.assign((size_t)ns, 0);
    offs.clear();
    mask.assign((size_t)n, 0u);
    int64_t shared = 0, lane = 0;
    std::vector<int32_t> un, tmp;
    un.reserve(2 * kSellSharedMax);
    tmp.reserve(2 * kSellSharedMax);
    for (int k = 0; k < ns; ++k) {
        const int r0 = k * kSell, r1 = std::min(n, r0 + kSell);
        un.clear();
        int mx = 0;
        for (int r = r0; r < r1; ++r) {
            const int a = rp[r], e = rp[r + 1];
            mx = std::max(mx, e - a);
            // merge the row's sorted offsets into the slice's list
            tmp.clear();
            size_t i = 0;
            for (int j = a; j < e; ++j) {
                if (j > a && cl[j] <= cl[j - 1]) return false;  // unsorted or repeated column
                const int32_t o = cl[j] - r;
                while (i < un.size() && un[i] < o) tmp.push_back(un[i++]);
                if (i < un.size() && un[i] == o) ++i;
                tmp.push_back(o);
            }
            while (i < un.size()) tmp.push_back(un[i++]);
            un.swap(tmp);
            if ((int)un.size() > kSellSharedMax) return false;
        }
        for (int r = r0; r < r1; ++r) {
            uint32_t m = 0;
            size_t i = 0;
            for (int j = rp[r]; j < rp[r + 1]; ++j) {
                const int32_t o = cl[j] - r;
                while (un[i] != o) ++i;
                m |= 1u << i;
            }
            mask[(size_t)r] = m;
        }
        u[(size_t)k] = (int32_t)un.size();
        offs.insert(offs.end(), un.begin(), un.end());
        shared += (int64_t)un.size();
        lane += mx;
    }
    return shared * 16 <= lane * 17;
}

// The shared-offset layout from shared_offsets' result: slice s spans
// 64 u[s] elements; its offsets sit at element sell_ptr[s] / 64 of sell_col
// (int32); values are filled on the device from the row masks.
static int build_sell_shared(spk_mat *A, hipStream_t s, const std::vector<int32_t> &u,
                             const std::vector<int32_t> &offs, const std::vector<uint32_t> &mask)
{
    const int n = A->n;
    const int ns = ceil_div(n, kSell);
    std::vector<int32_t> sp((size_t)ns + 1);
    int64_t acc = 0;
    int wmax = 0;
    for (int k = 0; k < ns; ++k) {
        sp[k] = (int32_t)acc;
        acc += (int64_t)kSell * u[(size_t)k];
        wmax = std::max(wmax, u[(size_t)k]);
        if (acc > 0x7fffffffLL) { set_error("SELL layout exceeds 2^31 entries"); return SPK_EINVAL; }
    }
    sp[ns] = (int32_t)acc;
    const size_t m = acc > 0 ? (size_t)acc : 1;
    const size_t no = offs.size() > 0 ? offs.size() : 1;
    SPK_HIP(hipMalloc(&A->sell_ptr, sizeof(int32_t) * ((size_t)ns + 1)));
    SPK_HIP(hipMalloc(&A->sell_col, sizeof(int32_t) * no));
    SPK_HIP(hipMalloc(&A->sell_mask, sizeof(uint32_t) * (size_t)n));
    SPK_HIP(hipMalloc(&A->sell_val, sizeof(double) * m));
    SPK_HIP(hipMemcpyAsync(A->sell_ptr, sp.data(), sizeof(int32_t) * ((size_t)ns + 1), hipMemcpyHostToDevice, s));
    if (!offs.empty())
        SPK_HIP(hipMemcpyAsync(A->sell_col, offs.data(), sizeof(int32_t) * offs.size(), hipMemcpyHostToDevice, s));
    SPK_HIP(hipMemcpyAsync(A->sell_mask, mask.data(), sizeof(uint32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sell_fill_shared, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rowptr, A->val,
                       A->sell_ptr, A->sell_mask, A->sell_val);
    SPK_HIP(hipGetLastError());
    A->sell_cw = 4;
    A->sell_sigma = 0;
    A->sell_u = pick_sell_u(wmax);
    A->sell_nnz = acc;
    A->sell_idx_bytes = 4 * (int64_t)offs.size() + 4ll * n;
    // the load policy counts cw bytes per entry plus one byte per row:
    // here no bytes per entry and the rest of the index bytes in the budget
    const int64_t extra = A->sell_idx_bytes - n;
    A->sell_plain = A->stream_loads ? 0 : sell_load_policy(acc, 0, ns, n, 6, kIterCacheBudget - extra);
    A->sell_plain_spmv = A->stream_loads ? 0 : sell_load_policy(acc, 0, ns, n, 2, kSpmvCacheBudget - extra);
    A->bytes += 4 * ((int64_t)ns + 1) + 8 * acc + A->sell_idx_bytes;
    if (A->val32) {
        SPK_HIP(hipMalloc(&A->sell_val32, sizeof(float) * m));
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for((int64_t)m)), dim3(kBlock), 0, s, (int64_t)m, A->sell_val,
                           A->sell_val32);
        SPK_HIP(hipGetLastError());
        A->bytes += 4 * acc;
    }
    // the host vectors are read by the copies above
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

// Build the SELL-64 copy: slice widths from rowptr on the host (setup only),
// entries filled by one device lane per layout position.  cw: 2 (int16
// offsets), 4 (int32), 1 (offsets shared per slice; SPK_EINVAL when the
// matrix does not qualify) or 0 (shared when the matrix qualifies, else int16
// when every |col - row| fits, else int32).  sigma > 0 builds SELL-C-sigma:
// within each window of sigma rows the rows are ordered by length, longest
// first (ties in row order), so that the rows sharing a slice have similar
// lengths and the padding shrinks on skewed matrices; the layout then
// carries the permutation.  Rows longer than 255 entries store their
// lengths in 16 bits.
static int setup_sell(spk_mat *A, hipStream_t s, int cw, int sigma = 0)
{
    if (A->sell_cw && A->sell_req == cw && A->sell_sigma == sigma) return SPK_OK;
    const int req = cw;
    const bool try_shared = (cw == 0 || cw == 1) && sigma == 0 && A->n > 0 && A->stats.max_len <= kSellSharedMax;
    if (cw == 1 && !try_shared) {
        set_error("shared SELL offsets need rows in matrix order of at most %d entries", kSellSharedMax);
        return SPK_EINVAL;
    }
    if (cw == 0 || cw == 1) cw = A->stats.max_delta <= 32767 ? 2 : 4;
    if (cw == 2 && A->stats.max_delta > 32767) {
        set_error("column offsets up to %d do not fit int16", A->stats.max_delta);
        return SPK_EINVAL;
    }
    if (A->stats.max_len > 65535) {
        set_error("SELL needs rows of at most 65535 entries (max %d)", A->stats.max_len);
        return SPK_EINVAL;
    }
    free_sell(A);
    const int n = A->n;
    std::vector<int32_t> rp((size_t)n + 1);
    SPK_HIP(hipMemcpyAsync(rp.data(), A->rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    SPK_HIP(hipStreamSynchronize(s));
    if (try_shared) {
        std::vector<int32_t> cl((size_t)A->nnz), u, offs;
        std::vector<uint32_t> mask;
        if (A->nnz > 0) {
            SPK_HIP(hipMemcpyAsync(cl.data(), A->col, sizeof(int32_t) * (size_t)A->nnz, hipMemcpyDeviceToHost, s));
            SPK_HIP(hipStreamSynchronize(s));
        }
        if (shared_offsets(rp, cl, n, u, offs, mask)) {
            const int rc = build_sell_shared(A, s, u, offs, mask);
            if (rc == SPK_OK) A->sell_req = req;
            return rc;
        }
        if (req == 1) {
            set_error("the rows of a slice use more than %d distinct column offsets (or are unsorted)",
                      kSellSharedMax);
            return SPK_EINVAL;
        }
    }
    std::vector<int32_t> perm;
    if (sigma > 0) {
        perm.resize((size_t)n);
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int w0 = 0; w0 < n; w0 += sigma) {
            const int w1 = (int)std::min<int64_t>((int64_t)w0 + sigma, n);
            std::stable_sort(perm.begin() + w0, perm.begin() + w1, [&](int32_t x, int32_t y) {
                return rp[x + 1] - rp[x] > rp[y + 1] - rp[y];
            });
        }
    }
    auto rlen = [&](int j) {
        const int r = sigma > 0 ? perm[j] : j;
        return rp[r + 1] - rp[r];
    };
    const int ns = ceil_div(n, kSell);
    std::vector<int32_t> sp((size_t)ns + 1);
    int64_t acc = 0;
    int wmax = 0;
    for (int k = 0; k < ns; ++k) {
        int mx = 0;
        for (int j = k * kSell; j < std::min(n, (k + 1) * kSell); ++j) mx = std::max(mx, rlen(j));
        wmax = std::max(wmax, mx);
        sp[k] = (int32_t)acc;
        acc += (int64_t)kSell * mx;
        if (acc > 0x7fffffffLL) { set_error("SELL layout exceeds 2^31 entries"); return SPK_EINVAL; }
    }
    sp[ns] = (int32_t)acc;
    const bool len16 = A->stats.max_len > 255;
    const size_t m = acc > 0 ? (size_t)acc : 1;
    SPK_HIP(hipMalloc(&A->sell_ptr, sizeof(int32_t) * ((size_t)ns + 1)));
    SPK_HIP(hipMalloc(&A->sell_col, (size_t)cw * m));
    if (len16) SPK_HIP(hipMalloc(&A->sell_len16, sizeof(uint16_t) * (size_t)(n > 0 ? n : 1)));
    else SPK_HIP(hipMalloc(&A->sell_len, (size_t)(n > 0 ? n : 1)));
    if (sigma > 0) SPK_HIP(hipMalloc(&A->sell_perm, sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    SPK_HIP(hipMalloc(&A->sell_val, sizeof(double) * m));
    SPK_HIP(hipMemcpyAsync(A->sell_ptr, sp.data(), sizeof(int32_t) * ((size_t)ns + 1), hipMemcpyHostToDevice, s));
    if (sigma > 0)
        SPK_HIP(hipMemcpyAsync(A->sell_perm, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    if (cw == 2)
        hipLaunchKernelGGL(k_sell_fill<int16_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rowptr, A->col,
                           A->val, A->sell_ptr, (const int32_t *)A->sell_perm, (int16_t *)A->sell_col, A->sell_val,
                           A->sell_len, A->sell_len16);
    else
        hipLaunchKernelGGL(k_sell_fill<int32_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rowptr, A->col,
                           A->val, A->sell_ptr, (const int32_t *)A->sell_perm, (int32_t *)A->sell_col, A->sell_val,
                           A->sell_len, A->sell_len16);
    SPK_HIP(hipGetLastError());
    A->sell_cw = cw;
    A->sell_req = req;
    A->sell_sigma = sigma;
    A->sell_u = pick_sell_u(wmax);
    A->sell_nnz = acc;
    A->sell_idx_bytes = (int64_t)cw * acc + n + (len16 ? n : 0);
    const int64_t extra = (len16 ? n : 0) + (sigma > 0 ? 4ll * n : 0);
    A->sell_plain = A->stream_loads ? 0 : sell_load_policy(acc, cw, ns, n, 6, kIterCacheBudget - extra);
    A->sell_plain_spmv = A->stream_loads ? 0 : sell_load_policy(acc, cw, ns, n, 2, kSpmvCacheBudget - extra);
    A->bytes += 4 * ((int64_t)ns + 1) + 8 * acc + A->sell_idx_bytes + (sigma > 0 ? 4ll * n : 0);
    if (A->val32) {
        SPK_HIP(hipMalloc(&A->sell_val32, sizeof(float) * m));
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for((int64_t)m)), dim3(kBlock), 0, s, (int64_t)m, A->sell_val,
                           A->sell_val32);
        SPK_HIP(hipGetLastError());
        A->bytes += 4 * acc;
    }
    // the (sigma-sorted) layout is read in the fill above: wait before the
    // host vectors go
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

}  // namespace spk

using namespace spk;

// ================================================================== C ABI
extern "C" {

const char *spk_last_error(void) { return g_err; }

const char *spk_status_str(int st)
{
    switch (st) {
    case SPK_OK: return "SPK_OK";
    case SPK_EINVAL: return "SPK_EINVAL";
    case SPK_ENOMEM: return "SPK_ENOMEM";
    case SPK_EHIP: return "SPK_EHIP";
    case SPK_EZERODIAG: return "SPK_EZERODIAG";
    case SPK_EBUSY: return "SPK_EBUSY";
    case SPK_EBUDGET: return "SPK_EBUDGET";
    case SPK_ENOTFOUND: return "SPK_ENOTFOUND";
    }
    return "SPK_UNKNOWN_STATUS";
}

const char *spk_reason_str(int r)
{
    switch (r) {
    case SPK_CONVERGED_RTOL: return "CONVERGED_RTOL";
    case SPK_CONVERGED_ATOL: return "CONVERGED_ATOL";
    case SPK_RUNNING: return "RUNNING";
    case SPK_DIVERGED_ITS: return "DIVERGED_ITS";
    case SPK_DIVERGED_INDEFINITE_MAT: return "DIVERGED_INDEFINITE_MAT";
    case SPK_DIVERGED_INDEFINITE_PC: return "DIVERGED_INDEFINITE_PC";
    case SPK_DIVERGED_NANORINF: return "DIVERGED_NANORINF";
    case SPK_DIVERGED_BREAKDOWN: return "DIVERGED_BREAKDOWN";
    case SPK_DIVERGED_STAGNATION: return "DIVERGED_STAGNATION";
    }
    return "UNKNOWN_REASON";
}

double spk_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int spk_runtime_version(void)
{
    int v = 0;
    if (hipRuntimeGetVersion(&v) != hipSuccess) return -1;
    return v;
}

static int create_impl(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                       const double *values, int memtype, uint32_t flags, hipStream_t s,
                       spk_mat *A)
{
    A->n = n;
    A->nnz = nnz;
    A->stream_loads = (flags & SPK_MAT_STREAM) != 0;
    SPK_HIP(hipGetDevice(&A->device));
    const bool borrow = (flags & SPK_MAT_BORROW) != 0;
    const size_t nzb = nnz > 0 ? (size_t)nnz : 1;
    if (borrow) {
        A->own_csr = false;
        A->rowptr = const_cast<int32_t *>(rowptr);
        A->col = const_cast<int32_t *>(colind);
        A->val = const_cast<double *>(values);
    } else {
        SPK_HIP(hipMalloc(&A->rowptr, sizeof(int32_t) * ((size_t)n + 1)));
        SPK_HIP(hipMalloc(&A->col, sizeof(int32_t) * nzb));
        SPK_HIP(hipMalloc(&A->val, sizeof(double) * nzb));
        A->bytes += 4 * ((int64_t)n + 1) + 12 * nnz;
        const hipMemcpyKind kind = memtype == SPK_MEM_HOST ? hipMemcpyHostToDevice
                                                           : hipMemcpyDeviceToDevice;
        if (memtype == SPK_MEM_HOST) {
            // stage through pinned memory in chunks (Response A4: pinned transfers)
            const size_t chunk = 64u << 20;
            char *pin = nullptr;
            SPK_HIP(hipHostMalloc((void **)&pin, chunk, hipHostMallocDefault));
            struct Part { void *dst; const void *src; size_t bytes; } parts[3] = {
                {A->rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1)},
                {A->col, colind, sizeof(int32_t) * (size_t)nnz},
                {A->val, values, sizeof(double) * (size_t)nnz}};
            int rc = SPK_OK;
            for (auto &pt : parts) {
                for (size_t off = 0; off < pt.bytes && rc == SPK_OK; off += chunk) {
                    const size_t len = std::min(chunk, pt.bytes - off);
                    memcpy(pin, (const char *)pt.src + off, len);
                    hipError_t e = hipMemcpyAsync((char *)pt.dst + off, pin, len,
                                                  hipMemcpyHostToDevice, s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                    if (e != hipSuccess) rc = hip_fail(e, "pinned upload", __FILE__, __LINE__);
                }
            }
            hipHostFree(pin);
            if (rc) return rc;
        } else {
            SPK_HIP(hipMemcpyAsync(A->rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1), kind, s));
            if (nnz > 0) {
                SPK_HIP(hipMemcpyAsync(A->col, colind, sizeof(int32_t) * nnz, kind, s));
                SPK_HIP(hipMemcpyAsync(A->val, values, sizeof(double) * nnz, kind, s));
            }
        }
    }
    SPK_HIP(hipMalloc(&A->dinv, sizeof(double) * (n > 0 ? n : 1)));
    A->bytes += 8 * (int64_t)n;

    // statistics + structural checks (memory safety of every later kernel)
    RowStats *dst = nullptr, *hst = nullptr;
    SPK_HIP(hipMalloc(&dst, sizeof(RowStats)));
    SPK_HIP(hipHostMalloc((void **)&hst, sizeof(RowStats), hipHostMallocDefault));
    RowStats init{};
    init.min_len = 0x7fffffff;
    int rc = SPK_OK;
    auto fail = [&](int code) { rc = code; };
    do {
        hipError_t e = hipMemcpyAsync(dst, &init, sizeof(RowStats), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { fail(hip_fail(e, "stats init", __FILE__, __LINE__)); break; }
        if (n > 0)
            hipLaunchKernelGGL(k_row_stats, dim3(grid_for(n)), dim3(kBlock), 0, s, n, nnz, A->rowptr,
                               dst);
        e = hipMemcpyAsync(hst, dst, sizeof(RowStats), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { fail(hip_fail(e, "row statistics", __FILE__, __LINE__)); break; }
        if (hst->bad_rowptr) {
            set_error("malformed rowptr: %d rows out of order or outside [0, nnz] "
                      "(rowptr[0] must be 0 and rowptr[n] = nnz)", hst->bad_rowptr);
            fail(SPK_EINVAL);
            break;
        }
        if (n > 0) {
            hipLaunchKernelGGL(k_slice_pad, dim3(grid_for(ceil_div(n, 64))), dim3(kBlock), 0, s, n,
                               A->rowptr, dst);
            hipLaunchKernelGGL(k_check_cols, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rowptr,
                               A->col, (flags & SPK_MAT_VALIDATE) ? 1 : 0, dst);
            hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A->rowptr,
                               A->col, A->val, A->dinv, dst);
        }
        e = hipMemcpyAsync(hst, dst, sizeof(RowStats), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { fail(hip_fail(e, "column checks", __FILE__, __LINE__)); break; }
        if (hst->bad_col) {
            set_error("%d column indices outside [0, n)", hst->bad_col);
            fail(SPK_EINVAL);
            break;
        }
        if (hst->unsorted) {
            set_error("%d entries not strictly ascending within their row", hst->unsorted);
            fail(SPK_EINVAL);
            break;
        }
        A->stats = *hst;
    } while (0);
    hipFree(dst);
    hipHostFree(hst);
    if (rc) return rc;

    choose_kernel(A);
    if (const char *f = getenv("SPK_FORCE_KERNEL")) {
        if (!strncmp(f, "stream", 6)) A->kernel = SPK_KERNEL_STREAM;
        else if (!strncmp(f, "merge", 5) && merge_fits(A)) A->kernel = SPK_KERNEL_MERGE;
        else if (!strncmp(f, "sell", 4) && A->stats.max_len <= 255) A->kernel = SPK_KERNEL_SELL;
        else if (!strncmp(f, "vector", 6)) {
            A->kernel = SPK_KERNEL_VECTOR;
            const char *c = strchr(f, ':');
            A->lanes = c ? atoi(c + 1) : 32;
        }
    }
    if (A->kernel != SPK_KERNEL_STREAM) A->R = 256;
    if (A->kernel == SPK_KERNEL_STREAM && A->R == 0) A->R = 32;
    if (A->kernel == SPK_KERNEL_SLICED &&
        (setup_sliced(A, s) != SPK_OK || (A->xs_merge && setup_sliced_merge(A, s) != SPK_OK))) {
        choose_kernel(A, true, false);  // no room for the copy: the unsliced family
        if (A->kernel != SPK_KERNEL_STREAM) A->R = 256;
    }
    apply_partition(A);
    if (A->kernel == SPK_KERNEL_MERGE) {
        rc = setup_merge(A, s);
        if (rc) return rc;
    }
    if (A->kernel == SPK_KERNEL_SELL) {
        rc = setup_sell(A, s, 0);
        if (rc) {
            if (getenv("SPK_FORCE_KERNEL")) return rc;
            free_sell(A);  // the layout did not fit: take the next family
            choose_kernel(A, false);
            if (A->kernel != SPK_KERNEL_STREAM) A->R = 256;
            apply_partition(A);
            if (A->kernel == SPK_KERNEL_MERGE) {
                rc = setup_merge(A, s);
                if (rc) return rc;
            }
        }
    }
    if (flags & SPK_MAT_MIXED) {
        rc = ensure_f32(A, s);
        if (rc) return rc;
    }
    SPK_HIP(hipStreamSynchronize(s));
    update_info(A);
    return SPK_OK;
}

int spk_mat_create_csr(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                       const double *values, int memtype, uint32_t flags, void *stream,
                       spk_mat **out)
{
    if (!out) { set_error("out is NULL"); return SPK_EINVAL; }
    *out = nullptr;
    if (n < 0 || nnz < 0 || nnz > 0x7fffffffLL) {
        set_error("n = %d, nnz = %lld: need 0 <= n and 0 <= nnz < 2^31", n, (long long)nnz);
        return SPK_EINVAL;
    }
    if (!rowptr || (nnz > 0 && (!colind || !values))) { set_error("NULL array"); return SPK_EINVAL; }
    if (memtype != SPK_MEM_HOST && memtype != SPK_MEM_DEVICE) {
        set_error("memtype %d", memtype);
        return SPK_EINVAL;
    }
    if ((flags & SPK_MAT_BORROW) && memtype != SPK_MEM_DEVICE) {
        set_error("SPK_MAT_BORROW needs SPK_MEM_DEVICE");
        return SPK_EINVAL;
    }
    if (flags & ~(uint32_t)(SPK_MAT_MIXED | SPK_MAT_VALIDATE | SPK_MAT_BORROW | SPK_MAT_STREAM)) {
        set_error("unknown flags 0x%x", flags);
        return SPK_EINVAL;
    }
    if (memtype == SPK_MEM_HOST) {
        if (rowptr[0] != 0 || rowptr[n] != nnz) {
            set_error("rowptr[0] = %d, rowptr[n] = %d, nnz = %lld", rowptr[0], rowptr[n],
                      (long long)nnz);
            return SPK_EINVAL;
        }
    }
    spk_mat *A = new (std::nothrow) spk_mat();
    if (!A) { set_error("out of host memory"); return SPK_ENOMEM; }
    A->stream = (hipStream_t)stream;
    const int rc = create_impl(n, nnz, rowptr, colind, values, memtype, flags,
                               (hipStream_t)stream, A);
    if (rc) {
        spk_mat_destroy(A);
        return rc;
    }
    *out = A;
    return SPK_OK;
}

int spk_mat_set_kernel(spk_mat *A, int kernel, int32_t param, void *stream)
{
    if (!A) { set_error("A is NULL"); return SPK_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    // solver graphs and partials depend on the partition: release them after
    // the handle's earlier work has finished
    free_workspace(A);
    free_multi(A);
    A->stream = s;
    switch (kernel) {
    case SPK_KERNEL_AUTO: choose_kernel(A); break;
    case SPK_KERNEL_STREAM: {
        int R = param;
        if (R == 0) {
            for (int t = 0; t < 6; ++t)
                if (A->stats.tile_max[t] <= TileLds<double>::kCap) { R = kTileRs[t]; break; }
            if (R == 0) R = 8;
        }
        if (R < 1 || R > kBlock) { set_error("stream rows per tile %d not in [1, 256]", R); return SPK_EINVAL; }
        A->kernel = SPK_KERNEL_STREAM;
        A->R = R;
        break;
    }
    case SPK_KERNEL_VECTOR:
        if (param < 1 || param > 64 || (param & (param - 1))) {
            set_error("lanes %d not a power of two in [1, 64]", param);
            return SPK_EINVAL;
        }
        A->kernel = SPK_KERNEL_VECTOR;
        A->lanes = param;
        A->R = 256;
        break;
    case SPK_KERNEL_MERGE:
        if (!merge_fits(A)) { set_error("merge path needs n + nnz < 2^31"); return SPK_EINVAL; }
        A->kernel = SPK_KERNEL_MERGE;
        A->R = 256;
        break;
    case SPK_KERNEL_SELL: {
        if (param != 0 && param != 1 && param != 16 && param != 32) {
            set_error("SELL column offsets %d not in {0, 1, 16, 32}", param);
            return SPK_EINVAL;
        }
        const int rc = setup_sell(A, s, param == 1 ? 1 : param / 8);
        if (rc) return rc;
        if (A->val32) {
            const int r2 = ensure_f32(A, s);
            if (r2) return r2;
            SPK_HIP(hipStreamSynchronize(s));
        }
        A->kernel = SPK_KERNEL_SELL;
        A->R = 256;
        break;
    }
    case SPK_KERNEL_SELL_SIGMA: {
        const int sigma = param == 0 ? 4096 : param;
        if (sigma < kSell || sigma % kSell != 0) {
            set_error("SELL-C-sigma window %d: a positive multiple of %d", param, kSell);
            return SPK_EINVAL;
        }
        const int rc = setup_sell(A, s, 0, sigma);
        if (rc) return rc;
        if (A->val32) {
            const int r2 = ensure_f32(A, s);
            if (r2) return r2;
            SPK_HIP(hipStreamSynchronize(s));
        }
        A->kernel = SPK_KERNEL_SELL;
        A->R = 256;
        break;
    }
    case SPK_KERNEL_SLICED: {
        const bool lanes_ok = param >= 1 && param <= 64 && !(param & (param - 1));
        if (param != 0 && param != kMergeItems && !lanes_ok) {
            set_error("sliced parameter %d: 0, a power of two in [1, 64] or %d (merge path)", param, kMergeItems);
            return SPK_EINVAL;
        }
        int rc = setup_sliced(A, s);
        if (rc) return rc;
        const int merge = param == kMergeItems || (param == 0 && sliced_merge_fits(A));
        if (merge) {
            rc = setup_sliced_merge(A, s);
            if (rc) return rc;
        }
        A->kernel = SPK_KERNEL_SLICED;
        A->xs_merge = merge;
        A->lanes = lanes_ok ? param : sliced_lanes(A);
        A->R = 256;
        break;
    }
    default:
        set_error("unknown kernel %d", kernel);
        return SPK_EINVAL;
    }
    if (A->kernel == SPK_KERNEL_MERGE) {
        const int rc = setup_merge(A, s);
        if (rc) return rc;
        SPK_HIP(hipStreamSynchronize(s));
    }
    if (kernel == SPK_KERNEL_AUTO && A->kernel == SPK_KERNEL_SLICED) {
        if (setup_sliced(A, s) != SPK_OK || (A->xs_merge && setup_sliced_merge(A, s) != SPK_OK)) {
            choose_kernel(A, true, false);
            if (A->kernel == SPK_KERNEL_MERGE) {
                const int r2 = setup_merge(A, s);
                if (r2) return r2;
                SPK_HIP(hipStreamSynchronize(s));
            }
        }
    }
    if (kernel == SPK_KERNEL_AUTO && A->kernel == SPK_KERNEL_SELL) {
        int rc = setup_sell(A, s, 0);
        if (rc == SPK_OK && A->val32) rc = ensure_f32(A, s);
        if (rc == SPK_OK) rc = hipStreamSynchronize(s) == hipSuccess ? SPK_OK : SPK_EHIP;
        if (rc) {
            free_sell(A);
            choose_kernel(A, false);
            if (A->kernel == SPK_KERNEL_MERGE) {
                const int r2 = setup_merge(A, s);
                if (r2) return r2;
                SPK_HIP(hipStreamSynchronize(s));
            }
        }
    }
    apply_partition(A);
    update_info(A);
    return SPK_OK;
}

int spk_mat_mult(const spk_mat *A, const double *x, double *y, void *stream)
{
    if (!A || (A->n > 0 && (!x || !y))) { set_error("NULL argument"); return SPK_EINVAL; }
    if (x == y && A->n > 0) { set_error("x and y must not alias"); return SPK_EINVAL; }
    A->stream = (hipStream_t)stream;
    return launch_spmv<double>(A, A->val, x, y, (hipStream_t)stream, nullptr, 0);
}

int spk_mat_mult_f32(const spk_mat *A, const float *x, float *y, void *stream)
{
    if (!A || (A->n > 0 && (!x || !y))) { set_error("NULL argument"); return SPK_EINVAL; }
    if (x == y && A->n > 0) { set_error("x and y must not alias"); return SPK_EINVAL; }
    A->stream = (hipStream_t)stream;
    if (!A->val32 && A->n > 0) { set_error("matrix has no FP32 values (create with SPK_MAT_MIXED)"); return SPK_EINVAL; }
    return launch_spmv<float>(A, A->val32, x, y, (hipStream_t)stream, nullptr, 0);
}

int spk_mat_get_info(const spk_mat *A, spk_mat_info *info)
{
    if (!A || !info) { set_error("NULL argument"); return SPK_EINVAL; }
    update_info(const_cast<spk_mat *>(A));
    *info = A->info;
    return SPK_OK;
}

int spk_pc_jacobi_apply(const spk_mat *A, const double *r, double *z, void *stream)
{
    if (!A || (A->n > 0 && (!r || !z))) { set_error("NULL argument"); return SPK_EINVAL; }
    if (A->n == 0) return SPK_OK;
    if (A->stats.zero_diag) {
        set_error("%d rows have no stored or a zero diagonal", A->stats.zero_diag);
        return SPK_EZERODIAG;
    }
    A->stream = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pmul, dim3(grid_stream(A->n)), dim3(kBlock), 0, (hipStream_t)stream, A->n,
                       A->dinv, r, z);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

int spk_mat_destroy(spk_mat *A)
{
    if (!A) return SPK_OK;
    // the handle's work is queued on the stream of its last call; HIP's
    // hipFree below waits for the device as HIP documents
    hipStreamSynchronize(A->stream);
    free_workspace(A);
    free_multi(A);
    if (A->own_csr) {
        hipFree(A->rowptr);
        hipFree(A->col);
        hipFree(A->val);
    }
    hipFree(A->val32);
    hipFree(A->dinv);
    hipFree(A->dinv32);
    hipFree(A->tile_row);
    hipFree(A->tile_k);
    hipFree(A->carry_row);
    hipFree(A->carry_val);
    free_sell(A);
    free_sliced(A);
    delete A;
    return SPK_OK;
}

// ------------------------------------------------------------------ vectors
int spk_vec_axpy(int32_t n, double alpha, const double *x, double *y, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) { set_error("bad argument"); return SPK_EINVAL; }
    if (n == 0) return SPK_OK;
    hipLaunchKernelGGL(k_axpy, dim3(grid_stream(n)), dim3(kBlock), 0, (hipStream_t)stream, n, alpha, x, y);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

int spk_vec_aypx(int32_t n, double beta, const double *x, double *y, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) { set_error("bad argument"); return SPK_EINVAL; }
    if (n == 0) return SPK_OK;
    hipLaunchKernelGGL(k_aypx, dim3(grid_stream(n)), dim3(kBlock), 0, (hipStream_t)stream, n, beta, x, y);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// Per-stream reduction scratch (partials + counter), created on first use.
struct DotScratch {
    double *part = nullptr;
};
static std::mutex g_dot_mu;
static std::map<std::pair<int, void *>, DotScratch> g_dot;

// The two dot kernels on partials `part` (2 x kMaxBlocksSingle doubles).
static int dot_enqueue(int32_t n, const double *x, const double *y, const double *w, int mode,
                       double *result, double *part, void *stream)
{
    int grid = grid_for(n > 0 ? n : 1);
    if (grid >= kXcd) grid -= grid % kXcd;
    hipLaunchKernelGGL(k_dot, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, n, x,
                       mode == 2 ? x : y, w, part);
    hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, grid,
                       w ? 1 : 0, mode, part, result);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int dot_launch(int32_t n, const double *x, const double *y, const double *w, int mode,
                      double *result, void *stream)
{
    if (n < 0 || !x || !result || (mode != 2 && !y)) { set_error("bad argument"); return SPK_EINVAL; }
    int dev = 0;
    SPK_HIP(hipGetDevice(&dev));
    DotScratch sc;
    {
        std::lock_guard<std::mutex> lk(g_dot_mu);
        auto it = g_dot.find({dev, stream});
        if (it == g_dot.end()) {
            SPK_HIP(hipMalloc(&sc.part, sizeof(double) * 2 * kMaxBlocksSingle));
            g_dot[{dev, stream}] = sc;
        } else {
            sc = it->second;
        }
    }
    return dot_enqueue(n, x, y, w, mode, result, sc.part, stream);
}

// Partials of the allocation-free fused dot: one launch has at most
// kMaxBlocksSingle blocks and two sums per block, so every n fits.  Each GPU
// holds its own copy for the life of the process; host code never passes this
// name to a kernel (on the host it is a stand-in, not a device address) but
// the address hipGetSymbolAddress returns for the current device.
constexpr int kScratchDoubles = 2 * kMaxBlocksSingle;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];  // device -> its copy of `scratch`

static int scratch_on_device(double **out)
{
    int dev = 0;
    SPK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d: the allocation-free entry points serve devices 0..%d", dev, kMaxDevices - 1);
        return SPK_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SPK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) { set_error("hipGetSymbolAddress returned no address for the scratch array"); return SPK_EHIP; }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return SPK_OK;
}

int spk_vec_dot(int32_t n, const double *x, const double *y, double *result, void *stream)
{
    return dot_launch(n, x, y, nullptr, 0, result, stream);
}

int spk_vec_dot2(int32_t n, const double *x, const double *y, const double *w, double *result,
                 void *stream)
{
    if (!w) { set_error("w is NULL"); return SPK_EINVAL; }
    return dot_launch(n, x, y, w, 1, result, stream);
}

int spk_vec_dot2_noalloc(int32_t n, const double *x, const double *y, const double *w, double *result,
                         void *stream)
{
    if (n < 0 || !x || !y || !w || !result) { set_error("bad argument"); return SPK_EINVAL; }
    const int grid = grid_for(n > 0 ? n : 1);
    if (2 * grid > kScratchDoubles) {  // cannot happen while grid_for caps the grid
        set_error("n = %d needs %d partials, more than the %d of the static scratch", n, 2 * grid,
                  kScratchDoubles);
        return SPK_EINVAL;
    }
    double *part = nullptr;
    const int rc = scratch_on_device(&part);
    if (rc != SPK_OK) return rc;
    return dot_enqueue(n, x, y, w, 1, result, part, stream);
}

int spk_vec_nrm2(int32_t n, const double *x, double *result, void *stream)
{
    return dot_launch(n, x, nullptr, nullptr, 2, result, stream);
}

int spk_bw_copy(int64_t n, const double *src, double *dst, void *stream)
{
    if (n < 0 || (n & 1) || (n > 0 && (!src || !dst))) { set_error("n must be even and >= 0"); return SPK_EINVAL; }
    if (n == 0) return SPK_OK;
    const int64_t m = n / 2;
    hipLaunchKernelGGL(k_copy, dim3(grid_stream(m)), dim3(kBlock), 0, (hipStream_t)stream, m,
                       (const dvec2 *)src, (dvec2 *)dst);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

int spk_cache_flush(void *scratch, int64_t bytes, void *stream)
{
    if (!scratch || bytes < 16) { set_error("bad argument"); return SPK_EINVAL; }
    const int64_t m = bytes / 16;
    int64_t g = (m + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_evict, dim3((int)g), dim3(kBlock), 0, (hipStream_t)stream, m, (dvec2 *)scratch);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

}  // extern "C"
