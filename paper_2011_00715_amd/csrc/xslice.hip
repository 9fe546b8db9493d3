// Column-sliced CSR: layout setup on the device (per-slice row counts, one
// exclusive scan, scatter) and the two-pass SpMV launch.

#include "scan.hpp"
#include "xslice.hpp"
#include "runtime.hpp"

namespace spk {

static int grid_rows(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxBlocksSingle) g = kMaxBlocksSingle;
    return (int)(g < 1 ? 1 : g);
}

static __global__ void k_xs_f32(int64_t m, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

bool sliced_fits(const spk_mat *A) { return (int64_t)kSlices * A->n + 1 < 0x7fff0000LL && A->n > 0; }

int sliced_lanes(const spk_mat *A)
{
    const double mean = A->n ? (double)A->nnz / ((double)kSlices * A->n) : 0.0;
    int L = 1;
    while (L < mean && L < 64) L <<= 1;  // next power of two of the mean slice-row length,
    return L >= 4 ? L / 2 : 2;           // halved: short slice rows leave half the lanes idle otherwise
}

// The merge path over the stacked slices has int32 diagonals.
bool sliced_merge_fits(const spk_mat *A) { return (int64_t)kSlices * A->n + A->nnz < 0x7fff0000LL; }

// Rows too uneven for a fixed number of lanes per slice row.
bool sliced_skewed(const spk_mat *A)
{
    const double mean = A->n ? (double)A->nnz / A->n : 0.0;
    return A->stats.max_len > 8 * mean + 8;
}

static void free_sliced_merge(spk_mat *A)
{
    hipFree(A->xs_tile_row);
    hipFree(A->xs_tile_k);
    hipFree(A->xs_carry_row);
    hipFree(A->xs_carry_val);
    hipFree(A->xs_slice_tile);
    A->xs_tile_row = A->xs_tile_k = A->xs_carry_row = A->xs_slice_tile = nullptr;
    A->xs_carry_val = nullptr;
    if (A->xs_tiles) A->bytes -= 20 * ((int64_t)A->xs_tiles + 1);
    A->xs_tiles = 0;
}

// Merge-path partition of the stacked slices (8n rows, nnz entries) and each
// slice's tile range.
int setup_sliced_merge(spk_mat *A, hipStream_t s)
{
    if (A->xs_tiles) return SPK_OK;
    if (!A->xs_ptr) { set_error("internal: no sliced layout"); return SPK_EINVAL; }
    const int n = A->n;
    const int64_t rows = (int64_t)kSlices * n;
    const int64_t items = rows + A->nnz;
    if (items >= 0x7fff0000LL) { set_error("merge path over the slices needs 8n + nnz < 2^31"); return SPK_EINVAL; }
    const int T = (int)((items + kMergeItems - 1) / kMergeItems);
    int32_t head[kSlices] = {};
    for (int q = 0; q < kSlices; ++q)
        SPK_HIP(hipMemcpyAsync(&head[q], A->xs_ptr + (size_t)q * n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPK_HIP(hipStreamSynchronize(s));
    int32_t st[kSlices + 1];
    int most = 0;
    for (int q = 0; q < kSlices; ++q) {
        const int64_t d = (int64_t)q * n + head[q];  // merge-path diagonal where slice q starts
        st[q] = (int32_t)((d + kMergeItems - 1) / kMergeItems);
    }
    st[kSlices] = T;
    for (int q = 0; q < kSlices; ++q) most = std::max(most, st[q + 1] - st[q]);
    hipError_t e = hipMalloc(&A->xs_tile_row, sizeof(int32_t) * ((size_t)T + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_tile_k, sizeof(int32_t) * ((size_t)T + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_carry_row, sizeof(int32_t) * (size_t)T);
    if (e == hipSuccess) e = hipMalloc(&A->xs_carry_val, sizeof(double) * (size_t)T);
    if (e == hipSuccess) e = hipMalloc(&A->xs_slice_tile, sizeof(int32_t) * (kSlices + 1));
    if (e == hipSuccess) e = hipMemcpyAsync(A->xs_slice_tile, st, sizeof(st), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        free_sliced_merge(A);
        return hip_fail(e, "sliced merge setup", __FILE__, __LINE__);
    }
    A->xs_tiles = T;
    A->xs_tile_grid = std::max(1, most) * kSlices;
    A->bytes += 20 * ((int64_t)T + 1);
    hipLaunchKernelGGL(k_merge_partition, dim3(ceil_div(T + 1, kBlock)), dim3(kBlock), 0, s, (int)rows,
                       (int)A->nnz, (const int32_t *)A->xs_ptr, T, A->xs_tile_row, A->xs_tile_k);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_sliced_merge(A);
        return hip_fail(e, "sliced merge partition", __FILE__, __LINE__);
    }
    return SPK_OK;
}

void free_sliced(spk_mat *A)
{
    free_sliced_merge(A);
    if (A->xs_ptr) {
        A->bytes -= 4 * ((int64_t)kSlices * A->n + 1) + 12 * A->nnz + 8 * (int64_t)kSlices * A->n;
        if (A->xs_val32) A->bytes -= 4 * A->nnz;
    }
    hipFree(A->xs_ptr);
    hipFree(A->xs_col);
    hipFree(A->xs_val);
    hipFree(A->xs_val32);
    hipFree(A->xs_part);
    A->xs_ptr = nullptr;
    A->xs_col = nullptr;
    A->xs_val = nullptr;
    A->xs_val32 = nullptr;
    A->xs_part = nullptr;
}

int ensure_sliced_f32(spk_mat *A, hipStream_t s)
{
    if (!A->xs_ptr || A->xs_val32 || A->nnz == 0) return SPK_OK;
    SPK_HIP(hipMalloc(&A->xs_val32, sizeof(float) * (size_t)A->nnz));
    hipLaunchKernelGGL(k_xs_f32, dim3(grid_rows(A->nnz)), dim3(kBlock), 0, s, A->nnz, (const double *)A->xs_val,
                       A->xs_val32);
    SPK_HIP(hipGetLastError());
    A->bytes += 4 * A->nnz;
    return SPK_OK;
}

int setup_sliced(spk_mat *A, hipStream_t s)
{
    if (A->xs_ptr) return SPK_OK;
    if (!sliced_fits(A)) {
        set_error("the sliced layout needs 8 n + 1 < 2^31");
        return SPK_EINVAL;
    }
    const int n = A->n;
    const int rows = kSlices * n;  // rows of the stacked slices
    int32_t *cnt = nullptr;
    long long *bsum = nullptr;
    int rc = SPK_OK;
    auto fail = [&](hipError_t e, const char *what) {
        hipFree(cnt);
        hipFree(bsum);
        free_sliced(A);
        return hip_fail(e, what, __FILE__, __LINE__);
    };
    hipError_t e = hipMalloc(&cnt, sizeof(int32_t) * (size_t)rows);
    if (e == hipSuccess) e = hipMalloc(&bsum, sizeof(long long) * ((size_t)scan_blocks(rows) + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_ptr, sizeof(int32_t) * ((size_t)rows + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_col, sizeof(int32_t) * (size_t)std::max<int64_t>(A->nnz, 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_val, sizeof(double) * (size_t)std::max<int64_t>(A->nnz, 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_part, sizeof(double) * (size_t)rows);
    if (e != hipSuccess) return fail(e, "hipMalloc");
    A->bytes += 4 * ((int64_t)rows + 1) + 12 * A->nnz + 8 * (int64_t)rows;
    hipLaunchKernelGGL(k_xs_count, dim3(grid_rows(n)), dim3(kBlock), 0, s, n, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, cnt);
    e = scan_exclusive(rows, cnt, A->xs_ptr, bsum, s);
    if (e != hipSuccess) return fail(e, "slice scan");
    hipLaunchKernelGGL(k_xs_fill, dim3(grid_rows(n)), dim3(kBlock), 0, s, n, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, (const double *)A->val, (const int32_t *)A->xs_ptr, A->xs_col,
                       A->xs_val);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(e, "slice fill");
    hipFree(cnt);
    hipFree(bsum);
    if (A->val32) rc = ensure_sliced_f32(A, s);
    return rc;
}

template <class V, int L>
static void launch_xs_l(const spk_mat *A, const V *xval, const V *x, V *part, hipStream_t s, const SysState *gst,
                        int gmode)
{
    constexpr int rpb = kBlock / L;
    int nb = ceil_div(ceil_div(A->n, rpb), 2);  // two row groups per lane group and block
    if (nb > kMaxBlocksSingle) nb = kMaxBlocksSingle;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((k_spmv_xs<V, L>), dim3(nb * kSlices), dim3(kBlock), 0, s, A->n, (const int32_t *)A->xs_ptr,
                       (const int32_t *)A->xs_col, xval, x, part, gst, gmode);
}

template <class V>
int launch_sliced(const spk_mat *A, const V *x, V *y, hipStream_t s, const SysState *gst, int gmode)
{
    const bool f64 = std::is_same<V, double>::value;
    const V *xval = f64 ? (const V *)A->xs_val : (const V *)A->xs_val32;
    if (!A->xs_ptr || !xval) {
        set_error("internal: no sliced layout%s", f64 ? "" : " with FP32 values");
        return SPK_EINVAL;
    }
    V *part = (V *)A->xs_part;
    if (A->xs_merge) {
        if (!A->xs_tiles) { set_error("internal: no merge partition of the slices"); return SPK_EINVAL; }
        const int rows = kSlices * A->n;
        V *cv = (V *)A->xs_carry_val;
        hipLaunchKernelGGL((k_spmv_xs_merge<V>), dim3(A->xs_tile_grid), dim3(kBlock), 0, s, rows,
                           (const int32_t *)A->xs_ptr, (const int32_t *)A->xs_col, xval, x, part,
                           (const int32_t *)A->xs_tile_row, (const int32_t *)A->xs_tile_k, A->xs_carry_row, cv,
                           (const int32_t *)A->xs_slice_tile, gst, gmode);
        hipLaunchKernelGGL((k_merge_fixup<V>), dim3(ceil_div(A->xs_tiles, kBlock)), dim3(kBlock), 0, s, rows,
                           A->xs_tiles, (const int32_t *)A->xs_carry_row, (const V *)cv, part, gst, gmode);
    } else {
    switch (A->lanes) {
    case 1: launch_xs_l<V, 1>(A, xval, x, part, s, gst, gmode); break;
    case 2: launch_xs_l<V, 2>(A, xval, x, part, s, gst, gmode); break;
    case 4: launch_xs_l<V, 4>(A, xval, x, part, s, gst, gmode); break;
    case 8: launch_xs_l<V, 8>(A, xval, x, part, s, gst, gmode); break;
    case 16: launch_xs_l<V, 16>(A, xval, x, part, s, gst, gmode); break;
    case 32: launch_xs_l<V, 32>(A, xval, x, part, s, gst, gmode); break;
    default: launch_xs_l<V, 64>(A, xval, x, part, s, gst, gmode); break;
    }
    }
    hipLaunchKernelGGL((k_xs_reduce<V>), dim3(grid_rows(A->n)), dim3(kBlock), 0, s, A->n, (const V *)part, y, gst,
                       gmode);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

template int launch_sliced<double>(const spk_mat *, const double *, double *, hipStream_t, const SysState *, int);
template int launch_sliced<float>(const spk_mat *, const float *, float *, hipStream_t, const SysState *, int);

}  // namespace spk
