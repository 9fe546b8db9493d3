// Column-sliced CSR: layout setup on the device (per-slice row counts, one
// exclusive scan, scatter) and the two-pass SpMV launch.
#include <hipcub/hipcub.hpp>

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

void free_sliced(spk_mat *A)
{
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
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int rc = SPK_OK;
    auto fail = [&](hipError_t e, const char *what) {
        hipFree(cnt);
        hipFree(tmp);
        free_sliced(A);
        return hip_fail(e, what, __FILE__, __LINE__);
    };
    hipError_t e = hipMalloc(&cnt, sizeof(int32_t) * ((size_t)rows + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_ptr, sizeof(int32_t) * ((size_t)rows + 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_col, sizeof(int32_t) * (size_t)std::max<int64_t>(A->nnz, 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_val, sizeof(double) * (size_t)std::max<int64_t>(A->nnz, 1));
    if (e == hipSuccess) e = hipMalloc(&A->xs_part, sizeof(double) * (size_t)rows);
    if (e != hipSuccess) return fail(e, "hipMalloc");
    A->bytes += 4 * ((int64_t)rows + 1) + 12 * A->nnz + 8 * (int64_t)rows;
    e = hipMemsetAsync(cnt + rows, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return fail(e, "hipMemsetAsync");
    hipLaunchKernelGGL(k_xs_count, dim3(grid_rows(n)), dim3(kBlock), 0, s, n, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, cnt);
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, A->xs_ptr, rows + 1, s);
    if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, A->xs_ptr, rows + 1, s);
    if (e != hipSuccess) return fail(e, "slice scan");
    hipLaunchKernelGGL(k_xs_fill, dim3(grid_rows(n)), dim3(kBlock), 0, s, n, (const int32_t *)A->rowptr,
                       (const int32_t *)A->col, (const double *)A->val, (const int32_t *)A->xs_ptr, A->xs_col,
                       A->xs_val);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(e, "slice fill");
    hipFree(cnt);
    hipFree(tmp);
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
    switch (A->lanes) {
    case 1: launch_xs_l<V, 1>(A, xval, x, part, s, gst, gmode); break;
    case 2: launch_xs_l<V, 2>(A, xval, x, part, s, gst, gmode); break;
    case 4: launch_xs_l<V, 4>(A, xval, x, part, s, gst, gmode); break;
    case 8: launch_xs_l<V, 8>(A, xval, x, part, s, gst, gmode); break;
    case 16: launch_xs_l<V, 16>(A, xval, x, part, s, gst, gmode); break;
    case 32: launch_xs_l<V, 32>(A, xval, x, part, s, gst, gmode); break;
    default: launch_xs_l<V, 64>(A, xval, x, part, s, gst, gmode); break;
    }
    hipLaunchKernelGGL((k_xs_reduce<V>), dim3(grid_rows(A->n)), dim3(kBlock), 0, s, A->n, (const V *)part, y, gst,
                       gmode);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

template int launch_sliced<double>(const spk_mat *, const double *, double *, hipStream_t, const SysState *, int);
template int launch_sliced<float>(const spk_mat *, const float *, float *, hipStream_t, const SysState *, int);

}  // namespace spk
