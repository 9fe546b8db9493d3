// Multiple right-hand sides: SpMM and K independent Jacobi-PCG solves that
// share every SpMM (Sec. 4 Response F3).
#include <string.h>

#include <algorithm>

#include "multi.hpp"
#include "runtime.hpp"

namespace spk {

struct MultiWs {
    int K = 0;
    int nblk = 0;
    double *B = nullptr, *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
    double *partials = nullptr;
    SysState *st = nullptr;
    SysState *pst = nullptr;  // pinned copy of the K states
    MultiCtl *ctl = nullptr;
    int32_t *pmask = nullptr; // pinned ring of published masks
    hipEvent_t ev[4] = {};
    hipStream_t cap = nullptr;
    hipGraphExec_t g = nullptr;
    int gk = 0;
};

void free_multi(spk_mat *A)
{
    MultiWs *w = A->mws;
    if (!w) return;
    hipStreamSynchronize(A->stream);
    if (w->g) hipGraphExecDestroy(w->g);
    for (auto &e : w->ev)
        if (e) hipEventDestroy(e);
    if (w->cap) hipStreamDestroy(w->cap);
    hipFree(w->B);
    hipFree(w->X);
    hipFree(w->R);
    hipFree(w->Z);
    hipFree(w->P);
    hipFree(w->Q);
    hipFree(w->partials);
    hipFree(w->st);
    hipFree(w->ctl);
    hipHostFree(w->pst);
    hipHostFree(w->pmask);
    delete w;
    A->mws = nullptr;
}

static bool valid_k(int K) { return K == 1 || K == 2 || K == 4 || K == 8 || K == 16; }

// Blocks of the multi kernels: at most half the single-vector kernels' cap.
// Every block writes one partial sum per column and every finalize block
// reduces nblk of them; measured with k = 8 on the 128^3 Laplacian (8192
// tiles), 1024 blocks solve in 182 ms against 192 ms with 2048.
constexpr int kMultiMaxBlocks = 1024;
static int multi_nblk(const spk_mat *A) { return pick_nblk(A->ntiles, kMultiMaxBlocks); }

static MultiDesc multi_desc(const spk_mat *A, int K)
{
    MultiDesc d{};
    d.n = A->n;
    d.K = K;
    d.nblk = multi_nblk(A);
    d.R = A->R;
    d.ntiles = A->ntiles;
    // the multi kernels walk SELL slices in matrix order with one-byte row
    // lengths; a sorted (SELL-C-sigma) or long-row layout goes through CSR
    d.sell = A->kernel == SPK_KERNEL_SELL && A->sell_cw != 0 && !A->sell_perm && (A->sell_len || A->sell_mask);
    d.rowptr = A->rowptr;
    d.col = A->col;
    d.val = A->val;
    d.dinv = A->dinv;
    d.sv = SellView{A->sell_ptr, A->sell_col, A->sell_len, 0, nullptr, nullptr, A->sell_mask};
    d.sell_val = A->sell_val;
    return d;
}

// Calls f(int16/int32 tag, integral_constant K) for the handle's offsets and K.
template <class F>
static void with_multi(const spk_mat *A, int K, F &&f)
{
    auto ci = [&](auto kc) {
        if (A->kernel == SPK_KERNEL_SELL && A->sell_cw == 4) f(int32_t{}, kc);
        else f(int16_t{}, kc);
    };
    switch (K) {
    case 1: ci(std::integral_constant<int, 1>{}); break;
    case 2: ci(std::integral_constant<int, 2>{}); break;
    case 4: ci(std::integral_constant<int, 4>{}); break;
    case 8: ci(std::integral_constant<int, 8>{}); break;
    default: ci(std::integral_constant<int, 16>{}); break;
    }
}

static int get_multi(spk_mat *A, int K, MultiWs **out)
{
    MultiWs *w = A->mws;
    if (w && (w->K != K || w->nblk != multi_nblk(A))) {
        free_multi(A);
        w = nullptr;
    }
    if (!w) {
        w = new (std::nothrow) MultiWs();
        if (!w) { set_error("out of host memory"); return SPK_ENOMEM; }
        A->mws = w;
        w->K = K;
        w->nblk = multi_nblk(A);
        const size_t nk = sizeof(double) * (size_t)std::max(A->n, 1) * K;
        for (double **p : {&w->B, &w->X, &w->R, &w->Z, &w->P, &w->Q}) SPK_HIP(hipMalloc((void **)p, nk));
        SPK_HIP(hipMalloc((void **)&w->partials, sizeof(double) * kNumPart * K * std::max(multi_nblk(A), 1)));
        SPK_HIP(hipMalloc((void **)&w->st, sizeof(SysState) * K));
        SPK_HIP(hipMalloc((void **)&w->ctl, sizeof(MultiCtl)));
        SPK_HIP(hipHostMalloc((void **)&w->pst, sizeof(SysState) * K, hipHostMallocDefault));
        SPK_HIP(hipHostMalloc((void **)&w->pmask, sizeof(int32_t) * 4, hipHostMallocDefault));
        for (auto &e : w->ev) SPK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        SPK_HIP(hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking));
    }
    *out = w;
    return SPK_OK;
}

static MultiDesc solve_desc(const spk_mat *A, MultiWs *w)
{
    MultiDesc d = multi_desc(A, w->K);
    d.B = w->B;
    d.X = w->X;
    d.Rv = w->R;
    d.Z = w->Z;
    d.P = w->P;
    d.Q = w->Q;
    d.partials = w->partials;
    d.st = w->st;
    d.ctl = w->ctl;
    return d;
}

static void enqueue_multi_iter(const spk_mat *A, const MultiDesc &d, hipStream_t s)
{
    const dim3 g(multi_nblk(A)), t(kBlock), cols(d.K);  // finalize: one block per column
    // the p/x pass: about 1024 elements per block, at most kMultiPxBlocks
    const dim3 gpx((unsigned)std::max<int64_t>(
        1, std::min<int64_t>(kMultiPxBlocks, ((int64_t)A->n * d.K + 1023) / 1024)));
    with_multi(A, d.K, [&](auto ct, auto kc) {
        using CI = decltype(ct);
        constexpr int K = decltype(kc)::value;
        hipLaunchKernelGGL((k_m_spmm_pq<CI, K>), g, t, 0, s, d);
        hipLaunchKernelGGL(k_m_fin_pq, cols, t, 0, s, d);
        hipLaunchKernelGGL((k_m_update<K>), g, t, 0, s, d);
        hipLaunchKernelGGL(k_m_fin_update, cols, t, 0, s, d);
        hipLaunchKernelGGL((k_m_px<K>), gpx, t, 0, s, d);
    });
}

static int multi_resid(const spk_mat *A, const MultiDesc &d, int purpose, int32_t mask, hipStream_t s)
{
    with_multi(A, d.K, [&](auto ct, auto kc) {
        using CI = decltype(ct);
        constexpr int K = decltype(kc)::value;
        hipLaunchKernelGGL((k_m_resid<CI, K>), dim3(multi_nblk(A)), dim3(kBlock), 0, s, d, mask);
    });
    hipLaunchKernelGGL(k_m_fin_resid, dim3(d.K), dim3(kBlock), 0, s, d, purpose, mask);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int multi_setup(const spk_mat *A, const MultiDesc &d, int32_t mask, hipStream_t s)
{
    with_multi(A, d.K, [&](auto, auto kc) {
        constexpr int K = decltype(kc)::value;
        hipLaunchKernelGGL((k_m_setup<K>), dim3(multi_nblk(A)), dim3(kBlock), 0, s, d, mask);
    });
    hipLaunchKernelGGL(k_m_fin_setup, dim3(d.K), dim3(kBlock), 0, s, d, mask);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// Replays batches of Kit iterations until no column runs (two in flight).
static int multi_batches(const spk_mat *A, MultiWs *w, const MultiDesc &d, int Kit, bool use_graph,
                         int max_batches, hipStream_t s)
{
    if (use_graph && (!w->g || w->gk != Kit)) {
        if (w->g) { hipGraphExecDestroy(w->g); w->g = nullptr; }
        hipGraph_t graph = nullptr;
        SPK_HIP(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < Kit; ++k) enqueue_multi_iter(A, d, w->cap);
        const hipError_t e = hipStreamEndCapture(w->cap, &graph);
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
        const hipError_t e2 = hipGraphInstantiate(&w->g, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e2 != hipSuccess) { w->g = nullptr; return hip_fail(e2, "hipGraphInstantiate", __FILE__, __LINE__); }
        w->gk = Kit;
    }
    int launched = 0, checked = 0;
    for (;;) {
        if (launched - checked < 2 && launched < max_batches) {
            if (use_graph) SPK_HIP(hipGraphLaunch(w->g, s));
            else for (int k = 0; k < Kit; ++k) enqueue_multi_iter(A, d, s);
            const int slot = launched % 4;
            hipLaunchKernelGGL(k_m_publish, dim3(1), dim3(64), 0, s, (const MultiCtl *)w->ctl, &w->pmask[slot]);
            SPK_HIP(hipGetLastError());
            SPK_HIP(hipEventRecord(w->ev[slot], s));
            ++launched;
            continue;
        }
        if (checked == launched) {
            SPK_HIP(hipStreamSynchronize(s));
            set_error("multi-RHS solver did not stop within %d batches", max_batches);
            return SPK_EHIP;
        }
        const int slot = checked % 4;
        SPK_HIP(hipEventSynchronize(w->ev[slot]));
        ++checked;
        if (w->pmask[slot] == 0) break;
    }
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

}  // namespace spk

using namespace spk;

extern "C" {

int spk_mat_mult_multi(const spk_mat *A, int32_t k, const double *X, double *Y, void *stream)
{
    if (!A) { set_error("A is NULL"); return SPK_EINVAL; }
    if (!valid_k(k)) { set_error("k = %d: supported k are 1, 2, 4, 8, 16", k); return SPK_EINVAL; }
    if (A->n == 0) return SPK_OK;
    if (!X || !Y) { set_error("NULL X or Y"); return SPK_EINVAL; }
    const size_t nk = (size_t)A->n * k;
    if (X < Y + nk && Y < X + nk) { set_error("X and Y must not overlap"); return SPK_EINVAL; }
    MultiDesc d = multi_desc(A, k);
    // SELL: up to one wavefront per slice (no partial sums to keep per block)
    if (d.sell) d.nblk = std::max(1, std::min(ceil_div(ceil_div(A->n, kSell), kBlock / kWave), 16384));
    hipStream_t s = (hipStream_t)stream;
    A->stream = s;
    with_multi(A, k, [&](auto ct, auto kc) {
        using CI = decltype(ct);
        constexpr int K = decltype(kc)::value;
        hipLaunchKernelGGL((k_spmm<CI, K>), dim3(d.nblk), dim3(kBlock), 0, s, d, X, Y);
    });
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

int spk_ksp_solve_multi(spk_mat *A, int32_t k, const double *B, double *X, const spk_ksp_opts *opts,
                        spk_ksp_result *res, void *stream)
{
    const double t0 = spk_now();
    if (!A || !res) { set_error("NULL A or res"); return SPK_EINVAL; }
    if (!valid_k(k)) { set_error("k = %d: supported k are 1, 2, 4, 8, 16", k); return SPK_EINVAL; }
    spk_ksp_opts o;
    spk_ksp_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != SPK_PREC_FP64) { set_error("multi-RHS solves are FP64 only"); return SPK_EINVAL; }
    if (o.maxit < 0 || !(o.rtol >= 0) || !(o.atol >= 0)) { set_error("bad rtol/atol/maxit"); return SPK_EINVAL; }
    const int n = A->n;
    memset(res, 0, sizeof(spk_ksp_result) * k);
    if (n == 0) {
        for (int q = 0; q < k; ++q) res[q].reason = SPK_CONVERGED_ATOL;
        return SPK_OK;
    }
    if (!B || !X) { set_error("NULL B or X"); return SPK_EINVAL; }
    const size_t nk = (size_t)n * k;
    if (B < X + nk && X < B + nk) { set_error("B and X must not overlap"); return SPK_EINVAL; }
    if (A->stats.zero_diag) {
        set_error("%d rows without a nonzero diagonal", A->stats.zero_diag);
        return SPK_EZERODIAG;
    }
    hipStream_t s = (hipStream_t)stream;
    A->stream = s;
    MultiWs *w = nullptr;
    int rc = get_multi(A, k, &w);
    if (rc) return rc;
    const MultiDesc d = solve_desc(A, w);
    const int32_t all = (int32_t)((1u << k) - 1u);
    const int Kit = o.graph_k > 0 ? o.graph_k : 8;
    const bool use_graph = o.graph_k > 0;
    SPK_HIP(hipMemcpyAsync(w->B, B, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    if (o.x0_nonzero) SPK_HIP(hipMemcpyAsync(w->X, X, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    else SPK_HIP(hipMemsetAsync(w->X, 0, sizeof(double) * nk, s));
    hipLaunchKernelGGL(k_m_init, dim3(1), dim3(64), 0, s, d, o.rtol, o.atol, o.maxit);
    if ((rc = multi_resid(A, d, kMultiSetup, all, s))) return rc;
    if ((rc = multi_setup(A, d, all, s))) return rc;
    int restarts[kMultiMax] = {};
    int breakdown = 0;  // columns that exhausted their restarts
    for (;;) {
        const int max_batches = (o.maxit + Kit - 1) / Kit + 2;
        if ((rc = multi_batches(A, w, d, Kit, use_graph, max_batches, s))) return rc;
        if ((rc = multi_resid(A, d, kMultiTrue, all, s))) return rc;
        SPK_HIP(hipMemcpyAsync(w->pst, w->st, sizeof(SysState) * k, hipMemcpyDeviceToHost, s));
        SPK_HIP(hipStreamSynchronize(s));
        int32_t again = 0;
        for (int q = 0; q < k; ++q) {
            const SysState &S = w->pst[q];
            const bool conv = S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL;
            if (conv && S.bnorm > 0 && S.iter > 0 && S.rnorm_true > S.thresh && !((breakdown >> q) & 1)) {
                if (restarts[q] == 3) breakdown |= 1 << q;
                else { ++restarts[q]; again |= 1 << q; }
            }
        }
        if (!again) break;
        hipLaunchKernelGGL(k_m_restart, dim3(1), dim3(64), 0, s, d, again);
        if ((rc = multi_setup(A, d, again, s))) return rc;
    }
    int32_t zero_b = 0;  // b = 0 returns x = 0, whatever x0 was
    for (int q = 0; q < k; ++q)
        if (w->pst[q].bnorm == 0.0) zero_b |= 1 << q;
    if (zero_b)
        with_multi(A, k, [&](auto, auto kc) {
            constexpr int K = decltype(kc)::value;
            hipLaunchKernelGGL((k_m_zero_cols<K>), dim3(std::min(ceil_div(n, kBlock), 1024)), dim3(kBlock), 0, s,
                               d, zero_b);
        });
    SPK_HIP(hipMemcpyAsync(X, w->X, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    SPK_HIP(hipStreamSynchronize(s));
    const double secs = spk_now() - t0;
    for (int q = 0; q < k; ++q) {
        const SysState &S = w->pst[q];
        spk_ksp_result &r = res[q];
        const bool conv = S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL;
        r.reason = S.status;
        if ((breakdown >> q) & 1) r.reason = SPK_DIVERGED_BREAKDOWN;
        else if (conv && S.iter > 0)
            r.reason = S.rnorm_true <= S.rtol * S.bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        r.iterations = S.iter;
        r.restarts = restarts[q];
        r.rnorm0 = S.rnorm0;
        r.rnorm = S.rnorm_true;
        r.bnorm = S.bnorm;
        r.true_rel_residual = S.bnorm > 0 ? S.rnorm_true / S.bnorm : 0.0;
        if (S.bnorm == 0.0) r.rnorm = 0.0;
        r.seconds = secs;
    }
    return SPK_OK;
}

}  // extern "C"
