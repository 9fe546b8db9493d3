// Jacobi-PCG solve driver: workspace, captured iteration graphs, pipelined
// convergence polling, FP64 and mixed-precision (FP32 inner CG + FP64
// iterative refinement) solves.
#include <string.h>

#include <cmath>

#include <algorithm>

#include "cheb.hpp"
#include "krylov.hpp"
#include "sr.hpp"
#include "runtime.hpp"

namespace spk {

void free_workspace(spk_mat *A)
{
    Workspace *w = A->ws;
    if (!w) return;
    hipStreamSynchronize(A->stream);
    if (w->g64) hipGraphExecDestroy(w->g64);
    if (w->gmix) hipGraphExecDestroy(w->gmix);
    for (auto &e : w->ev)
        if (e) hipEventDestroy(e);
    if (w->cap) hipStreamDestroy(w->cap);
    hipFree(w->ddesc);
    hipFree(w->blk_start);
    hipFree(w->st);
    hipFree(w->partials);
    hipFree(w->hist);
    hipFree(w->r);
    hipFree(w->z);
    hipFree(w->p);
    hipFree(w->q);
    hipFree(w->x);
    hipFree(w->b);
    hipFree(w->wpart);
    hipFree(w->r32);
    hipFree(w->z32);
    hipFree(w->p32);
    hipFree(w->q32);
    hipFree(w->d32);
    hipFree(w->p2);
    hipFree(w->p2_32);
    hipFree(w->s);
    hipFree(w->srp);
    hipFree(w->sc);
    if (w->gsr) hipGraphExecDestroy(w->gsr);
    for (auto &e : w->pev)
        if (e) hipEventDestroy(e);
    hipHostFree(w->pdesc);
    hipHostFree(w->pst);
    hipHostFree(w->pstatus);
    delete w;
    A->ws = nullptr;
}

template <class T>
static int dalloc(T **p, int64_t count, Workspace *w)
{
    const size_t b = sizeof(T) * (size_t)(count > 0 ? count : 1);
    SPK_HIP(hipMalloc((void **)p, b));
    w->bytes += (int64_t)b;
    return SPK_OK;
}

#define SPK_TRY(x)                  \
    do {                            \
        const int rc_ = (x);        \
        if (rc_ != SPK_OK) return rc_; \
    } while (0)

// The PCG product runs one wavefront per slice (plus the one-block fold of
// its partials, ~4.6 us) instead of the persistent grid when each lane of
// the persistent grid would stream more than this many SELL entries:
// 160^3 27-point makes 210 (FP64 iteration 313 -> 306 us, FP32 inner
// 181 -> 177 us with the wide product), the 7-point matrices of 150^3 and
// 160^3 45 and 55 (FP32 inner iterations 65 -> 70 and 79 -> 83 us slower),
// 128^3 28.
constexpr int64_t kWideEntriesPerLane = 96;

static __global__ void k_ws_init(int32_t *blk_start, int nblk, SysState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        blk_start[0] = 0;
        blk_start[1] = nblk;
        *st = SysState{};
    }
}

// Whether the fused iteration pays for one precision (kSellPlain64 / 32):
// it moves 8n (FP32: 4n) bytes less per iteration and saves a launch, but
// its kernel F holds one more vector (the second p buffer) besides the
// matrix.  When the three-kernel iteration's working set (the layout and
// six vectors) fits the Infinity Cache and the fused one's does not, the
// product loses its cache hits.  The 7-point 128^3 FP64 iteration (249 MB
// three-kernel, 266 MB fused, against a 268 MB cache) took 70.4 us fused
// and 64.4 us in three kernels, so the fused set must leave kFusedMargin of
// the cache free; its FP32 inner iteration (157 MB fused) went 44.1 ->
// 41.7 us.
constexpr int64_t kFusedMargin = 16ll << 20;
static bool fused_pays(const spk_mat *A, int bit)
{
    const int ns = ceil_div(A->n, kSell);
    // index bytes beyond the policy's own count (cw per entry, one per row):
    // 16-bit lengths, or shared offsets with row masks, and a permutation
    const int cw = A->sell_mask ? 0 : A->sell_cw;
    const int64_t extra =
        A->sell_idx_bytes - (int64_t)cw * A->sell_nnz - A->n + (A->sell_perm ? 4ll * A->n : 0);
    if (A->stream_loads) return true;
    const int six = sell_load_policy(A->sell_nnz, cw, ns, A->n, 6, kIterCacheBudget - extra);
    const int seven = sell_load_policy(A->sell_nnz, cw, ns, A->n, 7, kIterCacheBudget - extra - kFusedMargin);
    return !((six & bit) && !(seven & bit));
}

static int get_workspace(spk_mat *A, bool mixed, Workspace **out, hipStream_t s)
{
    Workspace *w = A->ws;
    if (!w) {
        w = new (std::nothrow) Workspace();
        if (!w) { set_error("out of host memory"); return SPK_ENOMEM; }
        A->ws = w;
        w->n = A->n;
        SPK_TRY(dalloc(&w->ddesc, 1, w));
        SPK_TRY(dalloc(&w->blk_start, 2, w));
        SPK_TRY(dalloc(&w->st, 1, w));
        SPK_TRY(dalloc(&w->partials, (int64_t)kNumPart * std::max(A->nblk, 1), w));
        SPK_TRY(dalloc(&w->r, A->n, w));
        SPK_TRY(dalloc(&w->z, A->n, w));
        SPK_TRY(dalloc(&w->p, A->n, w));
        SPK_TRY(dalloc(&w->q, A->n, w));
        SPK_TRY(dalloc(&w->x, A->n, w));
        SPK_TRY(dalloc(&w->b, A->n, w));
        // large SELL matrices take the wide product (one wavefront per slice)
        if (A->kernel == SPK_KERNEL_SELL && A->sell_cw && A->nblk > 0 &&
            A->sell_nnz > kWideEntriesPerLane * kBlock * A->nblk) {
            w->nwpart = ceil_div(ceil_div(A->n, kSell), kBlock / kWave);
            SPK_TRY(dalloc(&w->wpart, w->nwpart, w));
        }
        // the SELL product on the persistent grid takes the fused iteration
        if (A->kernel == SPK_KERNEL_SELL && A->sell_cw && A->nblk > 0 && !w->wpart) {
            w->fused64 = fused_pays(A, kSellPlain64);
            w->fused32 = fused_pays(A, kSellPlain32);
        }
        if (w->fused64) SPK_TRY(dalloc(&w->p2, A->n, w));
        SPK_HIP(hipHostMalloc((void **)&w->pdesc, sizeof(SysDesc), hipHostMallocDefault));
        SPK_HIP(hipHostMalloc((void **)&w->pst, sizeof(SysState), hipHostMallocDefault));
        SPK_HIP(hipHostMalloc((void **)&w->pstatus, sizeof(int32_t) * 8, hipHostMallocDefault));
        for (auto &e : w->ev) SPK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        SPK_HIP(hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking));
        hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(64), 0, s, w->blk_start, A->nblk, w->st);
        SPK_HIP(hipGetLastError());
        SysDesc &d = w->hdesc;
        d.n = A->n;
        d.R = A->R;
        d.ntiles = A->ntiles;
        d.nblk = A->nblk;
        d.rowptr = A->rowptr;
        d.col = A->col;
        d.val = A->val;
        d.dinv = A->dinv;
        d.x = w->x;
        d.b = w->b;
        d.r = w->r;
        d.z = w->z;
        d.p = w->p;
        d.q = w->q;
        d.partials = w->partials;
        d.st = w->st;
        d.sell_cw = A->kernel == SPK_KERNEL_SELL ? A->sell_cw : 0;
        d.sell_ptr = A->sell_ptr;
        d.sell_col = A->sell_col;
        d.sell_len = A->sell_len;
        d.sell_val = A->sell_val;
        d.sell_plain = A->sell_plain;
        d.sell_len16 = A->sell_len16;
        d.sell_perm = A->sell_perm;
        d.sell_mask = A->sell_mask;
        d.p2 = w->p2;
    }
    if (mixed && !w->has_mixed) {
        SPK_TRY(dalloc(&w->r32, A->n, w));
        SPK_TRY(dalloc(&w->z32, A->n, w));
        SPK_TRY(dalloc(&w->p32, A->n, w));
        SPK_TRY(dalloc(&w->q32, A->n, w));
        SPK_TRY(dalloc(&w->d32, A->n, w));
        if (w->fused32) SPK_TRY(dalloc(&w->p2_32, A->n, w));
        w->has_mixed = 1;
        SysDesc &d = w->hdesc;
        d.val32 = A->val32;
        d.dinv32 = A->dinv32;
        d.r32 = w->r32;
        d.z32 = w->z32;
        d.p32 = w->p32;
        d.q32 = w->q32;
        d.d32 = w->d32;
        d.p2_32 = w->p2_32;
        d.sell_val32 = A->sell_val32;
    }
    *out = w;
    return SPK_OK;
}

// Every pointer of the descriptor is owned by the workspace (b is copied in),
// so the descriptor travels by value in the kernel arguments and captured
// graphs stay valid from one solve to the next.  A profiled solve times the
// product kernel alone, so it runs the three-kernel iteration: its
// descriptor has no second p buffer (the results are the same bits).
static bool use_fused(const Workspace *w, bool mixed) { return (mixed ? w->fused32 : w->fused64) && !w->prof; }
static One batch_of(Workspace *w)
{
    One b{w->hdesc};
    if (!use_fused(w, false)) b.d.p2 = nullptr;
    if (!use_fused(w, true)) b.d.p2_32 = nullptr;
    return b;
}

// r = b - A x for the handle's kernel family.
static int launch_resid(spk_mat *A, Workspace *w, int purpose, bool gated, hipStream_t s)
{
    const One b = batch_of(w);
    const dim3 g(A->nblk), t(kBlock), one(1);
    if (A->kernel == SPK_KERNEL_STREAM) {
        if (gated) hipLaunchKernelGGL((k_resid_stream<kGateResid, One>), g, t, 0, s, b);
        else hipLaunchKernelGGL((k_resid_stream<kGateNone, One>), g, t, 0, s, b);
    } else if (A->kernel == SPK_KERNEL_SELL) {
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2) {
                if (gated) hipLaunchKernelGGL((k_resid_sell<kGateResid, int16_t, U, One>), g, t, 0, s, b);
                else hipLaunchKernelGGL((k_resid_sell<kGateNone, int16_t, U, One>), g, t, 0, s, b);
            } else {
                if (gated) hipLaunchKernelGGL((k_resid_sell<kGateResid, int32_t, U, One>), g, t, 0, s, b);
                else hipLaunchKernelGGL((k_resid_sell<kGateNone, int32_t, U, One>), g, t, 0, s, b);
            }
        });
    } else {
        SPK_TRY(launch_spmv<double>(A, A->val, w->x, w->r, s, gated ? w->st : nullptr,
                                    gated ? kGateResid : kGateNone));
        if (gated) hipLaunchKernelGGL((k_resid_combine<kGateResid, One>), g, t, 0, s, b);
        else hipLaunchKernelGGL((k_resid_combine<kGateNone, One>), g, t, 0, s, b);
    }
    if (gated) hipLaunchKernelGGL((k_fin_resid<kGateResid, One>), one, t, 0, s, b, purpose);
    else hipLaunchKernelGGL((k_fin_resid<kGateNone, One>), one, t, 0, s, b, purpose);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// The next event pair of a profiled solve (created on first use).
static int prof_pair(Workspace *w, hipEvent_t *e0, hipEvent_t *e1)
{
    const size_t k = 2 * (size_t)w->pev_used;
    while (w->pev.size() < k + 2) {
        hipEvent_t e = nullptr;
        SPK_HIP(hipEventCreate(&e));
        w->pev.push_back(e);
    }
    if (w->alive.size() < (size_t)w->pev_used + 1) w->alive.resize(w->pev_used + 1);
    w->alive[w->pev_used] = 1;
    *e0 = w->pev[k];
    *e1 = w->pev[k + 1];
    ++w->pev_used;
    return SPK_OK;
}

template <class V>
static int enqueue_iteration(spk_mat *A, Workspace *w, hipStream_t s)
{
    const One b = batch_of(w);
    const dim3 g(A->nblk), t(kBlock), one(1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (w->prof) {
        SPK_TRY(prof_pair(w, &e0, &e1));
        SPK_HIP(hipEventRecord(e0, s));
    }
    if (A->kernel == SPK_KERNEL_STREAM) {
        hipLaunchKernelGGL((k_pcg_spmv_stream<V, One>), g, t, 0, s, b);
    } else if (A->kernel == SPK_KERNEL_SELL && w->wpart) {
        const dim3 gw(w->nwpart);
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2) hipLaunchKernelGGL((k_pcg_spmv_sell_wide<V, int16_t, U>), gw, t, 0, s, b, w->wpart);
            else hipLaunchKernelGGL((k_pcg_spmv_sell_wide<V, int32_t, U>), gw, t, 0, s, b, w->wpart);
        });
        // the pair times the slice kernel, which moves the bytes; the fold
        // of its per-block partials (one block, a few microseconds) is outside
        if (e1) {
            SPK_HIP(hipEventRecord(e1, s));
            e1 = nullptr;
        }
        hipLaunchKernelGGL((k_fin_pq<V>), one, dim3(kFinPqThreads), 0, s, b, (const double *)w->wpart, w->nwpart);
    } else if (A->kernel == SPK_KERNEL_SELL) {
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2) hipLaunchKernelGGL((k_pcg_spmv_sell<V, int16_t, U, One>), g, t, 0, s, b);
            else hipLaunchKernelGGL((k_pcg_spmv_sell<V, int32_t, U, One>), g, t, 0, s, b);
        });
    } else {
        const V *val = std::is_same<V, double>::value ? (const V *)A->val : (const V *)A->val32;
        V *p = std::is_same<V, double>::value ? (V *)w->p : (V *)w->p32;
        V *q = std::is_same<V, double>::value ? (V *)w->q : (V *)w->q32;
        SPK_TRY(launch_spmv<V>(A, val, p, q, s, w->st, Vecs<V>::gate));
        hipLaunchKernelGGL((k_pcg_pq<V, One>), g, t, 0, s, b);
    }
    if (e1) SPK_HIP(hipEventRecord(e1, s));
    hipLaunchKernelGGL((k_pcg_update<V, One>), g, t, 0, s, b);
    hipLaunchKernelGGL((k_pcg_px<V, One>), g, t, 0, s, b);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// F of the fused iteration (the C part, then the next product).
template <class V, bool kStart>
static void launch_fused(spk_mat *A, Workspace *w, hipStream_t s)
{
    const One b = batch_of(w);
    const dim3 g(A->nblk), t(kBlock);
    with_sell_u(A->sell_u, [&](auto uc) {
        constexpr int U = decltype(uc)::value;
        if (A->sell_cw == 2) hipLaunchKernelGGL((k_pcg_fused_sell<V, int16_t, U, kStart, One>), g, t, 0, s, b);
        else hipLaunchKernelGGL((k_pcg_fused_sell<V, int32_t, U, kStart, One>), g, t, 0, s, b);
    });
}

// One batch of K iterations (mixed: preceded by the refinement kernels).
// Fused: a start kernel (a no-op unless a setup finalizer just ran) and K
// times B, F; F of the batch's last iteration holds its decision, which the
// next batch's refinement kernels (gated on the phase it sets) follow.
static int enqueue_batch(spk_mat *A, Workspace *w, bool mixed, int K, hipStream_t s)
{
    if (use_fused(w, mixed)) {
        const One b = batch_of(w);
        const dim3 g(A->nblk), t(kBlock);
        if (mixed) {
            hipLaunchKernelGGL(k_update_x<One>, g, t, 0, s, b);
            SPK_TRY(launch_resid(A, w, kResOuter, true, s));
            hipLaunchKernelGGL(k_setup32<One>, g, t, 0, s, b);
            hipLaunchKernelGGL(k_fin_setup32<One>, dim3(1), t, 0, s, b);
            launch_fused<float, true>(A, w, s);
            for (int k = 0; k < K; ++k) {
                hipLaunchKernelGGL((k_pcg_update<float, One>), g, t, 0, s, b);
                launch_fused<float, false>(A, w, s);
            }
        } else {
            launch_fused<double, true>(A, w, s);
            for (int k = 0; k < K; ++k) {
                hipLaunchKernelGGL((k_pcg_update<double, One>), g, t, 0, s, b);
                launch_fused<double, false>(A, w, s);
            }
        }
        SPK_HIP(hipGetLastError());
        return SPK_OK;
    }
    if (mixed) {
        const One b = batch_of(w);
        hipLaunchKernelGGL(k_update_x<One>, dim3(A->nblk), dim3(kBlock), 0, s, b);
        SPK_TRY(launch_resid(A, w, kResOuter, true, s));
        hipLaunchKernelGGL(k_setup32<One>, dim3(A->nblk), dim3(kBlock), 0, s, b);
        hipLaunchKernelGGL(k_fin_setup32<One>, dim3(1), dim3(kBlock), 0, s, b);
        hipLaunchKernelGGL((k_pcg_p_continue<float, One>), dim3(A->nblk), dim3(kBlock), 0, s, b);
        for (int k = 0; k < K; ++k) SPK_TRY(enqueue_iteration<float>(A, w, s));
    } else {
        for (int k = 0; k < K; ++k) SPK_TRY(enqueue_iteration<double>(A, w, s));
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int get_graph(spk_mat *A, Workspace *w, bool mixed, int K, hipGraphExec_t *out)
{
    hipGraphExec_t &g = mixed ? w->gmix : w->g64;
    int &gk = mixed ? w->gmix_k : w->g64_k;
    if (g && gk == K) { *out = g; return SPK_OK; }
    if (g) { hipGraphExecDestroy(g); g = nullptr; }
    hipGraph_t graph = nullptr;
    SPK_HIP(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch(A, w, mixed, K, w->cap);
    const hipError_t e = hipStreamEndCapture(w->cap, &graph);
    if (rc) { if (graph) hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    const hipError_t e2 = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e2 != hipSuccess) { g = nullptr; return hip_fail(e2, "hipGraphInstantiate", __FILE__, __LINE__); }
    gk = K;
    *out = g;
    return SPK_OK;
}

static __global__ void k_publish(const SysState *st, int32_t *host)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        host[0] = st->status;
        host[1] = st->phase;
    }
}

// Replays batches until the device reports that the solve stopped.  Two
// batches stay queued, so the GPU never waits for the host's status check
// (Challenge A1: keep the stream queue from draining).
static int run_batches(spk_mat *A, Workspace *w, bool mixed, int K, bool use_graph,
                       int max_batches, hipStream_t s)
{
    hipGraphExec_t g = nullptr;
    if (use_graph) SPK_TRY(get_graph(A, w, mixed, K, &g));
    constexpr int kDepth = 2;
    int launched = 0, checked = 0;
    for (;;) {
        if (launched - checked < kDepth && launched < max_batches) {
            if (use_graph) SPK_HIP(hipGraphLaunch(g, s));
            else SPK_TRY(enqueue_batch(A, w, mixed, K, s));
            const int slot = launched % 4;
            // one thread stores (status, phase) into pinned host memory: cheaper
            // than a device-to-host copy, which runs as a blit kernel
            hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, w->st, &w->pstatus[2 * slot]);
            SPK_HIP(hipEventRecord(w->ev[slot], s));
            ++launched;
            continue;
        }
        if (checked == launched) {
            SPK_HIP(hipStreamSynchronize(s));
            set_error("solver did not stop within %d batches of %d iterations", max_batches, K);
            return SPK_EHIP;
        }
        const int slot = checked % 4;
        SPK_HIP(hipEventSynchronize(w->ev[slot]));
        ++checked;
        if (w->pstatus[2 * slot] != SPK_RUNNING) break;
    }
    SPK_HIP(hipStreamSynchronize(s));
    if (w->prof) {
        // one iteration per batch: the batches queued after the one that
        // stopped the solve ran gated no-op products
        const int dead = launched - checked;
        for (int i = w->pev_used - dead; i < w->pev_used; ++i)
            if (i >= 0) w->alive[i] = 0;
    }
    return SPK_OK;
}

static int read_state(Workspace *w, hipStream_t s)
{
    SPK_HIP(hipMemcpyAsync(w->pst, w->st, sizeof(SysState), hipMemcpyDeviceToHost, s));
    SPK_HIP(hipStreamSynchronize(s));
    return SPK_OK;
}

static void fill_zero(double *p, int64_t n, hipStream_t s);

// Inner tolerance of a mixed solve: a refinement is due once the FP32
// residual fell by this factor since the last one.
double inner_rtol_of(const spk_ksp_opts &o)
{
    if (o.inner_rtol > 0) return o.inner_rtol;
    return o.precision == SPK_PREC_MIXED_IR ? 1e-4 : kRuDelta;
}

struct SolveOut {
    int reason = 0, iterations = 0, restarts = 0;
    double rnorm0 = 0, rnorm = 0, bnorm = 0, rnorm_true = 0;
};

// FP64 Jacobi-PCG on w->x (already initialised).
static int solve64(spk_mat *A, Workspace *w, const spk_ksp_opts &o, bool x_given_residual,
                   int hist_len, hipStream_t s, SolveOut *out)
{
    (void)x_given_residual;
    const int K = w->prof ? 1 : o.graph_k > 0 ? o.graph_k : 8;
    const bool use_graph = o.graph_k > 0 && !w->prof;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, w->st, o.rtol, o.atol, o.maxit, 0,
                       o.inner_rtol, o.inner_maxit, o.max_outer, hist_len);
    SPK_TRY(launch_resid(A, w, kResSetup, false, s));
    hipLaunchKernelGGL(k_setup64<One>, dim3(A->nblk), dim3(kBlock), 0, s, batch_of(w));
    hipLaunchKernelGGL(k_fin_setup64<One>, dim3(1), dim3(kBlock), 0, s, batch_of(w));
    SPK_HIP(hipGetLastError());
    int restarts = 0;
    for (;;) {
        SPK_TRY(read_state(w, s));
        const int done_iter = w->pst->iter;
        const int max_batches = (std::max(o.maxit - done_iter, 0) + K - 1) / K + 2;
        if (w->pst->status == SPK_RUNNING) SPK_TRY(run_batches(A, w, false, K, use_graph, max_batches, s));
        SPK_TRY(launch_resid(A, w, kResTrue, false, s));
        SPK_TRY(read_state(w, s));
        const SysState &S = *w->pst;
        const bool conv = S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL;
        if (conv && S.bnorm > 0 && S.iter > 0 && S.rnorm_true > S.thresh) {
            if (restarts == 3) {
                out->reason = SPK_DIVERGED_BREAKDOWN;
                break;
            }
            ++restarts;
            hipLaunchKernelGGL(k_state_restart, dim3(1), dim3(64), 0, s, w->st);
            hipLaunchKernelGGL(k_setup64<One>, dim3(A->nblk), dim3(kBlock), 0, s, batch_of(w));
            hipLaunchKernelGGL(k_fin_setup64<One>, dim3(1), dim3(kBlock), 0, s, batch_of(w));
            SPK_HIP(hipGetLastError());
            continue;
        }
        out->reason = S.status;
        if (conv && S.iter > 0)  // reason from the confirmed true residual
            out->reason = S.rnorm_true <= S.rtol * S.bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        break;
    }
    const SysState &S = *w->pst;
    out->iterations = S.iter;
    out->restarts = restarts;
    out->rnorm0 = S.rnorm0;
    out->rnorm = (S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL) && S.iter > 0
                     ? S.rnorm_true : S.rnorm;
    out->bnorm = S.bnorm;
    out->rnorm_true = S.rnorm_true;
    if (S.bnorm == 0.0) {
        fill_zero(w->x, A->n, s);
        out->rnorm_true = 0.0;
        out->rnorm = 0.0;
    }
    return SPK_OK;
}

static int solve_mixed(spk_mat *A, Workspace *w, const spk_ksp_opts &o, int hist_len,
                       hipStream_t s, SolveOut *out, int *inner, int *outer)
{
    const int K = w->prof ? 1 : o.graph_k > 0 ? o.graph_k : 8;
    const bool use_graph = o.graph_k > 0 && !w->prof;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, w->st, o.rtol, o.atol, o.maxit,
                       o.precision, inner_rtol_of(o), o.inner_maxit, o.max_outer, hist_len);
    SPK_HIP(hipGetLastError());
    const int max_batches = (o.maxit + K - 1) / K + 2 * (o.max_outer + 2);
    SPK_TRY(run_batches(A, w, true, K, use_graph, max_batches, s));
    SPK_TRY(launch_resid(A, w, kResTrue, false, s));
    SPK_TRY(read_state(w, s));
    const SysState &S = *w->pst;
    out->reason = S.status;
    out->iterations = 0;
    out->rnorm0 = S.rnorm0;
    out->rnorm = S.rnorm_true;
    out->bnorm = S.bnorm;
    out->rnorm_true = S.rnorm_true;
    *inner = S.iter;
    *outer = S.outer;
    if (S.bnorm == 0.0) {
        fill_zero(w->x, A->n, s);
        out->rnorm_true = out->rnorm = 0.0;
    }
    return SPK_OK;
}

__global__ void k_zero64(int64_t m, double *__restrict__ a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

// ------------------------------------------------------------------ single reduction
static SrDesc sr_desc(Workspace *w)
{
    SrDesc a;
    a.d = w->hdesc;
    a.s = w->s;
    a.part = w->srp;
    a.sc = (SrScal *)w->sc;
    return a;
}

// A_i of the single-reduction iteration (m < 0: the SpMV of a (re)start).
static int sr_spmv(spk_mat *A, Workspace *w, const SrDesc &a, int m, hipStream_t s)
{
    const dim3 g(A->nblk), t(kBlock);
    if (A->kernel == SPK_KERNEL_SELL) {
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2) hipLaunchKernelGGL((k_sr_spmv_sell<int16_t, U>), g, t, 0, s, a, m);
            else hipLaunchKernelGGL((k_sr_spmv_sell<int32_t, U>), g, t, 0, s, a, m);
        });
    } else if (A->kernel == SPK_KERNEL_STREAM) {
        hipLaunchKernelGGL(k_sr_spmv_stream, g, t, 0, s, a, m);
    } else {
        SPK_TRY(launch_spmv<double>(A, A->val, w->z, w->q, s, w->st, kGateInner64));
        hipLaunchKernelGGL(k_sr_dot, g, t, 0, s, a, m);
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int sr_batch(spk_mat *A, Workspace *w, const SrDesc &a, int K, hipStream_t s)
{
    for (int m = 0; m < K; ++m) {
        hipLaunchKernelGGL(k_sr_update, dim3(A->nblk), dim3(kBlock), 0, s, a, m);
        SPK_TRY(sr_spmv(A, w, a, m, s));
    }
    hipLaunchKernelGGL(k_sr_advance, dim3(1), dim3(64), 0, s, a.sc, K);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

// (Re)start at iteration b from the residual in r: u, w and their partials.
static int sr_start(spk_mat *A, Workspace *w, const SrDesc &a, int b, hipStream_t s)
{
    hipLaunchKernelGGL(k_sr_rebase, dim3(1), dim3(64), 0, s, a.sc, b);
    hipLaunchKernelGGL(k_sr_setup, dim3(A->nblk), dim3(kBlock), 0, s, a, b & 1);
    SPK_HIP(hipGetLastError());
    return sr_spmv(A, w, a, -1, s);
}

// FP64 single-reduction Jacobi-PCG on w->x (already initialised); the same
// stopping rule, restarts and results as solve64.
static int solve_sr(spk_mat *A, Workspace *w, const spk_ksp_opts &o, int hist_len, hipStream_t s,
                    SolveOut *out)
{
    if (!w->s) {
        SPK_HIP(hipMalloc((void **)&w->s, sizeof(double) * std::max(A->n, 1)));
        SPK_HIP(hipMalloc((void **)&w->srp, sizeof(double) * 6 * std::max(A->nblk, 1)));
        SPK_HIP(hipMalloc(&w->sc, sizeof(SrScal)));
        w->bytes += 8 * (int64_t)std::max(A->n, 1) + 48 * (int64_t)std::max(A->nblk, 1) + sizeof(SrScal);
    }
    const SrDesc a = sr_desc(w);
    const int K = o.graph_k > 0 ? o.graph_k : 8;
    const bool use_graph = o.graph_k > 0;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, w->st, o.rtol, o.atol, o.maxit, 0,
                       o.inner_rtol, o.inner_maxit, o.max_outer, hist_len);
    SPK_TRY(launch_resid(A, w, kResSetup, false, s));
    SPK_TRY(sr_start(A, w, a, 0, s));
    if (use_graph && (!w->gsr || w->gsr_k != K)) {
        if (w->gsr) { hipGraphExecDestroy(w->gsr); w->gsr = nullptr; }
        hipGraph_t graph = nullptr;
        SPK_HIP(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
        const int rc = sr_batch(A, w, a, K, w->cap);
        const hipError_t e = hipStreamEndCapture(w->cap, &graph);
        if (rc) { if (graph) hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
        const hipError_t e2 = hipGraphInstantiate(&w->gsr, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e2 != hipSuccess) { w->gsr = nullptr; return hip_fail(e2, "hipGraphInstantiate", __FILE__, __LINE__); }
        w->gsr_k = K;
    }
    int restarts = 0;
    for (;;) {
        SPK_TRY(read_state(w, s));
        if (w->pst->status == SPK_RUNNING) {
            const int max_batches = (std::max(o.maxit - w->pst->iter, 0) + K - 1) / K + 2;
            int launched = 0, checked = 0;
            for (;;) {
                if (launched - checked < 2 && launched < max_batches) {
                    if (use_graph) SPK_HIP(hipGraphLaunch(w->gsr, s));
                    else SPK_TRY(sr_batch(A, w, a, K, s));
                    const int slot = launched % 4;
                    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, w->st, &w->pstatus[2 * slot]);
                    SPK_HIP(hipEventRecord(w->ev[slot], s));
                    ++launched;
                    continue;
                }
                if (checked == launched) {
                    SPK_HIP(hipStreamSynchronize(s));
                    set_error("single-reduction solver did not stop within %d batches", max_batches);
                    return SPK_EHIP;
                }
                const int slot = checked % 4;
                SPK_HIP(hipEventSynchronize(w->ev[slot]));
                ++checked;
                if (w->pstatus[2 * slot] != SPK_RUNNING) break;
            }
            SPK_HIP(hipStreamSynchronize(s));
        }
        SPK_TRY(launch_resid(A, w, kResTrue, false, s));
        SPK_TRY(read_state(w, s));
        const SysState &S = *w->pst;
        const bool conv = S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL;
        if (conv && S.bnorm > 0 && S.iter > 0 && S.rnorm_true > S.thresh) {
            if (restarts == 3) {
                out->reason = SPK_DIVERGED_BREAKDOWN;
                break;
            }
            ++restarts;
            hipLaunchKernelGGL(k_state_restart, dim3(1), dim3(64), 0, s, w->st);
            SPK_TRY(sr_start(A, w, a, S.iter, s));
            continue;
        }
        out->reason = S.status;
        if (conv && S.iter > 0)
            out->reason = S.rnorm_true <= S.rtol * S.bnorm ? SPK_CONVERGED_RTOL : SPK_CONVERGED_ATOL;
        break;
    }
    const SysState &S = *w->pst;
    out->iterations = S.iter;
    out->restarts = restarts;
    out->rnorm0 = S.rnorm0;
    out->rnorm = (S.status == SPK_CONVERGED_RTOL || S.status == SPK_CONVERGED_ATOL) && S.iter > 0
                     ? S.rnorm_true : S.rnorm;
    out->bnorm = S.bnorm;
    out->rnorm_true = S.rnorm_true;
    if (S.bnorm == 0.0) {
        fill_zero(w->x, A->n, s);
        out->rnorm_true = 0.0;
        out->rnorm = 0.0;
    }
    return SPK_OK;
}

static void fill_zero(double *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxBlocksSingle) g = kMaxBlocksSingle;
    hipLaunchKernelGGL(k_zero64, dim3((int)g), dim3(kBlock), 0, s, n, p);
}

static int grid_n(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxBlocksSingle) g = kMaxBlocksSingle;
    return (int)(g < 1 ? 1 : g);
}

// One Chebyshev step: fused SpMV + update for the SELL and stream families,
// SpMV into tmp then the update pass for the others (V = double, or float
// with the handle's FP32 values).
template <class V>
int cheb_step(spk_mat *A, const ChebStep<V> &c, V *tmp, hipStream_t s)
{
    constexpr bool f64 = std::is_same<V, double>::value;
    const dim3 g(A->nblk), t(kBlock);
    if (A->kernel == SPK_KERNEL_SELL) {
        const SellView sv{A->sell_ptr, A->sell_col, A->sell_len, A->sell_plain, A->sell_len16, A->sell_perm, A->sell_mask};
        // up to one wavefront per slice (no partial sums to keep per block)
        const dim3 gs(std::max(1, std::min(ceil_div(ceil_div(A->n, kSell), kBlock / kWave), 16384)));
        const int n = A->n;
        const V *sval = f64 ? (const V *)A->sell_val : (const V *)A->sell_val32;
        if (!sval) { set_error("internal: no SELL values of this precision"); return SPK_EINVAL; }
        with_sell_u(A->sell_u, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            if (A->sell_cw == 2) hipLaunchKernelGGL((k_cheb_sell<V, int16_t, U>), gs, t, 0, s, n, sv, sval, c);
            else hipLaunchKernelGGL((k_cheb_sell<V, int32_t, U>), gs, t, 0, s, n, sv, sval, c);
        });
    } else if (A->kernel == SPK_KERNEL_STREAM) {
        const V *val = f64 ? (const V *)A->val : (const V *)A->val32;
        hipLaunchKernelGGL((k_cheb_stream<V>), g, t, 0, s, A->n, A->R, A->ntiles, A->nblk, A->rowptr, A->col, val,
                           c);
    } else {
        const V *val = f64 ? (const V *)A->val : (const V *)A->val32;
        SPK_TRY(launch_spmv<V>(A, val, c.dk, tmp, s, c.gate, c.gate ? kGateInner64 : kGateNone));
        hipLaunchKernelGGL((k_cheb_update<V>), dim3(grid_n(A->n)), t, 0, s, A->n, (const V *)tmp, c);
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

template int cheb_step<double>(spk_mat *, const ChebStep<double> &, double *, hipStream_t);
template int cheb_step<float>(spk_mat *, const ChebStep<float> &, float *, hipStream_t);

}  // namespace spk

using namespace spk;

extern "C" {

int spk_pc_chebyshev(const spk_mat *Ac, const double *b, double *x, double *r_out, int32_t steps,
                     double emin, double emax, int32_t x0_nonzero, void *stream)
{
    spk_mat *A = const_cast<spk_mat *>(Ac);
    if (!A) { set_error("A is NULL"); return SPK_EINVAL; }
    const int64_t n = A->n;
    if (n > 0 && (!b || !x)) { set_error("NULL b or x"); return SPK_EINVAL; }
    if (steps < 0) { set_error("steps = %d < 0", steps); return SPK_EINVAL; }
    auto overlap = [n](const double *a, const double *c) { return a && c && a < c + n && c < a + n; };
    if (n > 0 && (overlap(b, x) || overlap(r_out, x) || overlap(r_out, b))) {
        set_error("b, x and r_out must not overlap");
        return SPK_EINVAL;
    }
    if (A->stats.zero_diag) {
        set_error("%d rows without a nonzero diagonal", A->stats.zero_diag);
        return SPK_EZERODIAG;
    }
    if (!(emax > 0.0)) emax = A->info.gershgorin;
    if (!(emin > 0.0)) emin = emax / 10.0;
    if (!(emin > 0.0) || !(emax > emin) || !std::isfinite(emax)) {
        set_error("spectral interval [%g, %g]: need 0 < emin < emax", emin, emax);
        return SPK_EINVAL;
    }
    if (n == 0) return SPK_OK;
    hipStream_t s = (hipStream_t)stream;
    A->stream = s;
    Workspace *w = nullptr;
    SPK_TRY(get_workspace(A, false, &w, s));
    const double theta = 0.5 * (emax + emin), delta = 0.5 * (emax - emin), sigma = theta / delta;
    double *r = r_out ? r_out : w->r;
    double *dbuf[2] = {w->z, w->p};
    double *tmp = w->q;
    if (x0_nonzero) SPK_TRY(launch_spmv<double>(A, A->val, x, tmp, s, nullptr, kGateNone));
    hipLaunchKernelGGL((k_cheb_init<double, double>), dim3(grid_n(n)), dim3(kBlock), 0, s, (int)n, b,
                       x0_nonzero ? (const double *)tmp : nullptr, x, r, dbuf[0], (const double *)A->dinv,
                       1.0 / theta, (const SysState *)nullptr, (double *)nullptr);
    SPK_HIP(hipGetLastError());
    double rho = 1.0 / sigma;
    for (int k = 0; k < steps; ++k) {
        const bool last = k == steps - 1;
        if (last && !r_out) {  // the residual is not wanted: skip the last SpMV
            hipLaunchKernelGGL((k_cheb_last<double>), dim3(grid_n(n)), dim3(kBlock), 0, s, (int)n,
                               (const double *)dbuf[k & 1], x, (const SysState *)nullptr);
            SPK_HIP(hipGetLastError());
            break;
        }
        const double rho_next = 1.0 / (2.0 * sigma - rho);
        ChebStep<double> c;
        c.dk = dbuf[k & 1];
        c.dn = last ? nullptr : dbuf[(k + 1) & 1];
        c.r = r;
        c.x = x;
        c.dinv = A->dinv;
        c.c1 = rho_next * rho;
        c.c2 = 2.0 * rho_next / delta;
        SPK_TRY(cheb_step(A, c, tmp, s));
        rho = rho_next;
    }
    return SPK_OK;
}

void spk_ksp_opts_default(spk_ksp_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->atol = 0.0;
    o->maxit = 10000;
    o->precision = SPK_PREC_FP64;
    o->x0_nonzero = 0;
    o->graph_k = 8;
    o->inner_rtol = 0.0;  // automatic: see inner_rtol_of()
    o->inner_maxit = 10000;
    o->max_outer = 100;
    o->hist = nullptr;
    o->hist_len = 0;
}

int spk_ksp_solve(spk_mat *A, const double *b, double *x, const spk_ksp_opts *opts,
                  spk_ksp_result *res, void *stream)
{
    const double t0 = spk_now();
    if (!A || !res) { set_error("NULL argument"); return SPK_EINVAL; }
    memset(res, 0, sizeof(*res));
    spk_ksp_opts o;
    if (opts) o = *opts;
    else spk_ksp_opts_default(&o);
    if (A->n > 0 && (!b || !x)) { set_error("NULL b or x"); return SPK_EINVAL; }
    if (!(o.rtol >= 0) || !(o.atol >= 0) || o.maxit < 0 || o.graph_k < 0 || o.graph_k > 1024 ||
        o.precision < SPK_PREC_FP64 || o.precision > SPK_PREC_MIXED_IR || o.hist_len < 0 ||
        (o.hist_len > 0 && !o.hist) || !(o.inner_rtol >= 0 && o.inner_rtol < 1) || o.inner_maxit < 1 || o.max_outer < 0) {
        set_error("invalid solver options");
        return SPK_EINVAL;
    }
    if (A->stats.zero_diag) {
        set_error("%d rows have no stored or a zero diagonal (Jacobi needs 1/a_ii)",
                  A->stats.zero_diag);
        return SPK_EZERODIAG;
    }
    hipStream_t s = (hipStream_t)stream;
    A->stream = s;
    if (A->n == 0) {
        res->reason = SPK_CONVERGED_ATOL;
        res->seconds = spk_now() - t0;
        return SPK_OK;
    }
    const bool mixed = o.precision != SPK_PREC_FP64;
    if (mixed && o.single_reduction) {
        set_error("single_reduction needs precision SPK_PREC_FP64");
        return SPK_EINVAL;
    }
    if (o.profile && o.single_reduction) {
        set_error("profile is not available with single_reduction");
        return SPK_EINVAL;
    }
    if (mixed) SPK_TRY(ensure_f32(A, s));
    Workspace *w = nullptr;
    SPK_TRY(get_workspace(A, mixed, &w, s));
    if (o.hist_len > w->hist_cap) {
        // the history buffer is part of the descriptor baked into the graphs
        SPK_HIP(hipStreamSynchronize(s));
        if (w->g64) { hipGraphExecDestroy(w->g64); w->g64 = nullptr; }
        if (w->gmix) { hipGraphExecDestroy(w->gmix); w->gmix = nullptr; }
        if (w->gsr) { hipGraphExecDestroy(w->gsr); w->gsr = nullptr; }
        if (w->hist) hipFree(w->hist);
        w->hist = nullptr;
        SPK_HIP(hipMalloc(&w->hist, sizeof(double) * o.hist_len));
        w->bytes += 8 * (int64_t)(o.hist_len - w->hist_cap);
        w->hist_cap = o.hist_len;
        w->hdesc.hist = w->hist;
    }
    if (w->hist && o.hist_len > 0) SPK_HIP(hipMemsetAsync(w->hist, 0xff, sizeof(double) * o.hist_len, s));
    SPK_HIP(hipMemcpyAsync(w->b, b, sizeof(double) * A->n, hipMemcpyDeviceToDevice, s));
    if (o.x0_nonzero) SPK_HIP(hipMemcpyAsync(w->x, x, sizeof(double) * A->n, hipMemcpyDeviceToDevice, s));
    else fill_zero(w->x, A->n, s);
    SPK_HIP(hipGetLastError());

    SolveOut out;
    int inner = 0, outer = 0, fallback = 0;
    w->prof = o.profile != 0;
    w->pev_used = 0;
    if (mixed) {
        SPK_TRY(solve_mixed(A, w, o, o.hist_len, s, &out, &inner, &outer));
        if (out.reason == SPK_DIVERGED_STAGNATION) {
            // finish in FP64 from the current x
            fallback = 1;
            if (o.hist_len > 0) SPK_HIP(hipMemcpyAsync(o.hist, w->hist, sizeof(double) * o.hist_len,
                                                      hipMemcpyDeviceToHost, s));
            SolveOut o64;
            spk_ksp_opts o2 = o;
            o2.maxit = std::max(o.maxit - inner, 1);
            SPK_TRY(solve64(A, w, o2, true, 0, s, &o64));
            const double r0 = out.rnorm0;
            out = o64;
            out.rnorm0 = r0;
        }
    } else if (o.single_reduction) {
        SPK_TRY(solve_sr(A, w, o, o.hist_len, s, &out));
    } else {
        SPK_TRY(solve64(A, w, o, false, o.hist_len, s, &out));
    }
    SPK_HIP(hipMemcpyAsync(x, w->x, sizeof(double) * A->n, hipMemcpyDeviceToDevice, s));
    if (o.hist_len > 0 && !fallback)
        SPK_HIP(hipMemcpyAsync(o.hist, w->hist, sizeof(double) * o.hist_len, hipMemcpyDeviceToHost, s));
    SPK_HIP(hipStreamSynchronize(s));
    if (w->prof) {
        // the product launches of the counted iterations, in launch order
        int want = mixed && !fallback ? inner : out.iterations, got = 0;
        double ms = 0.0;
        for (int i = 0; i < w->pev_used && got < want; ++i) {
            if (!w->alive[i]) continue;
            float e = 0.f;
            SPK_HIP(hipEventElapsedTime(&e, w->pev[2 * i], w->pev[2 * i + 1]));
            ms += e;
            ++got;
        }
        res->product_ms = ms;
        res->product_launches = got;
        w->prof = false;
    }
    res->reason = out.reason;
    res->iterations = out.iterations;
    res->inner_iterations = inner;
    res->outer_steps = outer;
    res->restarts = out.restarts;
    res->fallback_fp64 = fallback;
    res->rnorm0 = out.rnorm0;
    res->rnorm = out.rnorm;
    res->bnorm = out.bnorm;
    res->true_rel_residual = out.bnorm > 0 ? out.rnorm_true / out.bnorm : 0.0;
    res->seconds = spk_now() - t0;
    return SPK_OK;
}

}  // extern "C"
