// Continuous-batching solve server (Response A6 of Sec. 4: many
// different-size problems solved simultaneously on one GPU).
//
//  * Requests are copied at submit and queued (FIFO).  Between batched steps,
//    queued requests are admitted while a slot and room in the device arena
//    (the HBM budget) are free; the upload goes through pinned staging
//    (Response A4).
//  * Every active system stays resident (matrix, FP32 copy, Krylov vectors,
//    scalars) until it finishes.  One batched step runs K iterations of every
//    active system: each kernel launch serves the whole slot table, and each
//    system reduces over its own blocks only, so a system's bits do not depend
//    on its neighbours in the batch.
//  * Statuses come back with one small copy per step, two steps in flight;
//    finished systems are retired asynchronously (true residual, x download).
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "krylov.hpp"
#include "runtime.hpp"

namespace spk {

enum : int { kQueued = 0, kActive = 1, kRetiring = 2, kDone = 3 };

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    // host copy of the system: in the pinned pool when it has room (the
    // upload is then a plain DMA), otherwise in pageable vectors that go
    // through the staging buffers
    int64_t pin_off = -1, pin_len = 0;
    int32_t *h_rowptr = nullptr, *h_col = nullptr;
    double *h_val = nullptr, *h_b = nullptr;
    std::vector<int32_t> rowptr, col;
    std::vector<double> val, b;
    spk_ksp_opts opts{};
    int mixed = 0;
    int R = 256, ntiles = 0, nblk = 0;
    // SELL-64 copy for large systems (built on the device at admission from
    // the uploaded CSR; slice offsets computed here at submit)
    int sell = 0, sell_u = 2;
    int64_t sell_nnz = 0;
    std::vector<int32_t> sell_ptr;
    int64_t bytes = 0;
    int state = kQueued;
    int slot = -1;
    std::vector<double> x;
    spk_ksp_result res{};
    double t_submit = 0, t_done = 0;
};

// First-fit allocator over [0, size) with 256-byte granules.
class Arena {
  public:
    void init(int64_t size) { free_[0] = size; total_ = size; }
    int64_t alloc(int64_t bytes)
    {
        bytes = (bytes + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = (bytes + 255) & ~int64_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }
    int64_t total() const { return total_; }

  private:
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0, total_ = 0;
};

struct Slot {
    Request *req = nullptr;
    int64_t off = -1, len = 0;
    SysDesc desc{};
    int restarts = 0;
    int fallback = 0;
    int mixed = 0;
    double *px = nullptr;  // pinned download buffer (when the pool has no room)
    int64_t px_cap = 0;
    int64_t x_off = -1;    // download block in the pinned pool, or -1
    double *x_dst = nullptr;
    hipEvent_t ev = nullptr;
    int64_t first_step = 0;  // first batched step that includes this system
    hipEvent_t ev_up = nullptr;      // upload from the pinned pool done
    int64_t pin_off = -1, pin_len = 0;  // pinned block to release after ev_up
};

#define SPK_TRY_RC(x)                  \
    do {                               \
        const int rc_ = (x);           \
        if (rc_ != SPK_OK) return rc_; \
    } while (0)

constexpr int kTableRing = 4;

constexpr int64_t kStageBytes = 16ll << 20;

}  // namespace spk

using namespace spk;

struct spk_server {
    spk_server_opts o{};
    hipStream_t s = nullptr;
    int dev = 0;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    SysState *d_states = nullptr;             // one per slot
    SysState *p_states[2] = {nullptr, nullptr};  // snapshots of in-flight steps
    hipEvent_t ev_step[2] = {nullptr, nullptr};
    std::deque<int> inflight;                 // snapshot buffers of queued steps
    SysDesc *d_slotdesc = nullptr;            // per-slot descriptor (single launches)
    int32_t *d_slotblk = nullptr;             // per-slot {0, nblk}
    SysDesc *p_slotdesc = nullptr;            // pinned source of d_slotdesc
    int32_t *p_slotblk = nullptr;
    SysState *p_slotstate = nullptr;          // pinned state copy taken at retirement
    // batched tables, three sections of max_slots entries (blk: max_slots + 1):
    // every active system, those with the stream-tile product, those with
    // the SELL product
    SysDesc *d_table = nullptr;
    int32_t *d_blk = nullptr;
    SysDesc *p_table[kTableRing] = {};
    int32_t *p_blk[kTableRing] = {};
    hipEvent_t ev_table[kTableRing] = {};
    int table_buf = 0;
    hipStream_t cs = nullptr;                 // copy stream for uploads
    hipEvent_t ev_up = nullptr;
    int64_t step_id = 0;                      // id of the next batched step
    std::deque<int64_t> inflight_id;
    bool table_dirty = true;
    int nsys = 0, nblocks = 0, n_mixed = 0, n_fp64 = 0;
    int nsys_st = 0, nblk_st = 0;             // stream-tile product section
    int nsys_sl = 0, nblk_sl = 0, u_sl = 2;   // SELL product section
    char *stage[2] = {nullptr, nullptr};
    hipEvent_t ev_stage[2] = {nullptr, nullptr};
    int stage_i = 0;
    char *pin_base = nullptr;                 // pinned pool for submitted systems
    Arena pin_arena;
    std::deque<Request *> queue;
    std::map<uint64_t, Request *> tickets;
    std::deque<uint64_t> done;  // finished tickets not yet reported by spk_server_completed
    uint64_t next_ticket = 1;
    std::mutex mu;
};

namespace spk {

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

// A served system gets the SELL-64 product (int16 offsets) when its rows are
// short (<= 64), its slices pad by at most 15 % and every |col - row| fits
// int16, whatever its size: when every active system takes the same product
// kernel, an iteration of the batched step is three launches instead of four
// (the stream-tile section then holds only the systems SELL cannot take).
// Launches, not bytes, bound the small systems, so the layout's build at
// admission (two small kernels) pays for itself within a step.

static int sell_plain_bits(int64_t stored, int nslices, int n)
{
    return sell_load_policy(stored, 2, nslices, n, 6, kIterCacheBudget);
}

// Device bytes a request occupies in the arena.
static int64_t request_bytes(const Request &q)
{
    const int64_t n = q.n, nz = q.nnz;
    int64_t b = align256(4 * (n + 1)) + align256(4 * nz) + align256(8 * nz) + align256(8 * n) /*dinv*/ +
                align256(8 * n) /*b*/ + align256(8 * n) /*x*/ + 4 * align256(8 * n) /*r z p q*/ +
                align256(8 * kNumPart * (int64_t)std::max(q.nblk, 1));
    if (q.mixed) b += align256(4 * nz) + align256(4 * n) + 5 * align256(4 * n);
    if (q.sell) {
        const int64_t ns = (n + kSell - 1) / kSell;
        b += align256(4 * (ns + 1)) + align256(2 * q.sell_nnz) + align256(n) + align256(8 * q.sell_nnz);
        b += align256(8 * n);  // second p buffer of the fused iteration
        if (q.mixed) b += align256(4 * q.sell_nnz) + align256(4 * n);
    }
    return b;
}

static int upload(spk_server *S, void *dst, const void *src, size_t bytes)
{
    for (size_t off = 0; off < bytes; off += kStageBytes) {
        const size_t len = std::min((size_t)kStageBytes, bytes - off);
        const int i = S->stage_i;
        S->stage_i ^= 1;
        SPK_HIP(hipEventSynchronize(S->ev_stage[i]));
        memcpy(S->stage[i], (const char *)src + off, len);
        SPK_HIP(hipMemcpyAsync((char *)dst + off, S->stage[i], len, hipMemcpyHostToDevice, S->cs));
        SPK_HIP(hipEventRecord(S->ev_stage[i], S->cs));
    }
    return SPK_OK;
}

static One slot_batch(spk_server *S, int k) { return One{S->slots[k].desc}; }

// Start an FP64 solve of slot k from the x in its buffer (setup residual).
static int start_fp64(spk_server *S, int k, const spk_ksp_opts &o, bool init_state)
{
    Slot &sl = S->slots[k];
    const One b = slot_batch(S, k);
    if (init_state)
        hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, S->s, sl.desc.st, o.rtol, o.atol,
                           o.maxit, 0, o.inner_rtol, o.inner_maxit, o.max_outer, 0);
    hipLaunchKernelGGL((k_resid_stream<kGateNone, One>), dim3(sl.desc.nblk), dim3(kBlock), 0, S->s, b);
    hipLaunchKernelGGL((k_fin_resid<kGateNone, One>), dim3(1), dim3(kBlock), 0, S->s, b, (int)kResSetup);
    hipLaunchKernelGGL(k_setup64<One>, dim3(sl.desc.nblk), dim3(kBlock), 0, S->s, b);
    hipLaunchKernelGGL(k_fin_setup64<One>, dim3(1), dim3(kBlock), 0, S->s, b);
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static __global__ void k_srv_zero(int64_t m, double *__restrict__ a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

static __global__ void k_srv_diag(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ dinv,
                           float *__restrict__ dinv32)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) d += val[k];
        const double v = 1.0 / d;  // nonzero: checked on the host at submit
        dinv[i] = v;
        if (dinv32) dinv32[i] = (float)v;
    }
}

static __global__ void k_srv_f32(int64_t m, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

static int grid1(int64_t m)
{
    int64_t g = (m + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

// Place request q in free slot k (arena space already reserved at sl.off).
static int admit(spk_server *S, Request *q, int k, int64_t off)
{
    Slot &sl = S->slots[k];
    sl.req = q;
    sl.off = off;
    sl.len = q->bytes;
    sl.restarts = 0;
    sl.fallback = 0;
    sl.mixed = q->mixed;
    char *p = S->arena_base + off;
    auto take = [&](int64_t bytes) {
        char *r = p;
        p += align256(bytes);
        return r;
    };
    const int64_t n = q->n, nz = q->nnz;
    SysDesc &d = sl.desc;
    d = SysDesc{};
    d.n = q->n;
    d.R = q->R;
    d.ntiles = q->ntiles;
    d.nblk = q->nblk;
    int32_t *rowptr = (int32_t *)take(4 * (n + 1));
    int32_t *col = (int32_t *)take(4 * nz);
    double *val = (double *)take(8 * nz);
    double *dinv = (double *)take(8 * n);
    double *b = (double *)take(8 * n);
    d.x = (double *)take(8 * n);
    d.r = (double *)take(8 * n);
    d.z = (double *)take(8 * n);
    d.p = (double *)take(8 * n);
    d.q = (double *)take(8 * n);
    d.partials = (double *)take(8 * kNumPart * (int64_t)std::max(q->nblk, 1));
    float *val32 = nullptr, *dinv32 = nullptr;
    if (q->mixed) {
        val32 = (float *)take(4 * nz);
        dinv32 = (float *)take(4 * n);
        d.r32 = (float *)take(4 * n);
        d.z32 = (float *)take(4 * n);
        d.p32 = (float *)take(4 * n);
        d.q32 = (float *)take(4 * n);
        d.d32 = (float *)take(4 * n);
    }
    int32_t *sell_ptr = nullptr;
    int16_t *sell_col = nullptr;
    uint8_t *sell_len = nullptr;
    double *sell_val = nullptr;
    float *sell_val32 = nullptr;
    if (q->sell) {
        const int64_t ns = (n + kSell - 1) / kSell;
        sell_ptr = (int32_t *)take(4 * (ns + 1));
        sell_col = (int16_t *)take(2 * q->sell_nnz);
        sell_len = (uint8_t *)take(n);
        sell_val = (double *)take(8 * q->sell_nnz);
        if (q->mixed) sell_val32 = (float *)take(4 * q->sell_nnz);
        // SELL systems take the fused iteration (B, then the p/x pass fused
        // into the next product): its second p buffers
        d.p2 = (double *)take(8 * n);
        if (q->mixed) d.p2_32 = (float *)take(4 * n);
        d.sell_cw = 2;
        d.sell_ptr = sell_ptr;
        d.sell_col = sell_col;
        d.sell_len = sell_len;
        d.sell_val = sell_val;
        d.sell_val32 = sell_val32;
        // ordinary loads when the layout and the iteration's vectors fit the
        // Infinity Cache (the handle's rule), else nontemporal
        d.sell_plain = sell_plain_bits(q->sell_nnz, (int)ns, q->n);
    }
    d.rowptr = rowptr;
    d.col = col;
    d.val = val;
    d.val32 = val32;
    d.dinv = dinv;
    d.dinv32 = dinv32;
    d.b = b;
    d.st = S->d_states + k;
    d.hist = nullptr;
    // uploads run on the copy stream and overlap the batched steps already
    // queued on the compute stream; the compute stream waits for them
    if (q->pin_off >= 0) {
        SPK_HIP(hipMemcpyAsync(rowptr, q->h_rowptr, 4 * (n + 1), hipMemcpyHostToDevice, S->cs));
        if (nz) SPK_HIP(hipMemcpyAsync(col, q->h_col, 4 * nz, hipMemcpyHostToDevice, S->cs));
        if (nz) SPK_HIP(hipMemcpyAsync(val, q->h_val, 8 * nz, hipMemcpyHostToDevice, S->cs));
        SPK_HIP(hipMemcpyAsync(b, q->h_b, 8 * n, hipMemcpyHostToDevice, S->cs));
        SPK_HIP(hipEventRecord(sl.ev_up, S->cs));
        sl.pin_off = q->pin_off;  // released once ev_up has completed
        sl.pin_len = q->pin_len;
        q->pin_off = -1;
    } else {
        SPK_TRY_RC(upload(S, rowptr, q->h_rowptr, 4 * (n + 1)));
        if (nz) SPK_TRY_RC(upload(S, col, q->h_col, 4 * nz));
        if (nz) SPK_TRY_RC(upload(S, val, q->h_val, 8 * nz));
        SPK_TRY_RC(upload(S, b, q->h_b, 8 * n));
    }
    if (q->sell)  // the request keeps sell_ptr until it is collected
        SPK_HIP(hipMemcpyAsync(sell_ptr, q->sell_ptr.data(), sizeof(int32_t) * q->sell_ptr.size(),
                               hipMemcpyHostToDevice, S->cs));
    // per-slot descriptor and block table for the single-system launches (the
    // pinned source of slot k is only rewritten after its previous occupant
    // retired, i.e. after this copy of the previous admission completed)
    S->p_slotdesc[k] = d;
    S->p_slotblk[2 * k] = 0;
    S->p_slotblk[2 * k + 1] = q->nblk;
    SPK_HIP(hipMemcpyAsync(S->d_slotdesc + k, S->p_slotdesc + k, sizeof(SysDesc), hipMemcpyHostToDevice, S->cs));
    SPK_HIP(hipMemcpyAsync(S->d_slotblk + 2 * k, S->p_slotblk + 2 * k, 2 * sizeof(int32_t),
                           hipMemcpyHostToDevice, S->cs));
    SPK_HIP(hipEventRecord(S->ev_up, S->cs));
    SPK_HIP(hipStreamWaitEvent(S->s, S->ev_up, 0));
    hipLaunchKernelGGL(k_srv_diag, dim3(grid1(n)), dim3(kBlock), 0, S->s, q->n, rowptr, col, val,
                       dinv, dinv32);
    if (q->mixed && nz)
        hipLaunchKernelGGL(k_srv_f32, dim3(grid1(nz)), dim3(kBlock), 0, S->s, nz, val, val32);
    if (q->sell) {
        hipLaunchKernelGGL(k_sell_fill<int16_t>, dim3(grid1(n)), dim3(kBlock), 0, S->s, q->n, rowptr, col, val,
                           sell_ptr, (const int32_t *)nullptr, sell_col, sell_val, sell_len, (uint16_t *)nullptr);
        if (q->mixed)
            hipLaunchKernelGGL(k_srv_f32, dim3(grid1(q->sell_nnz)), dim3(kBlock), 0, S->s, q->sell_nnz,
                               (const double *)sell_val, sell_val32);
    }
    hipLaunchKernelGGL(k_srv_zero, dim3(grid1(n)), dim3(kBlock), 0, S->s, n, d.x);
    SPK_HIP(hipGetLastError());
    const spk_ksp_opts &o = q->opts;
    if (q->mixed) {
        hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, S->s, d.st, o.rtol, o.atol, o.maxit,
                           o.precision, inner_rtol_of(o), o.inner_maxit, o.max_outer, 0);
        SPK_HIP(hipGetLastError());
    } else {
        const int rc = start_fp64(S, k, o, true);
        if (rc) return rc;
    }
    q->state = kActive;
    q->slot = k;
    sl.first_step = S->step_id;
    // pageable host copies are no longer needed once the staging buffers are
    // drained (pinned blocks are released in progress when ev_up completes)
    if (!q->rowptr.empty()) {
        SPK_HIP(hipEventSynchronize(S->ev_stage[0]));
        SPK_HIP(hipEventSynchronize(S->ev_stage[1]));
    }
    q->h_rowptr = q->h_col = nullptr;
    q->h_val = q->h_b = nullptr;
    std::vector<int32_t>().swap(q->rowptr);
    std::vector<int32_t>().swap(q->col);
    std::vector<double>().swap(q->val);
    std::vector<double>().swap(q->b);
    S->table_dirty = true;
    return SPK_OK;
}

static int admit_queued(spk_server *S)
{
    while (!S->queue.empty()) {
        Request *q = S->queue.front();
        int k = -1;
        for (int i = 0; i < (int)S->slots.size(); ++i)
            if (!S->slots[i].req) { k = i; break; }
        if (k < 0) break;
        const int64_t off = S->arena.alloc(q->bytes);
        if (off < 0) break;  // FIFO: wait until the head fits
        S->queue.pop_front();
        const int rc = admit(S, q, k, off);
        if (rc) return rc;
    }
    return SPK_OK;
}

// Bytes of a batched table of max_slots ms.
static size_t table_bytes(int ms)
{
    return sizeof(SysDesc) * 3 * (size_t)ms + sizeof(int32_t) * 3 * ((size_t)ms + 1);
}

static int rebuild_table(spk_server *S)
{
    const int i = S->table_buf;
    S->table_buf = (S->table_buf + 1) % kTableRing;
    SPK_HIP(hipEventSynchronize(S->ev_table[i]));
    const int ms = (int)S->slots.size();
    SysDesc *pt = S->p_table[i];
    int32_t *pb = S->p_blk[i];
    // section c: table entries pt[c ms ...], block starts pb[c (ms + 1) ...]
    int ns[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
    int nm = 0, nf = 0, u = 2;
    auto put = [&](int c, const SysDesc &d) {
        pt[c * ms + ns[c]] = d;
        pb[c * (ms + 1) + ns[c]] = nb[c];
        nb[c] += (d.nblk + kXcd - 1) / kXcd * kXcd;  // XCD-aligned start of the next system
        ++ns[c];
    };
    for (int k = 0; k < ms; ++k) {
        const Slot &sl = S->slots[k];
        if (!sl.req || sl.req->state != kActive) continue;
        put(0, sl.desc);
        if (sl.desc.sell_cw) {
            put(2, sl.desc);
            u = std::max(u, sl.req->sell_u);
        } else {
            put(1, sl.desc);
        }
        if (sl.mixed) ++nm; else ++nf;
    }
    for (int c = 0; c < 3; ++c) pb[c * (ms + 1) + ns[c]] = nb[c];
    S->nsys = ns[0];
    S->nblocks = nb[0];
    S->nsys_st = ns[1];
    S->nblk_st = nb[1];
    S->nsys_sl = ns[2];
    S->nblk_sl = nb[2];
    S->u_sl = u;
    S->n_mixed = nm;
    S->n_fp64 = nf;
    // one upload of the whole table (each copy on the compute stream is a
    // blit kernel of its own: one instead of up to six per rebuild)
    SPK_HIP(hipMemcpyAsync(S->d_table, pt, table_bytes(ms), hipMemcpyHostToDevice, S->s));
    SPK_HIP(hipEventRecord(S->ev_table[i], S->s));
    S->table_dirty = false;
    return SPK_OK;
}

static_assert(sizeof(SysState) % sizeof(int2) == 0, "SysState is copied as 8-byte words");

static __global__ void k_snapshot(const int2 *__restrict__ src, int2 *__restrict__ dst, int words)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) dst[i] = src[i];
}

// One batched step: K iterations of every active system.  SELL systems run
// the fused iteration (B, then F: the p/x pass fused into the next product;
// a start F after the refinement kernels begins a new CG sequence), the
// stream-tile systems the three kernels A, B, C; B covers all of them.  (A
// step captured as a hipGraph over tables padded to max_slots was measured
// slower: replaying it costs the host more than these launches.)
static int enqueue_step(spk_server *S)
{
    const int ms = (int)S->slots.size();
    const Batch b{S->d_table, S->d_blk, S->nsys};
    const Batch bst{S->d_table + ms, S->d_blk + (ms + 1), S->nsys_st};
    const Batch bsl{S->d_table + 2 * ms, S->d_blk + 2 * (ms + 1), S->nsys_sl};
    const dim3 g(S->nblocks), t(kBlock), f(S->nsys), gst(S->nblk_st), gsl(S->nblk_sl);
    const int K = S->o.graph_k > 0 ? S->o.graph_k : 8;
    hipStream_t st = S->s;
    auto fused = [&](auto vtag, auto start) {
        using V = decltype(vtag);
        constexpr bool kStart = decltype(start)::value;
        with_sell_u(S->u_sl, [&](auto uc) {
            constexpr int U = decltype(uc)::value;
            hipLaunchKernelGGL((k_pcg_fused_sell<V, int16_t, U, kStart, Batch>), gsl, t, 0, st, bsl);
        });
    };
    auto iteration = [&](auto vtag) {
        using V = decltype(vtag);
        if (S->nsys_st) hipLaunchKernelGGL((k_pcg_spmv_stream<V, Batch>), gst, t, 0, st, bst);
        hipLaunchKernelGGL((k_pcg_update<V, Batch>), g, t, 0, st, b);
        if (S->nsys_st) hipLaunchKernelGGL((k_pcg_px<V, Batch>), gst, t, 0, st, bst);
        if (S->nsys_sl) fused(V(), std::false_type{});
    };
    if (S->n_mixed) {
        hipLaunchKernelGGL(k_update_x<Batch>, g, t, 0, st, b);
        if (S->nsys_st) hipLaunchKernelGGL((k_resid_stream<kGateResid, Batch>), gst, t, 0, st, bst);
        if (S->nsys_sl)
            with_sell_u(S->u_sl, [&](auto uc) {
                constexpr int U = decltype(uc)::value;
                hipLaunchKernelGGL((k_resid_sell<kGateResid, int16_t, U, Batch>), gsl, t, 0, st, bsl);
            });
        hipLaunchKernelGGL((k_fin_resid<kGateResid, Batch>), f, t, 0, st, b, (int)kResOuter);
        hipLaunchKernelGGL(k_setup32<Batch>, g, t, 0, st, b);
        hipLaunchKernelGGL(k_fin_setup32<Batch>, f, t, 0, st, b);
        if (S->nsys_st) hipLaunchKernelGGL((k_pcg_p_continue<float, Batch>), gst, t, 0, st, bst);
    }
    if (S->nsys_sl) {  // first products of the sequences that start here
        if (S->n_fp64) fused(double(), std::true_type{});
        if (S->n_mixed) fused(float(), std::true_type{});
    }
    for (int k = 0; k < K; ++k) {
        if (S->n_fp64) iteration(double());
        if (S->n_mixed) iteration(float());
    }
    SPK_HIP(hipGetLastError());
    return SPK_OK;
}

static int begin_retire(spk_server *S, int k)
{
    Slot &sl = S->slots[k];
    Request *q = sl.req;
    const One b = slot_batch(S, k);
    hipLaunchKernelGGL((k_resid_stream<kGateNone, One>), dim3(sl.desc.nblk), dim3(kBlock), 0, S->s, b);
    hipLaunchKernelGGL((k_fin_resid<kGateNone, One>), dim3(1), dim3(kBlock), 0, S->s, b, (int)kResTrue);
    SPK_HIP(hipGetLastError());
    // x lands in a block of the pinned pool (no allocation on this path);
    // only when the pool is full does the slot's own buffer grow, and
    // freeing pinned memory waits for the device
    sl.x_dst = nullptr;
    if (S->pin_base) {
        const int64_t off = S->pin_arena.alloc(sizeof(double) * (int64_t)q->n);
        if (off >= 0) {
            sl.x_off = off;
            sl.x_dst = (double *)(S->pin_base + off);
        }
    }
    if (!sl.x_dst) {
        if (sl.px_cap < q->n) {
            if (sl.px) hipHostFree(sl.px);
            sl.px = nullptr;
            const int64_t cap = std::max<int64_t>(q->n, 1 << 16);
            SPK_HIP(hipHostMalloc((void **)&sl.px, sizeof(double) * cap, hipHostMallocDefault));
            sl.px_cap = cap;
        }
        sl.x_dst = sl.px;
    }
    SPK_HIP(hipMemcpyAsync(sl.x_dst, sl.desc.x, sizeof(double) * q->n, hipMemcpyDeviceToHost, S->s));
    SPK_HIP(hipMemcpyAsync(S->p_slotstate + k, S->d_states + k, sizeof(SysState), hipMemcpyDeviceToHost, S->s));
    SPK_HIP(hipEventRecord(sl.ev, S->s));
    q->state = kRetiring;
    S->table_dirty = true;
    return SPK_OK;
}

// Slot k's retirement copies have landed: check the true residual, then
// finish the request or restart / fall back.
static void release_x(spk_server *S, Slot &sl, int32_t n)
{
    if (sl.x_off >= 0) S->pin_arena.release(sl.x_off, sizeof(double) * (int64_t)n);
    sl.x_off = -1;
    sl.x_dst = nullptr;
}

static int end_retire(spk_server *S, int k, const SysState &st)
{
    Slot &sl = S->slots[k];
    Request *q = sl.req;
    const bool conv = st.status == SPK_CONVERGED_RTOL || st.status == SPK_CONVERGED_ATOL;
    if (!sl.mixed && conv && st.bnorm > 0 && st.iter > 0 && st.rnorm_true > st.thresh &&
        sl.restarts < 3) {
        release_x(S, sl, q->n);
        ++sl.restarts;  // true residual drifted: restart from it
        hipLaunchKernelGGL(k_state_restart, dim3(1), dim3(64), 0, S->s, sl.desc.st);
        hipLaunchKernelGGL(k_setup64<One>, dim3(sl.desc.nblk), dim3(kBlock), 0, S->s, slot_batch(S, k));
        hipLaunchKernelGGL(k_fin_setup64<One>, dim3(1), dim3(kBlock), 0, S->s, slot_batch(S, k));
        SPK_HIP(hipGetLastError());
        q->state = kActive;
        sl.first_step = S->step_id;
        S->table_dirty = true;
        return SPK_OK;
    }
    if (sl.mixed && st.status == SPK_DIVERGED_STAGNATION) {
        release_x(S, sl, q->n);
        // finish in FP64 from the current x
        sl.mixed = 0;
        sl.fallback = 1;
        q->res.inner_iterations = st.iter;
        q->res.outer_steps = st.outer;
        q->res.rnorm0 = st.rnorm0;
        spk_ksp_opts o = q->opts;
        o.maxit = std::max(o.maxit - st.iter, 1);
        const int rc = start_fp64(S, k, o, true);
        if (rc) return rc;
        q->state = kActive;
        sl.first_step = S->step_id;
        S->table_dirty = true;
        return SPK_OK;
    }
    q->x.assign(sl.x_dst, sl.x_dst + q->n);
    release_x(S, sl, q->n);
    spk_ksp_result &r = q->res;
    r.reason = st.status;
    if (!sl.mixed && conv && st.iter > 0 && st.rnorm_true > st.thresh) r.reason = SPK_DIVERGED_BREAKDOWN;
    if (sl.fallback) {
        r.iterations = st.iter;
        r.fallback_fp64 = 1;
    } else if (sl.mixed) {
        r.inner_iterations = st.iter;
        r.outer_steps = st.outer;
        r.rnorm0 = st.rnorm0;
    } else {
        r.iterations = st.iter;
        r.rnorm0 = st.rnorm0;
    }
    r.restarts = sl.restarts;
    r.bnorm = st.bnorm;
    r.rnorm = st.rnorm_true;
    r.true_rel_residual = st.bnorm > 0 ? st.rnorm_true / st.bnorm : 0.0;
    if (st.bnorm == 0.0) {
        std::fill(q->x.begin(), q->x.end(), 0.0);
        r.rnorm = r.true_rel_residual = 0.0;
    }
    q->t_done = spk_now();
    r.seconds = q->t_done - q->t_submit;
    q->state = kDone;
    S->done.push_back(q->ticket);
    q->slot = -1;
    S->arena.release(sl.off, sl.len);
    sl.req = nullptr;
    sl.off = -1;
    return SPK_OK;
}

// Read the state snapshot of the oldest queued step.
static int drain_one_step(spk_server *S)
{
    const int i = S->inflight.front();
    const int64_t id = S->inflight_id.front();
    S->inflight.pop_front();
    S->inflight_id.pop_front();
    SPK_HIP(hipEventSynchronize(S->ev_step[i]));
    const SysState *snap = S->p_states[i];
    for (int k = 0; k < (int)S->slots.size(); ++k) {
        Slot &sl = S->slots[k];
        if (!sl.req || sl.req->state != kActive) continue;
        if (sl.first_step > id) continue;  // joined after this snapshot
        if (snap[k].status != SPK_RUNNING) SPK_TRY_RC(begin_retire(S, k));
    }
    return SPK_OK;
}

// Writes one byte per page of a fresh pinned allocation, with several host
// threads, so that its pages are mapped before submissions copy into them:
// the first CPU write to a page costs a fault (copying a 74 MB system took
// 4.9 ms into untouched pinned pages against 0.96 ms into touched ones).
static void touch_pages(char *p, int64_t bytes)
{
    constexpr int64_t kPage = 4096;
    const int nt = 8;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([=] {
            const int64_t a = bytes * t / nt / kPage * kPage, e = bytes * (t + 1) / nt;
            for (int64_t o = a; o < e; o += kPage) p[o] = 0;
        });
    for (auto &x : th) x.join();
}

}  // namespace spk

extern "C" {

void spk_server_opts_default(spk_server_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->hbm_budget_bytes = 8ll << 30;
    o->max_slots = 64;
    o->graph_k = 8;
    o->max_blocks_per_system = 2048;
    o->pinned_bytes = 1ll << 30;
}

int spk_server_destroy(spk_server *S);

int spk_server_create(const spk_server_opts *opts, void *stream, spk_server **out)
{
    if (!out) { set_error("out is NULL"); return SPK_EINVAL; }
    *out = nullptr;
    spk_server_opts o;
    if (opts) o = *opts;
    else spk_server_opts_default(&o);
    if (o.hbm_budget_bytes < (1 << 20) || o.max_slots < 1 || o.max_slots > 4096 || o.graph_k < 1 ||
        o.graph_k > 256 || o.max_blocks_per_system < 1 || o.max_blocks_per_system > 8192 ||
        o.pinned_bytes < 0) {
        set_error("invalid server options");
        return SPK_EINVAL;
    }
    spk_server *S = new (std::nothrow) spk_server();
    if (!S) { set_error("out of host memory"); return SPK_ENOMEM; }
    S->o = o;
    S->s = (hipStream_t)stream;
    int rc = SPK_OK;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == SPK_OK) rc = hip_fail(e, what, __FILE__, __LINE__);
    };
    chk(hipGetDevice(&S->dev), "hipGetDevice");
    chk(hipMalloc(&S->arena_base, o.hbm_budget_bytes), "arena hipMalloc");
    S->arena.init(o.hbm_budget_bytes);
    S->slots.resize(o.max_slots);
    const size_t ms = o.max_slots;
    chk(hipMalloc(&S->d_states, sizeof(SysState) * ms), "states");
    chk(hipMalloc(&S->d_slotdesc, sizeof(SysDesc) * ms), "slot descs");
    chk(hipMalloc(&S->d_slotblk, sizeof(int32_t) * 2 * ms), "slot blocks");
    // batched table: 3 ms descriptors, then 3 (ms + 1) block starts, in one
    // buffer so that a rebuild is one upload
    const size_t tbytes = table_bytes((int)ms);
    chk(hipMalloc(&S->d_table, tbytes), "table");
    if (S->d_table) S->d_blk = (int32_t *)(S->d_table + 3 * ms);
    chk(hipHostMalloc((void **)&S->p_slotdesc, sizeof(SysDesc) * ms, hipHostMallocDefault), "pinned descs");
    chk(hipHostMalloc((void **)&S->p_slotblk, sizeof(int32_t) * 2 * ms, hipHostMallocDefault), "pinned blocks");
    chk(hipHostMalloc((void **)&S->p_slotstate, sizeof(SysState) * ms, hipHostMallocDefault), "pinned states");
    chk(hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking), "copy stream");
    chk(hipEventCreateWithFlags(&S->ev_up, hipEventDisableTiming), "event");
    for (int i = 0; i < 2; ++i) {
        chk(hipHostMalloc((void **)&S->p_states[i], sizeof(SysState) * ms, hipHostMallocDefault), "pinned states");
        chk(hipHostMalloc((void **)&S->stage[i], kStageBytes, hipHostMallocDefault), "pinned staging");
        chk(hipEventCreateWithFlags(&S->ev_step[i], hipEventDisableTiming), "event");
        chk(hipEventCreateWithFlags(&S->ev_stage[i], hipEventDisableTiming), "event");
    }
    for (int i = 0; i < kTableRing; ++i) {
        chk(hipHostMalloc((void **)&S->p_table[i], tbytes, hipHostMallocDefault), "pinned table");
        if (S->p_table[i]) S->p_blk[i] = (int32_t *)(S->p_table[i] + 3 * ms);
        chk(hipEventCreateWithFlags(&S->ev_table[i], hipEventDisableTiming), "event");
    }
    for (auto &sl : S->slots) {
        chk(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming), "event");
        chk(hipEventCreateWithFlags(&sl.ev_up, hipEventDisableTiming), "event");
    }
    if (o.pinned_bytes > 0 && rc == SPK_OK) {
        // best effort: without the pool, submissions use pageable memory
        if (hipHostMalloc((void **)&S->pin_base, o.pinned_bytes, hipHostMallocDefault) == hipSuccess) {
            S->pin_arena.init(o.pinned_bytes);
            touch_pages(S->pin_base, o.pinned_bytes);
        } else {
            S->pin_base = nullptr;
        }
    }
    if (rc == SPK_OK) {
        for (int i = 0; i < kTableRing; ++i) chk(hipEventRecord(S->ev_table[i], S->s), "event record");
        for (int i = 0; i < 2; ++i) chk(hipEventRecord(S->ev_stage[i], S->cs), "event record");
        chk(hipMemsetAsync(S->d_states, 0, sizeof(SysState) * ms, S->s), "memset");
        chk(hipStreamSynchronize(S->s), "sync");
    }
    if (rc != SPK_OK) {
        spk_server_destroy(S);
        return rc;
    }
    *out = S;
    return SPK_OK;
}

int spk_server_submit(spk_server *S, int32_t n, int64_t nnz, const int32_t *rowptr,
                      const int32_t *colind, const double *values, const double *b,
                      const spk_ksp_opts *opts, uint64_t *ticket)
{
    if (!S || !ticket) { set_error("NULL argument"); return SPK_EINVAL; }
    if (n < 1 || nnz < 0 || nnz > 0x7fffffffLL || !rowptr || !b || (nnz > 0 && (!colind || !values))) {
        set_error("invalid system (n = %d, nnz = %lld)", n, (long long)nnz);
        return SPK_EINVAL;
    }
    spk_ksp_opts o;
    if (opts) o = *opts;
    else spk_ksp_opts_default(&o);
    if (!(o.rtol >= 0) || !(o.atol >= 0) || o.maxit < 0 || !(o.inner_rtol >= 0 && o.inner_rtol < 1) || o.inner_maxit < 1 ||
        o.max_outer < 0 || o.precision < SPK_PREC_FP64 || o.precision > SPK_PREC_MIXED_IR) {
        set_error("invalid solver options");
        return SPK_EINVAL;
    }
    // host-side structure checks: everything the kernels index with
    if (rowptr[0] != 0 || rowptr[n] != nnz) {
        set_error("rowptr[0] must be 0 and rowptr[n] = nnz");
        return SPK_EINVAL;
    }
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) { set_error("rowptr not monotone at row %d", i); return SPK_EINVAL; }
    int64_t maxtile[6] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < 6; ++t)
        for (int64_t r0 = 0; r0 < n; r0 += kTileRs[t])
            maxtile[t] = std::max<int64_t>(maxtile[t], rowptr[std::min<int64_t>(r0 + kTileRs[t], n)] - rowptr[r0]);
    Request *q = new (std::nothrow) Request();
    if (!q) { set_error("out of host memory"); return SPK_ENOMEM; }
    q->n = n;
    q->nnz = nnz;
    q->opts = o;
    q->mixed = o.precision != SPK_PREC_FP64;
    q->R = 8;
    for (int t = 0; t < 6; ++t)
        if (maxtile[t] <= TileLds<double>::kCap) { q->R = kTileRs[t]; break; }
    q->ntiles = ceil_div(n, q->R);
    q->nblk = pick_nblk(q->ntiles, S->o.max_blocks_per_system);
    {
        // slice widths from the row pointers; the offsets are checked below
        const int32_t ns = ceil_div(n, kSell);
        int64_t acc = 0;
        int wmax = 0;
        std::vector<int32_t> sp((size_t)ns + 1);
        for (int32_t k = 0; k < ns; ++k) {
            int mx = 0;
            for (int32_t i = k * kSell; i < std::min(n, (k + 1) * kSell); ++i) mx = std::max(mx, rowptr[i + 1] - rowptr[i]);
            wmax = std::max(wmax, mx);
            sp[k] = (int32_t)std::min<int64_t>(acc, 0x7fffffff);
            acc += (int64_t)kSell * mx;
        }
        sp[ns] = (int32_t)std::min<int64_t>(acc, 0x7fffffff);
        if (wmax <= 64 && (double)acc <= 1.15 * (double)nnz && acc < 0x7fff0000LL) {
            q->sell = 1;
            q->sell_u = pick_sell_u(wmax);
            q->sell_nnz = acc;
            q->sell_ptr.swap(sp);
        }
    }
    q->bytes = request_bytes(*q);
    if (q->bytes > S->o.hbm_budget_bytes) {
        set_error("system needs %lld bytes, budget is %lld", (long long)q->bytes,
                  (long long)S->o.hbm_budget_bytes);
        delete q;
        return SPK_EBUDGET;
    }
    // host copy: pinned pool if it has room, else pageable memory
    const int64_t hb = align256(4 * ((int64_t)n + 1)) + align256(4 * nnz) + align256(8 * nnz) +
                       align256(8 * (int64_t)n);
    int64_t off = -1;
    if (S->pin_base) {
        std::lock_guard<std::mutex> lk(S->mu);
        off = S->pin_arena.alloc(hb);
    }
    try {
        if (off >= 0) {
            q->pin_off = off;
            q->pin_len = hb;
            char *p = S->pin_base + off;
            q->h_rowptr = (int32_t *)p;
            p += align256(4 * ((int64_t)n + 1));
            q->h_col = (int32_t *)p;
            p += align256(4 * nnz);
            q->h_val = (double *)p;
            p += align256(8 * nnz);
            q->h_b = (double *)p;
        } else {
            q->rowptr.resize((size_t)n + 1);
            q->col.resize((size_t)nnz);
            q->val.resize((size_t)nnz);
            q->b.resize((size_t)n);
            q->h_rowptr = q->rowptr.data();
            q->h_col = q->col.data();
            q->h_val = q->val.data();
            q->h_b = q->b.data();
        }
    } catch (...) {
        delete q;
        set_error("out of host memory");
        return SPK_ENOMEM;
    }
    // one pass over the nonzeros: copy, check the columns, find the diagonal;
    // large systems split the rows over a few host threads (the copy into
    // the pinned pool is what bounds admission when requests queue up)
    int rc = SPK_OK;
    memcpy(q->h_rowptr, rowptr, sizeof(int32_t) * ((size_t)n + 1));
    struct Bad {
        int32_t row = INT32_MAX;
        int32_t col = 0;
        int code = SPK_OK;
        int32_t maxd = 0;  // largest |col - row|
    };
    auto check_rows = [&](int32_t i0, int32_t i1, Bad &bad) {
        int32_t *__restrict__ hc = q->h_col;
        double *__restrict__ hv = q->h_val;
        for (int32_t i = i0; i < i1; ++i) {
            const int32_t a = rowptr[i], e = rowptr[i + 1];
            double d = 0.0;
            int32_t lo = i, hi = i;  // min / max column of the row (and i)
            for (int32_t k = a; k < e; ++k) {
                const int32_t c = colind[k];
                const double v = values[k];
                hc[k] = c;
                hv[k] = v;
                lo = c < lo ? c : lo;
                hi = c > hi ? c : hi;
                d += c == i ? v : 0.0;
            }
            bad.maxd = std::max(bad.maxd, std::max(i - lo, hi - i));
            if (lo < 0 || hi >= n) {
                for (int32_t k = a; k < e; ++k)
                    if (colind[k] < 0 || colind[k] >= n) { bad = {i, colind[k], SPK_EINVAL}; return; }
            }
            if (d == 0.0) { bad = {i, 0, SPK_EZERODIAG}; return; }
        }
    };
    const int nthreads = nnz >= (1 << 20) ? 8 : 1;
    std::vector<Bad> bad(nthreads);
    if (nthreads == 1) {
        check_rows(0, n, bad[0]);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < nthreads; ++t) {
            // row ranges with about equal nonzero counts
            const int64_t k0 = nnz * t / nthreads, k1 = nnz * (t + 1) / nthreads;
            const int32_t i0 = t == 0 ? 0 : (int32_t)(std::upper_bound(rowptr, rowptr + n + 1, (int32_t)k0) - rowptr - 1);
            const int32_t i1 = t == nthreads - 1 ? n : (int32_t)(std::upper_bound(rowptr, rowptr + n + 1, (int32_t)k1) - rowptr - 1);
            th.emplace_back(check_rows, std::max(i0, 0), std::min(i1, n), std::ref(bad[t]));
        }
        for (auto &x : th) x.join();
    }
    Bad first;
    for (const Bad &x : bad)
        if (x.code != SPK_OK && x.row < first.row) first = x;
    if (first.code == SPK_EINVAL) {
        set_error("column %d out of range in row %d", first.col, first.row);
        rc = SPK_EINVAL;
    } else if (first.code == SPK_EZERODIAG) {
        set_error("row %d has no stored or a zero diagonal", first.row);
        rc = SPK_EZERODIAG;
    }
    int32_t maxd = 0;
    for (const Bad &x : bad) maxd = std::max(maxd, x.maxd);
    if (q->sell && maxd > 32767) {  // offsets do not fit int16: stream tiles
        q->sell = 0;
        q->sell_nnz = 0;
        std::vector<int32_t>().swap(q->sell_ptr);
        q->bytes = request_bytes(*q);
    }
    if (rc != SPK_OK) {
        if (q->pin_off >= 0) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->pin_arena.release(q->pin_off, q->pin_len);
        }
        delete q;
        return rc;
    }
    memcpy(q->h_b, b, sizeof(double) * (size_t)n);
    q->t_submit = spk_now();
    std::lock_guard<std::mutex> lk(S->mu);
    q->ticket = S->next_ticket++;
    S->tickets[q->ticket] = q;
    S->queue.push_back(q);
    *ticket = q->ticket;
    return SPK_OK;
}

int spk_server_progress(spk_server *S, int32_t max_steps)
{
    if (!S || max_steps < 0) { set_error("bad argument"); return SPK_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    constexpr int kDepth = 2;
    for (int step = 0; step <= max_steps; ++step) {
        for (int k = 0; k < (int)S->slots.size(); ++k) {
            Slot &sl = S->slots[k];
            // return pinned host blocks whose upload has completed
            if (sl.pin_off >= 0) {
                const hipError_t e = hipEventQuery(sl.ev_up);
                if (e == hipSuccess) {
                    S->pin_arena.release(sl.pin_off, sl.pin_len);
                    sl.pin_off = -1;
                } else if (e != hipErrorNotReady) {
                    return hip_fail(e, "upload event", __FILE__, __LINE__);
                }
            }
            // finish retirements whose copies have landed
            if (!sl.req || sl.req->state != kRetiring) continue;
            const hipError_t e = hipEventQuery(sl.ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return hip_fail(e, "retire event", __FILE__, __LINE__);
            const SysState st = S->p_slotstate[k];
            SPK_TRY_RC(end_retire(S, k, st));
        }
        if (step == max_steps) break;
        SPK_TRY_RC(admit_queued(S));
        if (S->table_dirty) SPK_TRY_RC(rebuild_table(S));
        if (S->nsys > 0) {
            const int i = S->inflight.empty() ? 0 : (S->inflight.back() ^ 1);
            if ((int)S->inflight.size() >= kDepth) SPK_TRY_RC(drain_one_step(S));
            SPK_TRY_RC(enqueue_step(S));
            // snapshot of every slot's state into pinned host memory (a
            // kernel's stores: a device-to-host copy would run as a blit)
            const int words = (int)(sizeof(SysState) * S->slots.size() / sizeof(int2));
            hipLaunchKernelGGL(k_snapshot, dim3(ceil_div(words, kBlock)), dim3(kBlock), 0, S->s,
                               (const int2 *)S->d_states, (int2 *)S->p_states[i], words);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "state snapshot", __FILE__, __LINE__);
            const hipError_t e2 = hipEventRecord(S->ev_step[i], S->s);
            if (e2 != hipSuccess) return hip_fail(e2, "event", __FILE__, __LINE__);
            S->inflight.push_back(i);
            S->inflight_id.push_back(S->step_id++);
        } else {
            while (!S->inflight.empty()) SPK_TRY_RC(drain_one_step(S));
            bool retiring = false;
            for (auto &sl : S->slots)
                if (sl.req && sl.req->state == kRetiring) retiring = true;
            if (!retiring && S->queue.empty()) break;
            if (retiring) {
                const hipError_t e = hipStreamSynchronize(S->s);
                if (e != hipSuccess) return hip_fail(e, "sync", __FILE__, __LINE__);
            }
        }
    }
    int pending = (int)S->queue.size();
    for (auto &sl : S->slots)
        if (sl.req) ++pending;
    return pending;
}

int spk_server_poll(spk_server *S, uint64_t ticket, double *x_host, spk_ksp_result *res,
                    double *done_time)
{
    if (!S) { set_error("NULL server"); return SPK_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) { set_error("unknown ticket %llu", (unsigned long long)ticket); return SPK_ENOTFOUND; }
    Request *q = it->second;
    if (q->state != kDone) return SPK_EBUSY;
    if (x_host) memcpy(x_host, q->x.data(), sizeof(double) * q->n);
    if (res) *res = q->res;
    if (done_time) *done_time = q->t_done;
    S->tickets.erase(it);
    delete q;
    return SPK_OK;
}

int spk_server_completed(spk_server *S, uint64_t *tickets, int32_t cap)
{
    if (!S || cap < 0 || (cap > 0 && !tickets)) { set_error("bad argument"); return SPK_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t k = 0;
    while (k < cap && !S->done.empty()) {
        tickets[k++] = S->done.front();
        S->done.pop_front();
    }
    return k;
}

int spk_server_destroy(spk_server *S)
{
    if (!S) return SPK_OK;
    hipStreamSynchronize(S->s);
    if (S->cs) hipStreamSynchronize(S->cs);
    for (auto &kv : S->tickets) delete kv.second;
    for (auto &sl : S->slots) {
        if (sl.px) hipHostFree(sl.px);
        if (sl.ev) hipEventDestroy(sl.ev);
        if (sl.ev_up) hipEventDestroy(sl.ev_up);
    }
    for (int i = 0; i < 2; ++i) {
        hipHostFree(S->p_states[i]);
        hipHostFree(S->stage[i]);
        if (S->ev_step[i]) hipEventDestroy(S->ev_step[i]);
        if (S->ev_stage[i]) hipEventDestroy(S->ev_stage[i]);
    }
    for (int i = 0; i < kTableRing; ++i) {
        hipHostFree(S->p_table[i]);
        if (S->ev_table[i]) hipEventDestroy(S->ev_table[i]);
    }
    hipHostFree(S->p_slotdesc);
    hipHostFree(S->p_slotblk);
    hipHostFree(S->p_slotstate);
    if (S->ev_up) hipEventDestroy(S->ev_up);
    if (S->cs) hipStreamDestroy(S->cs);
    hipFree(S->arena_base);
    if (S->pin_base) hipHostFree(S->pin_base);
    hipFree(S->d_states);
    hipFree(S->d_slotdesc);
    hipFree(S->d_slotblk);
    hipFree(S->d_table);
    delete S;
    return SPK_OK;
}

}  // extern "C"
