// Host-side runtime structures of libspk.so.
#pragma once

#include <mutex>
#include <vector>

#include "spmv.hpp"

namespace spk {

struct RowStats {
    unsigned long long sum_len;
    unsigned long long sum_len2;
    int32_t max_len;
    int32_t min_len;
    int32_t bad_rowptr;      // rows with rowptr[i+1] < rowptr[i] or out of [0, nnz]
    int32_t bad_col;         // entries with col outside [0, n)
    int32_t unsorted;        // rows whose columns are not strictly ascending
    int32_t max_delta;       // max |col - row| over the stored entries
    int32_t zero_diag;       // rows without a nonzero diagonal
    int32_t tile_max[6];     // max nonzeros in an aligned tile of 256,128,64,32,16,8 rows
    unsigned long long sell_padded;  // entries of a SELL-64 layout (64 x longest row per slice)
    unsigned long long gersh_bits;   // bits of max_i sum_j |a_ij| / |a_ii| (non-negative double)
    int32_t hist[33];        // rows by bit length of their length
};

constexpr int kTileRs[6] = {256, 128, 64, 32, 16, 8};

// Load policy of the SELL entries: ordinary (cache-allocating) loads when
// the layout (entries, slice offsets, row lengths in that precision) and the
// n-vectors a pass touches beside it fit the 256 MB Infinity Cache,
// nontemporal loads above.  Measured on 3D 7-point Laplacians: a PCG
// iteration (6 vectors: x, r, z, p, q, dinv) gains from ordinary loads at
// 128^3 (249 MB in all) and loses from 134^3 (285 MB) on; back-to-back
// products (x and y) gain up to 150^3 (293 MB) and lose at 160^3 (355 MB).
constexpr int64_t kIterCacheBudget = 256ll << 20;
constexpr int64_t kSpmvCacheBudget = 288ll << 20;

inline int sell_load_policy(int64_t stored, int cw, int nslices, int n, int vectors, int64_t budget)
{
    const int64_t fixed = 4 * ((int64_t)nslices + 1) + n;
    int bits = 0;
    if ((8 + cw) * stored + fixed + 8ll * vectors * n <= budget) bits |= kSellPlain64;
    if ((4 + cw) * stored + fixed + 4ll * vectors * n <= budget) bits |= kSellPlain32;
    return bits;
}

// Solver workspace of one matrix (allocated on the first solve).
struct Workspace {
    int n = 0;
    int has_mixed = 0;
    SysDesc hdesc{};              // host copy of the descriptor
    SysDesc *ddesc = nullptr;     // device descriptor (read by the kernels)
    SysDesc *pdesc = nullptr;     // pinned staging for descriptor updates
    int32_t *blk_start = nullptr; // device {0, nblk}
    SysState *st = nullptr;       // device scalars
    SysState *pst = nullptr;      // pinned host copy
    int32_t *pstatus = nullptr;   // pinned ring of (status, phase) pairs
    hipEvent_t ev[4] = {};
    double *hist = nullptr;
    int hist_cap = 0;
    double *partials = nullptr;
    double *wpart = nullptr;      // partials of the wide SELL product (large matrices), or null
    int nwpart = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *x = nullptr;          // the solve's iterate (copied in and out)
    double *b = nullptr;          // the solve's right-hand side (copied in)
    float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    // fused iteration (SELL product on the persistent grid): the second p
    // buffers; fused64 / fused32 say which precisions take it (profiled
    // solves do not)
    bool fused64 = false, fused32 = false;
    double *p2 = nullptr;
    float *p2_32 = nullptr;
    hipStream_t cap = nullptr;    // private stream used only to capture graphs
    hipGraphExec_t g64 = nullptr, gmix = nullptr, gsr = nullptr;
    int g64_k = 0, gmix_k = 0, gsr_k = 0;
    // single-reduction solves (allocated on first use)
    double *s = nullptr;          // s = A p
    double *srp = nullptr;        // 2 sets x 3 partial arrays x nblk
    void *sc = nullptr;           // device scalars of the single-reduction recurrences
    int64_t bytes = 0;
    // profiled solves: one event pair around each iteration's product, in
    // launch order; `alive` is cleared for launches queued after the solve
    // had stopped
    bool prof = false;
    std::vector<hipEvent_t> pev;
    std::vector<char> alive;
    int pev_used = 0;
};

}  // namespace spk

namespace spk {
struct MultiWs;
}

struct spk_mat {
    int32_t n = 0;
    int64_t nnz = 0;
    int device = 0;
    int32_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;
    double *dinv = nullptr;
    float *dinv32 = nullptr;
    bool own_csr = true;
    spk::RowStats stats{};
    spk_mat_info info{};
    // SpMV selection
    int kernel = SPK_KERNEL_STREAM;
    int lanes = 0;          // VECTOR: lanes per row
    int R = 256;            // rows per tile (stream kernel and solver row partition)
    int ntiles = 0;
    int nblk = 0;
    // merge path
    int mtiles = 0;
    int32_t *tile_row = nullptr, *tile_k = nullptr, *carry_row = nullptr;
    double *carry_val = nullptr;
    // SELL-64 copy (built when the SELL family is selected)
    int sell_cw = 0;           // column offset width: 2 (int16) or 4 (int32; shared offsets too), 0 = none
    int sell_u = 8;            // entries per load round of the SELL kernels (from the widest slice)
    int64_t sell_nnz = 0;      // stored entries including padding
    int sell_plain = 0;        // kSellPlain64/32 bits: ordinary loads in the Krylov and smoother kernels
    int sell_plain_spmv = 0;   // the same for the standalone products
    bool stream_loads = false; // SPK_MAT_STREAM: always nontemporal
    int32_t *sell_ptr = nullptr;
    void *sell_col = nullptr;
    uint8_t *sell_len = nullptr;
    uint16_t *sell_len16 = nullptr;  // row lengths when some row exceeds 255 entries (sell_len then null)
    int32_t *sell_perm = nullptr;    // SELL-C-sigma: matrix row of each sorted position, or null
    int sell_sigma = 0;              // SELL-C-sigma window (rows), 0: rows in matrix order
    uint32_t *sell_mask = nullptr;   // shared offsets: per-row position masks (sell_col then
                                     // holds each slice's int32 offsets; sell_len is null)
    int64_t sell_idx_bytes = 0;      // bytes of offsets and row lengths / masks
    int sell_req = -1;               // the offset request the layout was built for (setup_sell's cw)
    double *sell_val = nullptr;
    float *sell_val32 = nullptr;
    // column-sliced copy (built when the SLICED family is selected): rows
    // s*n + i hold row i's entries with columns in the s-th eighth of [0, n)
    int32_t *xs_ptr = nullptr;   // 8n + 1 row pointers
    int32_t *xs_col = nullptr;
    double *xs_val = nullptr;
    float *xs_val32 = nullptr;
    void *xs_part = nullptr;     // 8n partial products (FP64 or FP32)
    int xs_merge = 0;            // 1: merge path over the stacked slices, 0: lanes per slice row
    int xs_tiles = 0;            // merge-path tiles of the stacked slices (0: not built)
    int xs_tile_grid = 0;        // blocks of the merge launch (8 x the most tiles of a slice)
    int32_t *xs_tile_row = nullptr, *xs_tile_k = nullptr, *xs_carry_row = nullptr;
    int32_t *xs_slice_tile = nullptr;  // kSlices + 1 tile ranges
    void *xs_carry_val = nullptr;
    spk::Workspace *ws = nullptr;
    spk::MultiWs *mws = nullptr;  // multi-right-hand-side solver workspace
    int64_t bytes = 0;
    // stream of the latest call that queued work on the handle: destroy and
    // re-planning wait for it (and nothing else) before releasing buffers
    mutable hipStream_t stream = nullptr;
};

namespace spk {

// y = A x with the handle's kernel (V = double or float); optional gate for
// launches inside captured solver graphs.
template <class V>
int launch_spmv(const spk_mat *A, const V *val, const V *x, V *y, hipStream_t s,
                const SysState *gate_st, int gate_mode);

void update_info(spk_mat *A);
constexpr double kRuDelta = 0.05;  // default refinement trigger with reliable updates
double inner_rtol_of(const spk_ksp_opts &o);
int ensure_f32(spk_mat *A, hipStream_t s);
void free_multi(spk_mat *A);
// column-sliced layout (xslice.hip)
bool sliced_fits(const spk_mat *A);
int sliced_lanes(const spk_mat *A);
int setup_sliced(spk_mat *A, hipStream_t s);
void free_sliced(spk_mat *A);
int ensure_sliced_f32(spk_mat *A, hipStream_t s);
int setup_sliced_merge(spk_mat *A, hipStream_t s);
bool sliced_skewed(const spk_mat *A);
bool sliced_merge_fits(const spk_mat *A);
template <class V>
int launch_sliced(const spk_mat *A, const V *x, V *y, hipStream_t s, const SysState *gst, int gmode);
template <class V>
struct ChebStep;
// One Chebyshev smoothing step on A (fused with its SpMV where the family
// allows); V = double, or float with the handle's FP32 values.
template <class V>
int cheb_step(spk_mat *A, const ChebStep<V> &c, V *tmp, hipStream_t s);

}  // namespace spk
