// Batches of independent, uneven gridding problems.
//
//   auv_batch_plan      host: validate items, pick bin size and kernel form per
//                       item (autotune table or defaults), lay out a workspace
//   auv_batch_launch    first call: upload item tables, capture
//                         batched binning (5 launches for all items)
//                         -> queue reset -> one persistent IDW launch per
//                         kernel form (sparse window / dense top-k, on two
//                         concurrent branches), + per-item launches for items
//                         they do not cover
//                       into a HIP graph; later calls replay the graph
//   auv_batch_launch_plain  the same items one after another, default sizes
//   auv_batch_autotune  time (bin size, form) candidates per item class
//
// The persistent kernels: each 64-lane wave takes its home queue (one per XCD:
// blocks are dealt round-robin to the 8 XCDs, so block b runs on XCD b % 8),
// pulls (item, tile) work with one atomic per tile, and moves on to the other
// queues when its own is drained.  Items are assigned to queues by longest
// processing time first on an estimated cost, so each XCD's L2 mostly sees
// the bins of a few items.
#include "idw_dense_impl.hpp"
#include "idw_span_impl.hpp"

#include <algorithm>
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

namespace auv {

namespace {

constexpr int kQueues = 8;
constexpr int kBatchDenseK = 16;  // largest max_pts the persistent dense path keeps
constexpr size_t kOvfMax = size_t(1) << 21;  // over-cap list entries at most (32 MiB)

struct IdwItem {
    auv_bin_view bv;
    IdwArgs a;
    WinGeom g;
    int32_t ntx, ntiles;
    int32_t dense, pmode;
    int32_t span;  // sparse items: the span form covers it (else the window form)
    // window items: nodes above the cap go to the over-cap list (cap <= 16,
    // dense keys fit), finished by k_overcap_dense after the persistent kernels
    int32_t cap_list;
};

// Queue heads of both forms, then the over-cap list's entry count.
__global__ void k_reset_queues(int32_t *qhead)
{
    if (threadIdx.x < 2 * kQueues + 1)
        qhead[threadIdx.x] = 0;
}

template <int kPmode, int kChunks>
__device__ inline void run_window(const IdwItem &it, int tile, const win::WinSmem &sm,
                                  win::CapSink sink)
{
    if (!it.cap_list)
        sink.count = nullptr;
    win::window_tile<3, kPmode, true, kChunks, AUV_P_FP32_REBASE>(it.bv, it.a, it.g, tile,
                                                                  it.ntx, sm, 0, 1, nullptr, sink);
}

// The window items' nodes above the cap, one lane per node: the dense form's
// ring search for the cap nearest.  Every tile of a wave's window kernel
// re-did such nodes one at a time, the whole wave per node; clustered
// soundings put hundreds of them in one tile.
__global__ __launch_bounds__(64) void k_overcap_dense(const IdwItem *__restrict__ items,
                                                      const int4 *__restrict__ list,
                                                      const int32_t *__restrict__ count, int cap)
{
    const int n = min(*count, cap);
    for (int e = blockIdx.x * 64 + (int)threadIdx.x; e < n; e += gridDim.x * 64) {
        const int4 v = list[e];
        const IdwItem &it = items[v.x];
        dense::dense_node<3, kBatchDenseK>(it.bv, it.a, v.z, v.y, it.pmode);
    }
}

// Grab the next `grab` work entries of queue q: returns the first (or -1 when
// the queue is drained).  One atomic per grab, issued by lane 0 and broadcast
// (wave-uniform).  Grabbing several tiles at once matters: every wave pulls
// from a few shared counters, and same-address device atomics serialise.
__device__ inline int pull(int32_t *qhead, int q, int len, int grab)
{
    int t = 0;
    if (threadIdx.x == 0)
        t = atomicAdd(&qhead[q], grab);
    t = __builtin_amdgcn_readfirstlane(t);
    return t < len ? t : -1;
}

// Guided grab size: half of the tiles still unclaimed as last seen by this
// wave (`seen`, the queue head after its previous grab) spread over the
// `waves` sharing the queue, at most gmax, at least one.  The grabs shrink
// toward one tile as the queue drains, so no wave is left with a long run of
// expensive tiles at the end while the others idle.
__device__ inline int grab_size(int seen, int len, int gmax, int waves)
{
    return max(1, min(gmax, (len - seen) / (2 * waves)));
}

// Persistent kernels, one per kernel form (the forms' register budgets differ
// by 2x, so sharing one kernel would halve the occupancy of the sparse form).
// Each wave starts on the queue of its own XCD and then drains the others.
// The window kernel is instantiated with the span form (its LDS is the union
// of both forms' arrays) and with a general power (a second window variant
// with running log-weight maxima) only when some item needs them: each costs
// LDS or registers, hence occupancy.
template <bool kSpan, bool kGeneral>
__global__ __launch_bounds__(64) void k_idw_batch_window(const IdwItem *__restrict__ items,
                                                         const int2 *__restrict__ work,
                                                         const int32_t *__restrict__ qoff,
                                                         const int32_t *__restrict__ qgrab,
                                                         int32_t *__restrict__ qhead, int qwaves,
                                                         int4 *__restrict__ ovf_list, int ovf_cap)
{
    struct WinLds {
        float2 nd[win::kAcc];
        int cnt[win::kAcc];
        float lo[win::kAcc];
        float hi[win::kAcc];
        unsigned long long key[win::kAcc];
        float emax[kGeneral ? win::kAcc : 1];
        int beg[win::kMaxRows];
        int off[win::kMaxRows + 1];
        int4 rec[win::kRecSlots];
    };
    struct NoSpan {
        char pad[16];
    };
    using SpanLds = typename std::conditional<kSpan, span::Smem<win::kTW, win::kTH>, NoSpan>::type;
    // one tile at a time: the span form's LDS and the window form's share
    // the same bytes
    __shared__ union {
        SpanLds sp;
        WinLds w;
    } lds;
    const win::WinSmem sm{lds.w.nd, lds.w.cnt, lds.w.lo, lds.w.hi, lds.w.key, nullptr, nullptr, nullptr,
                          lds.w.emax, lds.w.beg, lds.w.off, lds.w.rec, lds.w.rec + 1, nullptr};
    const int home = blockIdx.x & (kQueues - 1);
    for (int k = 0; k < kQueues; ++k) {
        const int q = (home + k) & (kQueues - 1);
        const int len = qoff[q + 1] - qoff[q], gmax = qgrab[q];
        int seen = 0;
        for (int g = grab_size(seen, len, gmax, qwaves), t0 = pull(qhead, q, len, g); t0 >= 0;
             seen = t0 + g, g = grab_size(seen, len, gmax, qwaves), t0 = pull(qhead, q, len, g)) {
            // the grab's work entries, one per lane, read at once
            const int tn = min(t0 + g, len) - t0;
            const int lane = threadIdx.x & 63;
            int2 wl = make_int2(0, 0);
            if (lane < tn)
                wl = work[qoff[q] + t0 + lane];
            for (int t = 0; t < tn; ++t) {
                // wave-uniform work entry: the item descriptor is then read
                // with scalar loads into SGPRs instead of vector registers
                const int2 w = make_int2(__builtin_amdgcn_readlane(wl.x, t),
                                         __builtin_amdgcn_readlane(wl.y, t));
                const IdwItem &it = items[w.x];
                // integer powers share one variant (the power is a runtime
                // value there); a general power needs the window form's
                // rescaling variant
                if constexpr (kSpan) {
                    if (it.span) {
                        __syncthreads();  // the previous tile is finished with the LDS
                        span::span_tile<3, -1, win::kTW, win::kTH>(it.bv, it.a, it.g, w.y,
                                                                   it.ntx, lds.sp);
                        continue;
                    }
                }
                // nodes above the cap go to the over-cap list (when there is one)
                win::CapSink sk;
                if (ovf_list) {
                    sk.count = qhead + 2 * kQueues;
                    sk.list = ovf_list;
                    sk.cap = ovf_cap;
                    sk.item = w.x;
                }
                if constexpr (kGeneral) {
                    if (it.pmode == 0) {
                        run_window<0, 1>(it, w.y, sm, sk);
                        continue;
                    }
                }
                run_window<-1, 1>(it, w.y, sm, sk);
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_idw_batch_dense(const IdwItem *__restrict__ items,
                                                        const int2 *__restrict__ work,
                                                        const int32_t *__restrict__ qoff,
                                                        const int32_t *__restrict__ qgrab,
                                                        int32_t *__restrict__ qhead, int qwaves)
{
    const int home = blockIdx.x & (kQueues - 1);
    for (int k = 0; k < kQueues; ++k) {
        const int q = (home + k) & (kQueues - 1);
        const int len = qoff[q + 1] - qoff[q], gmax = qgrab[q];
        int seen = 0;
        for (int g = grab_size(seen, len, gmax, qwaves), t0 = pull(qhead, q, len, g); t0 >= 0;
             seen = t0 + g, g = grab_size(seen, len, gmax, qwaves), t0 = pull(qhead, q, len, g)) {
            // the grab's work entries, one per lane, read at once
            const int tn = min(t0 + g, len) - t0;
            const int lane = threadIdx.x & 63;
            int2 wl = make_int2(0, 0);
            if (lane < tn)
                wl = work[qoff[q] + t0 + lane];
            for (int t = 0; t < tn; ++t) {
                // wave-uniform work entry (scalar loads of the descriptor)
                const int2 w = make_int2(__builtin_amdgcn_readlane(wl.x, t),
                                         __builtin_amdgcn_readlane(wl.y, t));
                const IdwItem &it = items[w.x];
                dense::dense_tile<3, kBatchDenseK>(it.bv, it.a, w.y, it.ntx, it.pmode);
            }
        }
    }
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int pmode_of(double p)
{
    if (p == 1.0)
        return 1;
    if (p == 2.0)
        return 2;
    if (p == 3.0)
        return 3;
    return 0;
}

// Expected soundings per disk: input count over the grid grown by r.
double disk_population(const auv_batch_item &it)
{
    const double r = it.params.radius;
    const double area = (it.grid.nx * it.grid.dx + 2 * r) * (it.grid.ny * it.grid.dy + 2 * r);
    return (double)it.n / area * 3.141592653589793 * r * r;
}

struct ClassKey {
    int dens, side;
    bool operator<(const ClassKey &o) const
    {
        return dens != o.dens ? dens < o.dens : side < o.side;
    }
};

ClassKey class_of(const auv_batch_item &it)
{
    ClassKey k;
    k.dens = (int)std::floor(std::log2(disk_population(it) + 1.0));
    k.side = (int)std::lround(std::log2((double)std::max(it.grid.nx, it.grid.ny)));
    return k;
}

bool dense_allowed(const auv_batch_item &it)
{
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < it.n)
        ++bits;
    const double Rd = std::rint(it.params.radius * kLatticePerMetre);
    return it.params.max_pts >= 1 && it.params.max_pts <= 32 &&
           it.params.precision == AUV_P_FP32_REBASE && Rd < 2147483648.0 &&
           dense::dense_key_ok((int32_t)Rd, bits);
}

struct Choice {
    int32_t bin_log2;
    int32_t algo;                // AUV_ALGO_SPARSE or AUV_ALGO_DENSE
    int32_t tile_w = 0, tile_h = 0;  // node tile per wave (0: the form's default)
};

// Default node tile of a form.
Choice with_default_tile(Choice c)
{
    c.tile_w = c.algo == AUV_ALGO_DENSE ? dense::kDT : win::kTW;
    c.tile_h = c.algo == AUV_ALGO_DENSE ? dense::kDT : win::kTH;
    return c;
}

// The other node tiles the autotuner may try for a (bin size, form) choice.
std::vector<Choice> tile_variants(const Choice &c)
{
    std::vector<Choice> v;
    if (c.algo == AUV_ALGO_DENSE) {
        for (int tw : {16, 4}) {
            Choice d = c;
            d.tile_w = tw;
            d.tile_h = 64 / tw;
            v.push_back(d);
        }
    } else {
        Choice d = c;
        d.tile_w = win::kTW;
        d.tile_h = 8;
        v.push_back(d);
    }
    return v;
}

// Candidate (bin size, form) pairs the autotuner may time for an item.
std::vector<Choice> candidates(const auv_batch_item &it, int32_t sR)
{
    std::vector<Choice> c;
    // the sparse form re-does every node over the cap exactly: hopeless once
    // a disk holds several times the cap (timing it there costs seconds)
    const bool sparse_ok = !dense_allowed(it) || disk_population(it) < 4.0 * it.params.max_pts;
    for (int d = -1; d <= 1 && sparse_ok; ++d)
        if (sR + d >= 12 && sR + d <= 26)
            c.push_back({sR + d, AUV_ALGO_SPARSE});
    // dense: bins down to 1/64 of the default side (very dense tiles want bins
    // holding a few soundings, so the ring search stops after a few rings)
    if (dense_allowed(it) && disk_population(it) >= 0.5 * it.params.max_pts)
        for (int d = -6; d <= -1; ++d)
            if (sR + d >= 12)
                c.push_back({sR + d, AUV_ALGO_DENSE});
    return c;
}

}  // namespace

}  // namespace auv

// ------------------------------------------------------------- the batch --

struct auv_batch {
    std::vector<auv_batch_item> items;
    std::vector<auv_grid> grids;
    std::vector<auv::BinGeom> geom;        // batched form
    std::vector<auv::BinGeom> geom_plain;  // plain form
    std::vector<int32_t> algo;             // batched form
    std::vector<auv::Choice> tile;         // batched form: node tile per wave
    std::vector<size_t> slice_off;         // per-item workspace slice
    std::vector<size_t> slice_size;
    std::vector<uint8_t> persistent;       // covered by the persistent kernel
    size_t tables_bytes = 0, ws_bytes = 0;
    // host copies of the device tables (valid for `bound_ws`)
    std::vector<auv::RowItem> rows;
    std::vector<auv::IdwItem> idw;
    std::vector<int32_t> offs;  // hist, scatter, sort offsets, then qoff
    std::vector<int2> work;
    int32_t hist_blocks = 0, scatter_blocks = 0, sort_blocks = 0, nrow_items = 0;
    int32_t nwork_window = 0, nwork_dense = 0;
    int32_t blocks_window = 0, blocks_dense = 0;  // persistent grid sizes
    bool any_span = false, any_general = false;    // window items needing those variants
    int32_t ovf_cap = 0;                           // entries of the over-cap list
    int32_t max_nbx = 0, max_nby = 0;  // largest bin domain of the row-binned items
    double keys_per_row = 0.0;          // largest mean of soundings per bin row
    hipStream_t cap_stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<int32_t> row_items;  // items binned by the batched row path
    // graph
    void *bound_ws = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace auv {

namespace {

auv_status validate_item(const auv_batch_item &it, int i)
{
    const std::string tag = "item " + std::to_string(i) + ": ";
    if (it.n < 0 || it.n >= INT32_MAX)
        return fail(AUV_ERR_INVALID, tag + "n must be in [0, 2^31-1)");
    if (it.n > 0 && (!it.x || !it.y || !it.z))
        return fail(AUV_ERR_INVALID, tag + "null sounding pointer");
    if (!it.z_out)
        return fail(AUV_ERR_INVALID, tag + "z_out is null");
    const auv_idw_params &p = it.params;
    if (!(p.power > 0.0) || !(p.power <= 64.0) || p.min_pts < 0 || p.max_pts < 0)
        return fail(AUV_ERR_INVALID, tag + "bad power / min_pts / max_pts");
    if (p.precision != AUV_P_FP32_REBASE)
        return fail(AUV_ERR_INVALID, tag + "batches run the exact FP64-rebase form only");
    if (p.algo < AUV_ALGO_AUTO || p.algo > AUV_ALGO_SPAN)
        return fail(AUV_ERR_INVALID, tag + "unknown algo");
    return AUV_OK;
}

// Build the bin view and IDW arguments of item i with its workspace slice.
void item_views(const auv_batch *b, int i, char *ws, const BinGeom &geom, int32_t algo,
                BinWorkspace *w, auv_bin_view *bv, IdwArgs *a, Choice tile = Choice{0, 0})
{
    const auv_batch_item &it = b->items[i];
    bin_workspace_layout(it.n, geom, ws + b->slice_off[i], w);
    auv_bin_view v{};
    v.cell_start = w->cell_start;
    v.X = w->X;
    v.Y = w->Y;
    v.res = w->res;
    v.z = w->z;
    v.idx = w->idx;
    v.rec = w->rec;
    v.nbx = geom.nbx;
    v.nby = geom.nby;
    v.halo = geom.halo;
    v.bin_log2 = geom.s;
    v.R = geom.R;
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < it.n)
        ++bits;
    v.idx_bits = bits;
    *bv = v;
    IdwArgs x;
    std::memset(&x, 0, sizeof(x));
    x.dx = it.grid.dx;
    x.dy = it.grid.dy;
    x.nx = it.grid.nx;
    x.ny = it.grid.ny;
    x.R = geom.R;
    x.R_stage = geom.R;
    x.inv_r2 = (float)(1.0 / ((double)geom.R * geom.R));
    x.r2f = (float)(it.params.radius * it.params.radius);
    x.x0 = it.grid.x0;
    x.y0 = it.grid.y0;
    x.power = (float)it.params.power;
    x.min_pts = it.params.min_pts;
    x.max_pts = it.params.max_pts;
    x.precision = AUV_P_FP32_REBASE;
    x.mode = (it.nn_idx_out || it.nn_z_out) ? 3 : 1;
    x.z_out = it.z_out;
    x.cnt_out = it.cnt_out;
    x.nn_idx_out = it.nn_idx_out;
    x.nn_z_out = it.nn_z_out;
    x.dense = algo == AUV_ALGO_DENSE;
    x.span = algo == AUV_ALGO_SPAN;
    x.pmode = pmode_of(it.params.power);
    x.tile_w = tile.tile_w;
    x.tile_h = tile.tile_h;
    *a = x;
}

int32_t auto_algo(const auv_batch_item &it)
{
    if (it.params.algo != AUV_ALGO_AUTO)
        return it.params.algo;
    return dense_allowed(it) && disk_population(it) >= 0.5 * it.params.max_pts ? AUV_ALGO_DENSE
                                                                          : AUV_ALGO_SPARSE;
}

std::map<ClassKey, Choice> read_tune(const char *path)
{
    std::map<ClassKey, Choice> t;
    if (!path)
        return t;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string tag, k1, k2;
        ClassKey key;
        Choice c;
        double ms;
        if (is >> tag >> key.dens >> key.side >> k1 >> c.bin_log2 >> k2 >> c.algo && tag == "class") {
            std::string k3;
            int tw = 0, th = 0;
            if (is >> k3 && k3 == "tile" && is >> tw >> th) {
                c.tile_w = tw;
                c.tile_h = th;
            }
            t[key] = c;
        }
        (void)ms;
    }
    return t;
}

// The persistent kernels' descriptor of one item; false when they do not
// cover it (window over 64 cells, key over 64 bits, cap above the dense limit).
bool make_idw_item(const auv_batch_item &it, const auv_bin_view &bv, const IdwArgs &a,
                   int32_t algo, IdwItem *out)
{
    IdwItem d{};
    d.bv = bv;
    d.a = a;
    d.pmode = pmode_of(it.params.power);
    d.dense = algo == AUV_ALGO_DENSE;
    d.span = 0;
    bool ok = true;
    if (d.dense) {
        ok = it.params.max_pts >= 1 && it.params.max_pts <= kBatchDenseK &&
             dense::dense_key_ok(a.R, bv.idx_bits);
        const int tw = dense::dense_tile_w(a), th = 64 / tw;
        d.ntx = (it.grid.nx + tw - 1) / tw;
        d.ntiles = d.ntx * ((it.grid.ny + th - 1) / th);
    } else {
        ok = window_geometry(a, &d.g) && d.g.nchunks == 1;
        const unsigned __int128 top = (unsigned __int128)((unsigned long long)a.R * a.R)
                                      << bv.idx_bits;
        ok = ok && top < ((unsigned __int128)1 << 64);
        d.span = ok && a.span && span::span_ok(bv, a, d.g, d.pmode) ? 1 : 0;
        d.cap_list = ok && !d.span && it.params.max_pts >= 1 &&
                             it.params.max_pts <= kBatchDenseK &&
                             dense::dense_key_ok(a.R, bv.idx_bits)
                         ? 1
                         : 0;
        const int th = win::tile_rows(a);
        d.ntx = (it.grid.nx + win::kTW - 1) / win::kTW;
        d.ntiles = d.ntx * ((it.grid.ny + th - 1) / th);
    }
    *out = d;
    return ok;
}

// Build the device tables for workspace `ws` (host copies kept in the batch).
auv_status build_tables(auv_batch *b, char *ws)
{
    const int count = (int)b->items.size();
    b->rows.assign(count, RowItem{});
    b->max_nbx = b->max_nby = 0;
    b->keys_per_row = 0.0;
    b->idw.assign(count, IdwItem{});
    b->row_items.clear();
    std::vector<int32_t> hist(1, 0), scat(1, 0), sort(1, 0);
    std::vector<double> cost(count, 0.0), tile_cost(count, 0.0);
    for (int i = 0; i < count; ++i) {
        const auv_batch_item &it = b->items[i];
        BinWorkspace w;
        auv_bin_view bv;
        IdwArgs a;
        item_views(b, i, ws, b->geom[i], b->algo[i], &w, &bv, &a, b->tile[i]);
        if (row_path_ok(b->geom[i])) {
            b->rows[b->row_items.size()] =
                make_row_item(&b->grids[i], b->geom[i], it.x, it.y, it.z, it.n, w);
            b->row_items.push_back(i);
            hist.push_back(hist.back() + row_hist_blocks(it.n));
            scat.push_back(scat.back() + row_scatter_blocks(it.n));
            sort.push_back(sort.back() + b->geom[i].nby);
            b->max_nbx = std::max(b->max_nbx, b->geom[i].nbx);
            b->max_nby = std::max(b->max_nby, b->geom[i].nby);
            b->keys_per_row =
                std::max(b->keys_per_row, (double)it.n / std::max(1, b->geom[i].nby));
        }
        IdwItem &d = b->idw[i];
        const bool ok = make_idw_item(it, bv, a, b->algo[i], &d) && row_path_ok(b->geom[i]);
        b->persistent[i] = ok ? 1 : 0;
        if (d.dense) {
            cost[i] = (double)it.n + (double)it.grid.nx * it.grid.ny * 4.0;
            tile_cost[i] = cost[i] / std::max(1, d.ntiles);
        } else {
            // a window tile costs a fixed part plus one visit per sounding
            // within reach of its box (uniform density over the grid grown
            // by the radius)
            const double r = it.params.radius;
            const double rho = (double)it.n / ((it.grid.nx * it.grid.dx + 2.0 * r) *
                                               (it.grid.ny * it.grid.dy + 2.0 * r));
            const double bw = win::kTW * it.grid.dx + 2.0 * r;
            const double bh = win::tile_rows(a) * it.grid.dy + 2.0 * r;
            tile_cost[i] = 20.0 + rho * bw * bh;
            cost[i] = tile_cost[i] * std::max(1, d.ntiles);
        }
    }
    b->nrow_items = (int32_t)b->row_items.size();
    b->hist_blocks = hist.back();
    b->scatter_blocks = scat.back();
    b->sort_blocks = sort.back();
    // longest processing time first: items to the least loaded queue, one
    // queue set per kernel form
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i)
        order[i] = i;
    // items with the longest tiles first (a wave takes a tile alone, so a
    // long tile late in a queue would end the kernel late); to the least
    // loaded queue by total cost
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        return tile_cost[x] != tile_cost[y] ? tile_cost[x] > tile_cost[y] : cost[x] > cost[y];
    });
    b->work.clear();
    std::vector<int32_t> qoff(2 * kQueues + 1, 0);
    for (int form = 0; form < 2; ++form) {
        std::vector<std::vector<int>> q(kQueues);
        std::vector<double> load(kQueues, 0.0);
        for (int i : order) {
            if (!b->persistent[i] || b->idw[i].dense != form)
                continue;
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            q[k].push_back(i);
            load[k] += cost[i];
        }
        for (int k = 0; k < kQueues; ++k) {
            for (int i : q[k])
                for (int t = 0; t < b->idw[i].ntiles; ++t)
                    b->work.push_back(make_int2(i, t));
            qoff[form * kQueues + k + 1] = (int32_t)b->work.size();
        }
    }
    b->nwork_window = qoff[kQueues];
    b->nwork_dense = qoff[2 * kQueues] - qoff[kQueues];
    // tiles per grab: about 8 grabs per wave from its home queue
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // waves per CU of the two concurrent persistent kernels: the window
    // kernel could hold 15 (its LDS, about 10.6 KB per wave) and the dense
    // kernel 24 (80 registers), but they share the CUs.  Measured on the
    // 256-tile batch: window 12 + dense 8 per CU 2.15 ms; window 16 + dense
    // 8 2.33 ms, 10 + 8 2.16 ms, 8 + 8 2.27 ms; 16 + 12 2.43 ms, 16 + 6
    // 2.33 ms, 16 + 4 2.67 ms.
    b->blocks_window = std::max(1, std::min(b->nwork_window, cus * 12));
    b->blocks_dense = std::max(1, std::min(b->nwork_dense, cus * 8));
    b->any_span = b->any_general = false;
    for (int i = 0; i < count; ++i) {
        if (!b->persistent[i] || b->idw[i].dense)
            continue;
        b->any_span = b->any_span || b->idw[i].span;
        b->any_general = b->any_general || b->idw[i].pmode == 0;
    }
    std::vector<int32_t> grab(2 * kQueues, 1);
    for (int form = 0; form < 2; ++form) {
        const int per_queue = std::max(1, (form ? b->blocks_dense : b->blocks_window) / kQueues);
        for (int k = 0; k < kQueues; ++k) {
            const int len = qoff[form * kQueues + k + 1] - qoff[form * kQueues + k];
            grab[form * kQueues + k] = std::max(1, std::min(16, len / (8 * per_queue)));
        }
    }
    b->offs.clear();
    b->offs.insert(b->offs.end(), hist.begin(), hist.end());
    b->offs.insert(b->offs.end(), scat.begin(), scat.end());
    b->offs.insert(b->offs.end(), sort.begin(), sort.end());
    b->offs.insert(b->offs.end(), qoff.begin(), qoff.end());
    b->offs.insert(b->offs.end(), grab.begin(), grab.end());
    return AUV_OK;
}

// Table region at the start of the workspace.
struct Tables {
    RowItem *rows;
    IdwItem *idw;
    int32_t *offs;
    int32_t *qhead;
    int4 *ovf;  // over-cap list
    int2 *work;
};

Tables table_ptrs(const auv_batch *b, char *ws)
{
    const size_t count = b->items.size();
    size_t off = 0;
    Tables t;
    t.rows = reinterpret_cast<RowItem *>(ws + off);
    off += align256(sizeof(RowItem) * count);
    t.idw = reinterpret_cast<IdwItem *>(ws + off);
    off += align256(sizeof(IdwItem) * count);
    t.offs = reinterpret_cast<int32_t *>(ws + off);
    off += align256(sizeof(int32_t) * (3 * (count + 1) + 4 * kQueues + 1));
    t.qhead = reinterpret_cast<int32_t *>(ws + off);
    off += align256(sizeof(int32_t) * (2 * kQueues + 1));
    t.ovf = reinterpret_cast<int4 *>(ws + off);
    off += align256(sizeof(int4) * (size_t)b->ovf_cap);
    t.work = reinterpret_cast<int2 *>(ws + off);
    return t;
}

size_t tables_size(size_t count, size_t max_tiles, size_t ovf_cap)
{
    return align256(sizeof(RowItem) * count) + align256(sizeof(IdwItem) * count) +
           align256(sizeof(int32_t) * (3 * (count + 1) + 4 * kQueues + 1)) +
           align256(sizeof(int32_t) * (2 * kQueues + 1)) + align256(sizeof(int4) * ovf_cap) +
           align256(sizeof(int2) * std::max<size_t>(max_tiles, 1));
}

void launch_batch_window(int blocks, bool any_span, bool any_general, const IdwItem *idw,
                         const int2 *work, const int32_t *qoff, const int32_t *qgrab,
                         int32_t *qhead, int4 *ovf_list, int ovf_cap, hipStream_t st)
{
    const int qw = std::max(1, blocks / kQueues);
    const unsigned nb = (unsigned)blocks;
    if (any_span && any_general)
        k_idw_batch_window<true, true><<<nb, 64, 0, st>>>(idw, work, qoff, qgrab, qhead, qw,
                                                           ovf_list, ovf_cap);
    else if (any_span)
        k_idw_batch_window<true, false><<<nb, 64, 0, st>>>(idw, work, qoff, qgrab, qhead, qw,
                                                            ovf_list, ovf_cap);
    else if (any_general)
        k_idw_batch_window<false, true><<<nb, 64, 0, st>>>(idw, work, qoff, qgrab, qhead, qw,
                                                            ovf_list, ovf_cap);
    else
        k_idw_batch_window<false, false><<<nb, 64, 0, st>>>(idw, work, qoff, qgrab, qhead, qw,
                                                             ovf_list, ovf_cap);
}

// Enqueue the whole batched form on `st` (captured by the caller).
auv_status enqueue_batched(auv_batch *b, char *ws, hipStream_t st)
{
    const Tables t = table_ptrs(b, ws);
    const int count = (int)b->items.size();
    const int nr = b->nrow_items;
    AUV_TRY_S(launch_binning_batch(t.rows, t.offs, t.offs + (nr + 1), t.offs + 2 * (nr + 1), nr,
                                   b->hist_blocks, b->scatter_blocks, b->sort_blocks,
                                   b->max_nbx, b->max_nby, b->keys_per_row, st));
    for (int i = 0; i < count; ++i) {
        if (row_path_ok(b->geom[i]))
            continue;
        BinWorkspace w;
        auv_bin_view bv;
        IdwArgs a;
        item_views(b, i, ws, b->geom[i], b->algo[i], &w, &bv, &a, b->tile[i]);
        const auv_batch_item &it = b->items[i];
        AUV_TRY_S(launch_binning(&b->grids[i], b->geom[i], it.x, it.y, it.z, it.n, w, st));
    }
    if (!b->work.empty()) {
        k_reset_queues<<<1, 64, 0, st>>>(t.qhead);
        const int32_t *qoff = t.offs + 3 * (nr + 1);
        const int32_t *qgrab = qoff + 2 * kQueues + 1;
        // the dense form runs on a forked branch of the graph, concurrently
        if (b->nwork_dense > 0) {
            AUV_HIP(hipEventRecord(b->ev_fork, st));
            AUV_HIP(hipStreamWaitEvent(b->cap_stream2, b->ev_fork, 0));
            k_idw_batch_dense<<<b->blocks_dense, 64, 0, b->cap_stream2>>>(
                t.idw, t.work, qoff + kQueues, qgrab + kQueues, t.qhead + kQueues,
                std::max(1, b->blocks_dense / kQueues));
            AUV_HIP(hipGetLastError());
            AUV_HIP(hipEventRecord(b->ev_join, b->cap_stream2));
        }
        if (b->nwork_window > 0)
            launch_batch_window(b->blocks_window, b->any_span, b->any_general, t.idw, t.work,
                                qoff, qgrab, t.qhead, b->ovf_cap > 0 ? t.ovf : nullptr,
                                b->ovf_cap, st);
        AUV_HIP(hipGetLastError());
        if (b->nwork_dense > 0)
            AUV_HIP(hipStreamWaitEvent(st, b->ev_join, 0));
        if (b->nwork_window > 0 && b->ovf_cap > 0) {
            int dev = 0, cus = 256;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            k_overcap_dense<<<cus * 4, 64, 0, st>>>(t.idw, t.ovf, t.qhead + 2 * kQueues,
                                                    b->ovf_cap);
            AUV_HIP(hipGetLastError());
        }
    }
    for (int i = 0; i < count; ++i) {
        if (b->persistent[i])
            continue;
        AUV_TRY_S(launch_idw(b->idw[i].bv, b->idw[i].a, st));
    }
    return AUV_OK;
}

}  // namespace
}  // namespace auv

using namespace auv;

extern "C" {

auv_status auv_batch_plan(const auv_batch_item *items, int32_t count, const char *tune_path,
                          auv_batch **out)
{
    if (!out)
        return fail(AUV_ERR_INVALID, "out is null");
    *out = nullptr;
    if (!items || count < 1)
        return fail(AUV_ERR_INVALID, "need at least one item");
    auv_batch *b = new (std::nothrow) auv_batch;
    if (!b)
        return fail(AUV_ERR_INVALID, "out of host memory");
    b->items.assign(items, items + count);
    b->grids.resize(count);
    b->geom.resize(count);
    b->geom_plain.resize(count);
    b->algo.resize(count);
    b->tile.resize(count);
    b->slice_off.resize(count);
    b->slice_size.resize(count);
    b->persistent.assign(count, 0);
    const std::map<ClassKey, Choice> tune = read_tune(tune_path);
    size_t off = 0, max_tiles = 0, ovf_nodes = 0;
    for (int i = 0; i < count; ++i) {
        const auv_batch_item &it = b->items[i];
        auv_status st = validate_item(it, i);
        if (st == AUV_OK) {
            auv_grid *g = nullptr;
            st = auv_grid_create(&it.grid, &g);
            if (st == AUV_OK) {
                b->grids[i] = *g;
                auv_grid_destroy(g);
            }
        }
        if (st == AUV_OK)
            st = bin_geometry(&b->grids[i], it.params.radius, 0, &b->geom_plain[i]);
        if (st != AUV_OK) {
            delete b;
            return st;
        }
        Choice c{b->geom_plain[i].s, auto_algo(it)};
        const auto f = tune.find(class_of(it));
        if (f != tune.end() && it.params.algo == AUV_ALGO_AUTO &&
            (f->second.algo == AUV_ALGO_SPARSE || dense_allowed(it)))
            c = f->second;
        b->algo[i] = c.algo;
        b->tile[i] = c.tile_w > 0 ? c : with_default_tile(c);
        st = bin_geometry(&b->grids[i], it.params.radius, c.bin_log2, &b->geom[i]);
        if (st != AUV_OK) {
            b->geom[i] = b->geom_plain[i];
            b->algo[i] = auto_algo(it);
            b->tile[i] = with_default_tile(Choice{0, b->algo[i]});
        }
        // slice: the largest layout any form or autotune candidate may use
        size_t need = std::max(bin_workspace_layout(it.n, b->geom[i], nullptr, nullptr),
                               bin_workspace_layout(it.n, b->geom_plain[i], nullptr, nullptr));
        for (const Choice &cc : candidates(it, b->geom_plain[i].s)) {
            BinGeom gg;
            if (bin_geometry(&b->grids[i], it.params.radius, cc.bin_log2, &gg) == AUV_OK &&
                (int64_t)gg.nbx * gg.nby <= (int64_t)1 << 24)
                need = std::max(need, bin_workspace_layout(it.n, gg, nullptr, nullptr));
        }
        b->slice_size[i] = align256(need);
        const size_t tiles8 = (size_t)((it.grid.nx + 7) / 8) * ((it.grid.ny + 7) / 8);
        max_tiles += tiles8;
        // over-cap list: room for every node of the capped window items, up
        // to a bound (nodes beyond it are re-done inside their tiles)
        if (b->algo[i] != AUV_ALGO_DENSE && it.params.max_pts >= 1 &&
            it.params.max_pts <= kBatchDenseK)
            ovf_nodes += (size_t)it.grid.nx * (size_t)it.grid.ny;
    }
    b->ovf_cap = (int32_t)std::min<size_t>(ovf_nodes, kOvfMax);
    b->tables_bytes = align256(tables_size(count, max_tiles, (size_t)b->ovf_cap));
    off = b->tables_bytes;
    for (int i = 0; i < count; ++i) {
        b->slice_off[i] = off;
        off += b->slice_size[i];
    }
    b->ws_bytes = off;
    *out = b;
    return AUV_OK;
}

auv_status auv_batch_workspace_size(const auv_batch *batch, size_t *bytes)
{
    if (!batch || !bytes)
        return fail(AUV_ERR_INVALID, "null argument");
    *bytes = batch->ws_bytes;
    return AUV_OK;
}

auv_status auv_batch_item_plan(const auv_batch *batch, int32_t item, int32_t *bin_log2,
                               int32_t *algo, int32_t *tile_w, int32_t *tile_h)
{
    if (!batch || item < 0 || item >= (int32_t)batch->items.size())
        return fail(AUV_ERR_INVALID, "bad batch or item");
    if (bin_log2)
        *bin_log2 = batch->geom[item].s;
    if (algo)
        *algo = batch->algo[item];
    if (tile_w)
        *tile_w = batch->tile[item].tile_w;
    if (tile_h)
        *tile_h = batch->tile[item].tile_h;
    return AUV_OK;
}

static auv_status check_ws(const auv_batch *b, void *ws, size_t ws_bytes)
{
    if (!b)
        return fail(AUV_ERR_INVALID, "batch is null");
    if (!ws || ws_bytes < b->ws_bytes)
        return fail(AUV_ERR_BUDGET, "workspace smaller than auv_batch_workspace_size");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(AUV_ERR_INVALID, "workspace must be 256-byte aligned");
    return AUV_OK;
}

auv_status auv_batch_launch(auv_batch *b, void *ws, size_t ws_bytes, auv_stream stream)
{
    AUV_TRY_S(check_ws(b, ws, ws_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    if (b->exec && b->bound_ws == ws) {
        AUV_HIP(hipGraphLaunch(b->exec, st));
        return AUV_OK;
    }
    // (re)bind: tables for this workspace, then capture
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    AUV_TRY_S(build_tables(b, base));
    const Tables t = table_ptrs(b, base);
    AUV_HIP(hipMemcpyAsync(t.rows, b->rows.data(), sizeof(RowItem) * b->rows.size(),
                           hipMemcpyHostToDevice, st));
    AUV_HIP(hipMemcpyAsync(t.idw, b->idw.data(), sizeof(IdwItem) * b->idw.size(),
                           hipMemcpyHostToDevice, st));
    AUV_HIP(hipMemcpyAsync(t.offs, b->offs.data(), sizeof(int32_t) * b->offs.size(),
                           hipMemcpyHostToDevice, st));
    if (!b->work.empty())
        AUV_HIP(hipMemcpyAsync(t.work, b->work.data(), sizeof(int2) * b->work.size(),
                               hipMemcpyHostToDevice, st));
    // the tables must be in place before any replay reads them
    AUV_HIP(hipStreamSynchronize(st));
    if (!b->cap_stream) {
        AUV_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        AUV_HIP(hipStreamCreateWithFlags(&b->cap_stream2, hipStreamNonBlocking));
        AUV_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        AUV_HIP(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    }
    AUV_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const auv_status es = enqueue_batched(b, base, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
    if (es != AUV_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return es;
    }
    if (ce != hipSuccess)
        return hip_fail(ce, "hipStreamEndCapture");
    b->graph = g;
    AUV_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->bound_ws = ws;
    AUV_HIP(hipGraphLaunch(b->exec, st));
    return AUV_OK;
}

auv_status auv_batch_launch_plain(auv_batch *b, void *ws, size_t ws_bytes, auv_stream stream)
{
    AUV_TRY_S(check_ws(b, ws, ws_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    for (int i = 0; i < (int)b->items.size(); ++i) {
        const auv_batch_item &it = b->items[i];
        BinWorkspace w;
        auv_bin_view bv;
        IdwArgs a;
        item_views(b, i, base, b->geom_plain[i], auto_algo(it), &w, &bv, &a);
        AUV_TRY_S(launch_binning(&b->grids[i], b->geom_plain[i], it.x, it.y, it.z, it.n, w, st));
        AUV_TRY_S(launch_idw(bv, a, st));
    }
    return AUV_OK;
}

auv_status auv_batch_autotune(const auv_batch_item *items, int32_t count, void *ws,
                              size_t ws_bytes, auv_stream stream, const char *tune_path)
{
    if (!tune_path)
        return fail(AUV_ERR_INVALID, "tune_path is null");
    auv_batch *b = nullptr;
    AUV_TRY_S(auv_batch_plan(items, count, nullptr, &b));
    struct Guard {
        auv_batch *b;
        ~Guard() { auv_batch_destroy(b); }
    } guard{b};
    AUV_TRY_S(check_ws(b, ws, ws_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    // one representative per class: the item with the most soundings
    std::map<ClassKey, int> rep;
    for (int i = 0; i < count; ++i) {
        const ClassKey k = class_of(b->items[i]);
        const auto f = rep.find(k);
        if (f == rep.end() || b->items[i].n > b->items[f->second].n)
            rep[k] = i;
    }
    hipEvent_t e0, e1;
    AUV_HIP(hipEventCreate(&e0));
    AUV_HIP(hipEventCreate(&e1));
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the tables region of the workspace holds the throughput runs' work list
    size_t work_cap = 0;
    for (int k = 0; k < count; ++k)
        work_cap += (size_t)((b->items[k].grid.nx + 7) / 8) * ((b->items[k].grid.ny + 7) / 8);
    std::ostringstream table;
    table << "# auvgrid autotune table: class <log2 disk population> <log2 grid side> "
             "bin_log2 <s> algo <1 sparse | 2 dense> tile <nodes across> <nodes down> "
             "ms <time>\n";
    auv_status result = AUV_OK;
    for (const auto &kv : rep) {
        const int i = kv.second;
        const auv_batch_item &it = b->items[i];
        Choice best = with_default_tile(Choice{b->geom_plain[i].s, auto_algo(it)});
        float best_ms = 1e30f;
        // min of three timed runs (after one untimed) of binning + IDW
        // Time of a candidate in the setting it will run in: binning the item
        // (min of three runs after one untimed), plus the persistent kernel of
        // its form over enough repetitions of the item's tiles to fill the
        // chip (all reading the same bins), per repetition; items the
        // persistent kernels do not cover get their own IDW launch instead.
        auto time_choice = [&](const Choice &c, float *out_ms) -> auv_status {
            *out_ms = 1e30f;
            BinGeom gg;
            if (bin_geometry(&b->grids[i], it.params.radius, c.bin_log2, &gg) != AUV_OK ||
                (int64_t)gg.nbx * gg.nby > (int64_t)1 << 24 ||
                bin_workspace_layout(it.n, gg, nullptr, nullptr) > b->slice_size[i])
                return AUV_OK;
            BinWorkspace w;
            auv_bin_view bv;
            IdwArgs a;
            item_views(b, i, base, gg, c.algo, &w, &bv, &a, c);
            auto min_of_runs = [&](auto &&enqueue, float *best) -> auv_status {
                *best = 1e30f;
                for (int rep_i = 0; rep_i < 4; ++rep_i) {
                    AUV_HIP(hipEventRecord(e0, st));
                    AUV_TRY_S(enqueue());
                    AUV_HIP(hipEventRecord(e1, st));
                    AUV_HIP(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    AUV_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (rep_i > 0)
                        *best = std::min(*best, ms);
                }
                return AUV_OK;
            };
            float bin_ms, idw_ms;
            AUV_TRY_S(min_of_runs(
                [&] { return launch_binning(&b->grids[i], gg, it.x, it.y, it.z, it.n, w, st); },
                &bin_ms));
            IdwItem d;
            if (!make_idw_item(it, bv, a, c.algo, &d) || !row_path_ok(gg) || d.ntiles < 1) {
                AUV_TRY_S(min_of_runs([&] { return launch_idw(bv, a, st); }, &idw_ms));
                *out_ms = bin_ms + idw_ms;
                return AUV_OK;
            }
            const int64_t target = (int64_t)cus * 16 * 8;  // tiles: ~8 per resident wave
            const int copies = (int)std::max<int64_t>(
                1, std::min<int64_t>((target + d.ntiles - 1) / d.ntiles,
                                     (int64_t)work_cap / d.ntiles));
            const int nwork = copies * d.ntiles;
            std::vector<int2> work(nwork);
            for (int t = 0; t < nwork; ++t)
                work[t] = make_int2(0, t % d.ntiles);
            const int blocks = std::max(1, std::min(nwork, cus * (d.dense ? 8 : 16)));
            const int per_queue = std::max(1, blocks / kQueues);
            std::vector<int32_t> offs(2 * kQueues + 1);
            for (int k = 0; k <= kQueues; ++k)
                offs[k] = (int32_t)((int64_t)nwork * k / kQueues);
            for (int k = 0; k < kQueues; ++k)
                offs[kQueues + 1 + k] =
                    std::max(1, std::min(16, (offs[k + 1] - offs[k]) / (8 * per_queue)));
            const Tables t = table_ptrs(b, base);
            AUV_HIP(hipMemcpyAsync(t.idw, &d, sizeof(d), hipMemcpyHostToDevice, st));
            AUV_HIP(hipMemcpyAsync(t.work, work.data(), sizeof(int2) * nwork,
                                   hipMemcpyHostToDevice, st));
            AUV_HIP(hipMemcpyAsync(t.offs, offs.data(), sizeof(int32_t) * offs.size(),
                                   hipMemcpyHostToDevice, st));
            AUV_TRY_S(min_of_runs(
                [&]() -> auv_status {
                    k_reset_queues<<<1, 64, 0, st>>>(t.qhead);
                    if (d.dense)
                        k_idw_batch_dense<<<blocks, 64, 0, st>>>(t.idw, t.work, t.offs,
                                                                 t.offs + kQueues + 1, t.qhead,
                                                                 per_queue);
                    else
                        launch_batch_window(blocks, d.span != 0, d.pmode == 0, t.idw, t.work,
                                            t.offs, t.offs + kQueues + 1, t.qhead, nullptr, 0,
                                            st);
                    AUV_HIP(hipGetLastError());
                    return AUV_OK;
                },
                &idw_ms));
            *out_ms = bin_ms + idw_ms / (float)copies;
            return AUV_OK;
        };
        // bin size and form at the form's default tile, then the other node
        // tiles of the winner
        for (const Choice &c0 : candidates(it, b->geom_plain[i].s)) {
            const Choice c = with_default_tile(c0);
            float ms;
            result = time_choice(c, &ms);
            if (result != AUV_OK)
                break;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        if (result == AUV_OK && best_ms < 1e30f) {
            for (const Choice &c : tile_variants(best)) {
                float ms;
                result = time_choice(c, &ms);
                if (result != AUV_OK)
                    break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
        if (result != AUV_OK)
            break;
        table << "class " << kv.first.dens << " " << kv.first.side << " bin_log2 "
              << best.bin_log2 << " algo " << best.algo << " tile " << best.tile_w << " "
              << best.tile_h << " ms " << best_ms << "\n";
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != AUV_OK)
        return result;
    std::ofstream f(tune_path);
    if (!f)
        return fail(AUV_ERR_INVALID, std::string("cannot write ") + tune_path);
    f << table.str();
    return AUV_OK;
}

void auv_batch_destroy(auv_batch *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    if (b->cap_stream2)
        (void)hipStreamDestroy(b->cap_stream2);
    if (b->ev_fork)
        (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join)
        (void)hipEventDestroy(b->ev_join);
    delete b;
}

}  // extern "C"
