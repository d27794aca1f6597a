// Serving: per-vehicle resident IDW sums, updated by streams of requests.
//
// One launch (one request in FIFO mode, up to max_batch requests of distinct
// vehicles in batched mode) enqueues on the session stream:
//   k_serve_stage       reads the launch table and each request's slot
//                       (bounding-box seed + x, y, z) from pinned host memory
//                       and writes them to the device (no runtime copy: the
//                       copy path of the runtime stalled now and then)
//   batched row binning (the kernels behind auv_bin_points); its histogram
//                       kernel also widens each request's lattice bounding
//                       box over the binned soundings
//   k_serve_update<c>   persistent: (request, node tile) work over the tiles
//                       within the radius of each request's bounding box;
//                       the window-form gather accumulates the tile in LDS
//                       (16 waves per tile, combined in fixed order), then
//                       each node's resident sums get one read-modify-write
//   an event, which the worker thread observes to complete the tickets.
// A vehicle has at most one request per launch and launches run in stream
// order, so a vehicle's sums see its requests in submission order and no two
// waves update one node at the same time.
#include "idw_window_impl.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace auv {
namespace {

constexpr int kMaxBatchReq = 64;
constexpr size_t kSlotHeader = 256;

struct ServeItem {
    auv_bin_view bv;
    IdwArgs a;
    WinGeom g;
    int32_t ntx;
    const int32_t *bbox;  // X min, Y min, X max, Y max (lattice units, binned soundings)
};

__device__ inline long long floor_div(long long a, long long b)
{
    const long long q = a / b;
    return (a % b != 0 && (a < 0) != (b < 0)) ? q - 1 : q;
}

// Persistent update over (request, tile) work, one tile per block of
// kServeParts waves.  A request's soundings are dense, so one wave per tile
// would run hundreds of window visits in series: the waves of the block take
// interleaved chunks of the tile's candidates into their own LDS sums, which
// are then combined in wave order (so the result does not depend on timing)
// and added to the resident sums with one read-modify-write per node.  Lane i
// of every wave holds request i's tile rectangle (count <= 64); a wave-wide
// prefix turns the pulled work index into (request, tile).  A request
// covers few tiles (about 85 for 26k soundings), far fewer than the chip has
// SIMDs, so a tile's latency is the request's: 16 waves per tile (96 KB of
// LDS, one block per CU) measured p50 0.16 ms against 0.21 ms with 4.
constexpr int kServeParts = 16;
static_assert(win::kNodes <= 64 * kServeParts, "at most one node per thread when combining");

template <int kChunks>
__global__ __launch_bounds__(64 * kServeParts) void k_serve_update(
    const ServeItem *__restrict__ items, int count, int32_t *__restrict__ counter)
{
    __shared__ float2 s_nd[kServeParts][win::kAcc];
    __shared__ int s_cnt[kServeParts][win::kAcc];
    __shared__ float s_lo[kServeParts][win::kAcc];
    __shared__ float s_hi[kServeParts][win::kAcc];
    __shared__ float s_emax[1];
    __shared__ int s_beg[kServeParts][win::kMaxRows];
    __shared__ int s_off[kServeParts][win::kMaxRows + 1];
    __shared__ int4 s_rec[kServeParts][win::kRecSlots];
    __shared__ float s_zref[kServeParts];
    __shared__ int s_task;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const win::WinSmem sm{s_nd[wave], s_cnt[wave], s_lo[wave], s_hi[wave], nullptr, nullptr, nullptr,
                          nullptr, s_emax, s_beg[wave], s_off[wave], s_rec[wave],
                          s_rec[wave] + 1, nullptr};
    int t0x = 0, t0y = 0, tcols = 1, nt = 0;
    if (lane < count) {
        const ServeItem &it = items[lane];
        const int4 bb = *reinterpret_cast<const int4 *>(it.bbox);
        if (it.g.nchunks == kChunks && bb.x <= bb.z && bb.y <= bb.w) {
            // nodes with a lattice coordinate within R of the box
            const long long R = it.a.R;
            const long long b0 = max(0ll, -floor_div(-((long long)bb.x - R - it.g.X0), it.g.DXl));
            const long long b1 = min((long long)it.a.nx - 1,
                                     floor_div((long long)bb.z + R - it.g.X0, it.g.DXl));
            const long long a0 = max(0ll, -floor_div(-((long long)bb.y - R - it.g.Y0), it.g.DYl));
            const long long a1 = min((long long)it.a.ny - 1,
                                     floor_div((long long)bb.w + R - it.g.Y0, it.g.DYl));
            if (b0 <= b1 && a0 <= a1) {
                t0x = (int)(b0 / win::kTW);
                t0y = (int)(a0 / win::kTH);
                tcols = (int)(b1 / win::kTW) - t0x + 1;
                nt = tcols * ((int)(a1 / win::kTH) - t0y + 1);
            }
        }
    }
    int incl = nt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += u;
    }
    const int total = __shfl(incl, 63, 64);
    const int excl = incl - nt;
    for (;;) {
        if (threadIdx.x == 0)
            s_task = atomicAdd(counter, 1);
        __syncthreads();
        const int t = s_task;
        __syncthreads();  // every wave has its task before s_task is rewritten
        if (t >= total)
            break;
        const int i = __ffsll((long long)__ballot(incl > t)) - 1;
        const int loc = t - __builtin_amdgcn_readlane(excl, i);
        const int c = __builtin_amdgcn_readlane(tcols, i);
        const int tx = __builtin_amdgcn_readlane(t0x, i) + loc % c;
        const int ty = __builtin_amdgcn_readlane(t0y, i) + loc / c;
        const ServeItem &it = items[i];
        float zr = 0.0f;
        win::window_tile<5, -1, true, kChunks, AUV_P_FP32_REBASE>(
            it.bv, it.a, it.g, ty * it.ntx + tx, it.ntx, sm, wave, kServeParts, &zr);
        if (lane == 0)
            s_zref[wave] = zr;
        __syncthreads();
        // combine the parts in wave order: one node per thread
        const int tb0 = tx * win::kTW, ta0 = ty * win::kTH;
        const int la = threadIdx.x / win::kTW, lb = threadIdx.x - la * win::kTW;
        const int q = la * win::kRS + lb;
        if (la < min(win::kTH, it.a.ny - ta0) && lb < min(win::kTW, it.a.nx - tb0)) {
            double num = 0.0;
            float den = 0.0f, lo = INFINITY, hi = -INFINITY;
            int cnt = 0;
#pragma unroll
            for (int w = 0; w < kServeParts; ++w) {
                const int cw = s_cnt[w][q];
                if (cw > 0) {
                    const float2 nd = s_nd[w][q];
                    num += (double)nd.x + (double)nd.y * ((double)s_zref[w] - it.a.zref_acc);
                    den += nd.y;
                    cnt += cw;
                    lo = fminf(lo, s_lo[w][q]);
                    hi = fmaxf(hi, s_hi[w][q]);
                }
            }
            if (cnt > 0) {
                const int64_t o = (int64_t)(ta0 + la) * it.a.nx + tb0 + lb;
                const int c0 = it.a.acc_cnt[o];
                it.a.acc_num[o] += (float)num;
                it.a.acc_den[o] += den;
                it.a.acc_cnt[o] = c0 + cnt;
                // the depth range of every sounding accumulated so far
                it.a.acc_lo[o] = c0 > 0 ? fminf(it.a.acc_lo[o], lo) : lo;
                it.a.acc_hi[o] = c0 > 0 ? fmaxf(it.a.acc_hi[o], hi) : hi;
            }
        }
        __syncthreads();  // the LDS is reused by the next tile
    }
}

// Host-to-device staging of one launch: job j copies bytes [0, n) from
// pinned, coherent host memory (device-visible) to device memory, 16 bytes
// per lane.  Sizes and addresses are multiples of 16.
constexpr int kStageJobs = kMaxBatchReq + 1;
constexpr int kStageThreads = 256;
constexpr int kStageChunk = kStageThreads * 16 * 4;  // bytes per block

struct StageJob {
    const int4 *src;
    int4 *dst;
    int64_t n16;  // 16-byte words
};
struct StageArgs {
    int32_t count;
    StageJob job[kStageJobs];
};

__global__ __launch_bounds__(kStageThreads) void k_serve_stage(StageArgs args)
{
    const int j = blockIdx.y;
    if (j >= args.count)
        return;
    const StageJob jb = args.job[j];
    const int64_t base = (int64_t)blockIdx.x * (kStageChunk / 16);
    int4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + u * kStageThreads + threadIdx.x;
        if (i < jb.n16)
            v[u] = jb.src[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + u * kStageThreads + threadIdx.x;
        if (i < jb.n16)
            jb.dst[i] = v[u];
    }
}

// Read-out: z = z_ref + num / den, clamped to the depth range of the node's
// soundings; NaN where no sounding, or fewer than min_pts and no hit (a hit's
// weight makes den >= 2^80).
__global__ void k_serve_read(const float *__restrict__ num, const float *__restrict__ den,
                             const int32_t *__restrict__ cnt, const float *__restrict__ lo,
                             const float *__restrict__ hi, int64_t m, double zref,
                             int32_t min_pts, float *__restrict__ z_out,
                             int32_t *__restrict__ cnt_out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cnt[i];
        const float d = den[i];
        const bool hit = d >= win::kHitW;
        const bool hole = c == 0 || (c < min_pts && !hit);
        z_out[i] = hole ? NAN
                        : (float)fmin(fmax(zref + (double)num[i] / (double)d, (double)lo[i]),
                                      (double)hi[i]);
        if (cnt_out)
            cnt_out[i] = c;
    }
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// First-fit sub-allocator over the caller's arena (offsets, 256-byte units).
class Arena {
  public:
    void reset(size_t bytes)
    {
        free_.clear();
        if (bytes)
            free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Ticket {
    int32_t state, vehicle, slot;
    int64_t n;
    double t_arrival, t_launch, t_done;
};

struct Vehicle {
    auv_grid grid;
    BinGeom geom;
    WinGeom wg;
    IdwArgs base;
    double zref;
    int64_t nodes;
    bool admitted;
    size_t off;
    int64_t submitted, done;
};

struct Pick {
    uint64_t ticket;
    int32_t vehicle, slot;
    int64_t n;
};

struct Launch {
    std::vector<Pick> picks;
    int table;
    hipEvent_t ev;
};

// Launch table: device copy of what the kernels of one launch read.
struct TableLayout {
    size_t items, rows, offs, counters, bytes;
};

TableLayout table_layout()
{
    TableLayout t;
    size_t o = 0;
    t.items = o;
    o += align256(sizeof(ServeItem) * kMaxBatchReq);
    t.rows = o;
    o += align256(sizeof(RowItem) * kMaxBatchReq);
    t.offs = o;
    o += align256(sizeof(int32_t) * 3 * (kMaxBatchReq + 1));
    t.counters = o;
    o += align256(sizeof(int32_t) * 4);
    t.bytes = o;
    return t;
}

int32_t idx_bits_for(int64_t n)
{
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < n)
        ++bits;
    return bits;
}

}  // namespace
}  // namespace auv

struct auv_session {
    auv_session_desc desc;
    std::vector<auv::Vehicle> veh;
    int device = 0;
    int cus = 256;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    auv::Arena alloc;
    size_t slot_stage_bytes = 0, slot_ws_bytes = 0, per_vehicle = 0;
    std::vector<char *> slot_host, slot_map, slot_dev, slot_ws;  // slot_map: device view of slot_host
    std::vector<int32_t> free_slots;
    std::vector<char *> table_host, table_map, table_dev;  // table_map: device view of table_host
    hipEvent_t read_ev = nullptr;  // orders a read-out before the next launch
    std::vector<int> free_tables;
    std::vector<hipEvent_t> free_events, all_events;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_slot, cv_done;
    std::deque<auv::Pick> pending;
    std::deque<auv::Ticket> tickets;
    std::deque<auv::Launch> inflight;
    bool stop = false;
    bool failed = false;
    std::string error;
    std::thread worker;
    // requests queued so far; read by the worker without the lock while it
    // waits for a launch to finish
    std::atomic<uint64_t> n_queued{0};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace auv {
namespace {

auv_status validate_desc(const auv_session_desc *d, std::vector<Vehicle> *veh)
{
    if (!d)
        return fail(AUV_ERR_INVALID, "desc is null");
    if (d->n_vehicles < 1 || d->n_vehicles > 65536 || !d->grids)
        return fail(AUV_ERR_INVALID, "need 1..65536 vehicles and their grids");
    const auv_idw_params &p = d->params;
    if (!(p.power == 1.0 || p.power == 2.0 || p.power == 3.0))
        return fail(AUV_ERR_INVALID, "serving supports power 1, 2 or 3");
    if (p.max_pts != 0)
        return fail(AUV_ERR_INVALID, "serving needs max_pts 0 (a cap is not additive)");
    if (p.min_pts < 0)
        return fail(AUV_ERR_INVALID, "min_pts must be >= 0");
    if (p.precision != AUV_P_FP32_REBASE)
        return fail(AUV_ERR_INVALID, "serving runs the exact FP64-rebase form only");
    if (d->max_request < 1 || d->max_request > (1 << 24))
        return fail(AUV_ERR_INVALID, "max_request must be in [1, 2^24]");
    if (d->slots < 1 || d->slots > 4096)
        return fail(AUV_ERR_INVALID, "slots must be in [1, 4096]");
    if (d->mode != AUV_SERVE_FIFO && d->mode != AUV_SERVE_BATCHED)
        return fail(AUV_ERR_INVALID, "unknown serving mode");
    if (d->max_batch < 0 || d->max_batch > kMaxBatchReq)
        return fail(AUV_ERR_INVALID, "max_batch must be in [0, 64]");
    veh->assign(d->n_vehicles, Vehicle{});
    const int32_t bits = idx_bits_for(d->max_request);
    for (int v = 0; v < d->n_vehicles; ++v) {
        Vehicle &V = (*veh)[v];
        auv_grid *g = nullptr;
        auv_status st = auv_grid_create(&d->grids[v], &g);
        if (st != AUV_OK)
            return fail(st, "vehicle " + std::to_string(v) + ": " + auv_last_error());
        V.grid = *g;
        auv_grid_destroy(g);
        st = bin_geometry(&V.grid, p.radius, 0, &V.geom);
        if (st != AUV_OK)
            return fail(st, "vehicle " + std::to_string(v) + ": " + auv_last_error());
        if (!row_path_ok(V.geom))
            return fail(AUV_ERR_RANGE, "vehicle " + std::to_string(v) +
                                           ": grid too large for the row binning (8192 bins)");
        IdwArgs &a = V.base;
        std::memset(&a, 0, sizeof(a));
        a.dx = V.grid.d.dx;
        a.dy = V.grid.d.dy;
        a.nx = V.grid.d.nx;
        a.ny = V.grid.d.ny;
        a.R = V.geom.R;
        a.R_stage = V.geom.R;
        a.inv_r2 = (float)(1.0 / ((double)V.geom.R * V.geom.R));
        a.r2f = (float)(p.radius * p.radius);
        a.x0 = V.grid.d.x0;
        a.y0 = V.grid.d.y0;
        a.power = (float)p.power;
        a.pmode = (int32_t)p.power;
        a.min_pts = p.min_pts;
        a.max_pts = 0;
        a.precision = AUV_P_FP32_REBASE;
        a.mode = 5;
        V.zref = d->z_ref ? d->z_ref[v] : 0.0;
        if (!std::isfinite(V.zref))
            return fail(AUV_ERR_INVALID, "z_ref must be finite");
        a.zref_acc = V.zref;
        if (!window_geometry(a, &V.wg))
            return fail(AUV_ERR_INVALID, "vehicle " + std::to_string(v) +
                                             ": needs dx * 2^16 even and at most 256 nodes "
                                             "within a radius window");
        const unsigned __int128 top = (unsigned __int128)((unsigned long long)a.R * a.R) << bits;
        if (top >= ((unsigned __int128)1 << 64))
            return fail(AUV_ERR_RANGE, "radius too large for max_request");
        V.nodes = (int64_t)a.nx * a.ny;
    }
    return AUV_OK;
}

void budget_of(const auv_session_desc *d, const std::vector<Vehicle> &veh, size_t *stage,
               size_t *ws, size_t *fixed, size_t *per_vehicle)
{
    *stage = align256(kSlotHeader + 24 * (size_t)d->max_request);
    *ws = 0;
    int64_t nodes = 0;
    for (const Vehicle &V : veh) {
        *ws = std::max(*ws, align256(bin_workspace_layout(d->max_request, V.geom, nullptr, nullptr)));
        nodes = std::max(nodes, V.nodes);
    }
    const size_t tables = 2 * align256(table_layout().bytes);
    *fixed = tables + (size_t)d->slots * (*stage + *ws);
    // five planes: weighted depth, weight, count, smallest and largest depth
    *per_vehicle = 5 * align256(4 * (size_t)nodes);
}

// Enqueue one launch (no lock held; picks carry everything it needs).
auv_status enqueue_launch(auv_session *s, const std::vector<Pick> &picks, int table, hipEvent_t ev)
{
    const TableLayout L = table_layout();
    char *th = s->table_host[table];
    char *td = s->table_dev[table];
    ServeItem *items = reinterpret_cast<ServeItem *>(th + L.items);
    RowItem *rows = reinterpret_cast<RowItem *>(th + L.rows);
    int32_t *offs = reinterpret_cast<int32_t *>(th + L.offs);
    const int B = (int)picks.size();
    int32_t *hist_off = offs, *scat_off = offs + (B + 1), *sort_off = offs + 2 * (B + 1);
    int32_t *counters = reinterpret_cast<int32_t *>(th + L.counters);
    hist_off[0] = scat_off[0] = sort_off[0] = 0;
    bool chunks[win::kMaxChunks + 1] = {false, false, false, false, false};
    int64_t ntot = 0;
    int32_t max_nbx = 0, max_nby = 0;
    for (int i = 0; i < B; ++i) {
        const Pick &p = picks[i];
        const Vehicle &V = s->veh[p.vehicle];
        char *dev = s->slot_dev[p.slot];
        const double *x = reinterpret_cast<const double *>(dev + kSlotHeader);
        const double *y = x + p.n, *z = y + p.n;
        BinWorkspace w;
        bin_workspace_layout(p.n, V.geom, s->slot_ws[p.slot], &w);
        rows[i] = make_row_item(&V.grid, V.geom, x, y, z, p.n, w);
        rows[i].bbox = reinterpret_cast<int32_t *>(dev);  // seeded empty by the submit
        ServeItem &it = items[i];
        std::memset(&it, 0, sizeof(it));
        auv_bin_view &v = it.bv;
        v.cell_start = w.cell_start;
        v.X = w.X;
        v.Y = w.Y;
        v.res = w.res;
        v.z = w.z;
        v.idx = w.idx;
        v.rec = w.rec;
        v.nbx = V.geom.nbx;
        v.nby = V.geom.nby;
        v.halo = V.geom.halo;
        v.bin_log2 = V.geom.s;
        v.R = V.geom.R;
        v.idx_bits = idx_bits_for(p.n);
        it.a = V.base;
        float *acc = reinterpret_cast<float *>(s->arena + V.off);
        const size_t plane = align256(4 * (size_t)V.nodes) / 4;
        it.a.acc_num = acc;
        it.a.acc_den = acc + plane;
        it.a.acc_cnt = reinterpret_cast<int32_t *>(acc + 2 * plane);
        it.a.acc_lo = acc + 3 * plane;
        it.a.acc_hi = acc + 4 * plane;
        it.g = V.wg;
        it.ntx = (V.grid.d.nx + win::kTW - 1) / win::kTW;
        it.bbox = reinterpret_cast<const int32_t *>(dev);
        chunks[V.wg.nchunks] = true;
        hist_off[i + 1] = hist_off[i] + row_hist_blocks(p.n);
        scat_off[i + 1] = scat_off[i] + row_scatter_blocks(p.n);
        sort_off[i + 1] = sort_off[i] + V.geom.nby;
        max_nbx = std::max(max_nbx, V.geom.nbx);
        max_nby = std::max(max_nby, V.geom.nby);
        ntot += p.n;
    }
    for (int c = 0; c < 4; ++c)
        counters[c] = 0;
    // device pointers inside the table
    ServeItem *d_items = reinterpret_cast<ServeItem *>(td + L.items);
    RowItem *d_rows = reinterpret_cast<RowItem *>(td + L.rows);
    int32_t *d_offs = reinterpret_cast<int32_t *>(td + L.offs);
    int32_t *d_counters = reinterpret_cast<int32_t *>(td + L.counters);
    hipStream_t st = s->stream;
    // the table and the requests reach the device through one staging kernel
    StageArgs sa;
    sa.count = 1 + B;
    sa.job[0] = StageJob{reinterpret_cast<const int4 *>(s->table_map[table]),
                         reinterpret_cast<int4 *>(td), (int64_t)(L.bytes / 16)};
    int64_t most = sa.job[0].n16;
    for (int i = 0; i < B; ++i) {
        const Pick &p = picks[i];
        const int64_t n16 = (int64_t)((kSlotHeader + 24 * (size_t)p.n + 15) / 16);
        sa.job[1 + i] = StageJob{reinterpret_cast<const int4 *>(s->slot_map[p.slot]),
                                 reinterpret_cast<int4 *>(s->slot_dev[p.slot]), n16};
        most = std::max(most, n16);
    }
    const dim3 sgrid((unsigned)((most * 16 + kStageChunk - 1) / kStageChunk), (unsigned)sa.count);
    k_serve_stage<<<sgrid, kStageThreads, 0, st>>>(sa);
    AUV_TRY_S(launch_binning_batch(d_rows, d_offs, d_offs + (B + 1), d_offs + 2 * (B + 1), B,
                                   hist_off[B], scat_off[B], sort_off[B], max_nbx, max_nby,
                                   // a swath request fills a few rows of the vehicle's
                                   // grid densely: the largest key area
                                   1e30, st));
    // as many persistent blocks as fit at once (8 waves per CU)
    const int per_cu = std::max(1, 8 / kServeParts);
    const int blocks = (int)std::min<int64_t>((int64_t)per_cu * s->cus, 16 + ntot / 256);
    const int threads = 64 * kServeParts;
    if (chunks[1])
        k_serve_update<1><<<blocks, threads, 0, st>>>(d_items, B, d_counters + 0);
    if (chunks[2])
        k_serve_update<2><<<blocks, threads, 0, st>>>(d_items, B, d_counters + 1);
    if (chunks[3])
        k_serve_update<3><<<blocks, threads, 0, st>>>(d_items, B, d_counters + 2);
    if (chunks[4])
        k_serve_update<4><<<blocks, threads, 0, st>>>(d_items, B, d_counters + 3);
    AUV_HIP(hipGetLastError());
    AUV_HIP(hipEventRecord(ev, st));
    return AUV_OK;
}

void complete_front(auv_session *s, hipError_t q)
{
    Launch &L = s->inflight.front();
    const double t = s->now();
    for (const Pick &p : L.picks) {
        Ticket &tk = s->tickets[p.ticket - 1];
        tk.state = q == hipSuccess ? AUV_T_DONE : AUV_T_FAILED;
        tk.t_done = t;
        s->free_slots.push_back(p.slot);
        s->veh[p.vehicle].done += 1;
    }
    if (q != hipSuccess && !s->failed) {
        s->failed = true;
        s->error = std::string("launch failed: ") + hipGetErrorString(q);
    }
    s->free_tables.push_back(L.table);
    s->free_events.push_back(L.ev);
    s->inflight.pop_front();
}

void worker_main(auv_session *s)
{
    (void)hipSetDevice(s->device);
    const size_t max_inflight = s->desc.mode == AUV_SERVE_BATCHED ? 2 : 1;
    const size_t max_batch = s->desc.mode == AUV_SERVE_BATCHED
                                 ? (size_t)(s->desc.max_batch ? s->desc.max_batch : kMaxBatchReq)
                                 : 1;
    std::vector<uint8_t> taken(s->veh.size(), 0);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progressed = false;
        while (!s->inflight.empty()) {
            const hipError_t q = hipEventQuery(s->inflight.front().ev);
            if (q == hipErrorNotReady)
                break;
            complete_front(s, q);
            progressed = true;
        }
        if (progressed) {
            s->cv_slot.notify_all();
            s->cv_done.notify_all();
        }
        if (s->stop && s->pending.empty() && s->inflight.empty())
            break;
        if (s->inflight.size() < max_inflight && !s->pending.empty()) {
            // oldest first, at most one request per vehicle
            std::vector<Pick> picks;
            std::deque<Pick> rest;
            for (const Pick &p : s->pending) {
                if (picks.size() < max_batch && !taken[p.vehicle]) {
                    taken[p.vehicle] = 1;
                    picks.push_back(p);
                } else {
                    rest.push_back(p);
                }
            }
            for (const Pick &p : picks)
                taken[p.vehicle] = 0;
            s->pending.swap(rest);
            const double t = s->now();
            for (const Pick &p : picks) {
                s->tickets[p.ticket - 1].state = AUV_T_RUNNING;
                s->tickets[p.ticket - 1].t_launch = t;
            }
            const int table = s->free_tables.back();
            s->free_tables.pop_back();
            hipEvent_t ev = s->free_events.back();
            s->free_events.pop_back();
            lk.unlock();
            const auv_status st = enqueue_launch(s, picks, table, ev);
            const std::string msg = st == AUV_OK ? std::string() : std::string(auv_last_error());
            if (st != AUV_OK) {
                // part of the launch may be enqueued: let the stream settle,
                // then complete what is in flight, and this launch as failed
                (void)hipStreamSynchronize(s->stream);
            }
            lk.lock();
            if (st != AUV_OK && !s->failed) {
                s->failed = true;
                s->error = "launch failed: " + msg;
            }
            s->inflight.push_back(Launch{picks, table, ev});
            if (st != AUV_OK) {
                while (s->inflight.size() > 1)
                    complete_front(s, hipEventQuery(s->inflight.front().ev));
                complete_front(s, hipErrorLaunchFailure);
                s->cv_slot.notify_all();
                s->cv_done.notify_all();
            }
            continue;
        }
        if (!s->inflight.empty()) {
            // wait for the oldest launch without the session lock, so that
            // submits and polls never queue behind the worker; leave early
            // when a request arrives that a free launch could take
            const hipEvent_t ev = s->inflight.front().ev;
            const bool room = s->inflight.size() < max_inflight;
            const uint64_t seen = s->n_queued.load(std::memory_order_acquire);
            lk.unlock();
            while (hipEventQuery(ev) == hipErrorNotReady) {
                if (room && s->n_queued.load(std::memory_order_acquire) != seen)
                    break;
                std::this_thread::yield();
            }
            lk.lock();
            continue;
        }
        s->cv_work.wait(lk);
    }
}

}  // namespace
}  // namespace auv

using namespace auv;

extern "C" {

auv_status auv_session_budget(const auv_session_desc *desc, size_t *fixed, size_t *per_vehicle)
{
    if (!fixed || !per_vehicle)
        return fail(AUV_ERR_INVALID, "null output");
    std::vector<Vehicle> veh;
    AUV_TRY_S(validate_desc(desc, &veh));
    size_t stage, ws;
    budget_of(desc, veh, &stage, &ws, fixed, per_vehicle);
    return AUV_OK;
}

auv_status auv_session_create(const auv_session_desc *desc, void *arena, size_t arena_bytes,
                              auv_session **out)
{
    if (!out)
        return fail(AUV_ERR_INVALID, "out is null");
    *out = nullptr;
    std::vector<Vehicle> veh;
    AUV_TRY_S(validate_desc(desc, &veh));
    if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) != 0)
        return fail(AUV_ERR_INVALID, "arena must be a 256-byte aligned device pointer");
    size_t stage, ws, fixed, per_vehicle;
    budget_of(desc, veh, &stage, &ws, &fixed, &per_vehicle);
    if (arena_bytes < fixed)
        return fail(AUV_ERR_BUDGET, "arena of " + std::to_string(arena_bytes) +
                                        " bytes is below the fixed part of " +
                                        std::to_string(fixed));
    auv_session *s = new (std::nothrow) auv_session;
    if (!s)
        return fail(AUV_ERR_INVALID, "out of host memory");
    s->desc = *desc;
    s->desc.grids = nullptr;
    s->desc.z_ref = nullptr;
    s->veh = std::move(veh);
    s->arena = static_cast<char *>(arena);
    s->arena_bytes = arena_bytes;
    s->slot_stage_bytes = stage;
    s->slot_ws_bytes = ws;
    s->per_vehicle = per_vehicle;
    s->t0 = std::chrono::steady_clock::now();
    struct Undo {
        auv_session *s;
        bool keep = false;
        ~Undo()
        {
            if (!keep)
                auv_session_destroy(s);
        }
    } undo{s};
    AUV_HIP(hipGetDevice(&s->device));
    (void)hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
    AUV_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    AUV_HIP(hipEventCreateWithFlags(&s->read_ev, hipEventDisableTiming));
    // carve: tables, then slots; the rest is for vehicles
    const TableLayout L = table_layout();
    size_t off = 0;
    for (int t = 0; t < 2; ++t) {
        char *h = nullptr, *m = nullptr;
        // coherent: the staging kernel reads what the host wrote just before
        AUV_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), L.bytes,
                              hipHostMallocMapped | hipHostMallocCoherent));
        s->table_host.push_back(h);
        AUV_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&m), h, 0));
        s->table_map.push_back(m);
        s->table_dev.push_back(s->arena + off);
        off += align256(L.bytes);
        s->free_tables.push_back(t);
        hipEvent_t ev;
        AUV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        s->all_events.push_back(ev);
        s->free_events.push_back(ev);
    }
    for (int i = 0; i < desc->slots; ++i) {
        char *h = nullptr, *m = nullptr;
        AUV_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), stage,
                              hipHostMallocMapped | hipHostMallocCoherent));
        s->slot_host.push_back(h);
        AUV_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&m), h, 0));
        s->slot_map.push_back(m);
        s->slot_dev.push_back(s->arena + off);
        off += stage;
        s->slot_ws.push_back(s->arena + off);
        off += ws;
    }
    for (int i = desc->slots - 1; i >= 0; --i)
        s->free_slots.push_back(i);
    s->alloc.reset(0);
    if (arena_bytes > off)
        s->alloc.release(off, (arena_bytes - off) & ~size_t(255));
    s->worker = std::thread(worker_main, s);
    undo.keep = true;
    *out = s;
    return AUV_OK;
}

auv_status auv_session_submit(auv_session *s, int32_t vehicle, const double *x, const double *y,
                              const double *z, int64_t n, double t_arrival, uint64_t *ticket)
{
    if (!s || !ticket)
        return fail(AUV_ERR_INVALID, "null session or ticket");
    if (vehicle < 0 || vehicle >= (int32_t)s->veh.size())
        return fail(AUV_ERR_INVALID, "vehicle out of range");
    if (n < 0 || n > s->desc.max_request)
        return fail(AUV_ERR_INVALID, "n must be in [0, max_request]");
    if (n > 0 && (!x || !y || !z))
        return fail(AUV_ERR_INVALID, "null sounding pointer");
    int32_t slot;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop)
            return fail(AUV_ERR_STATE, "session is shutting down");
        Vehicle &V = s->veh[vehicle];
        if (!V.admitted) {
            size_t off;
            if (!s->alloc.alloc(s->per_vehicle, &off))
                return fail(AUV_ERR_BUDGET, "vehicle " + std::to_string(vehicle) +
                                                " cannot be admitted: the arena has no room "
                                                "for its grid sums");
            V.off = off;
            V.admitted = true;
            // cleared in stream order before any launch that reads it
            const hipError_t e = hipMemsetAsync(s->arena + off, 0, s->per_vehicle, s->stream);
            if (e != hipSuccess) {
                s->alloc.release(off, s->per_vehicle);
                V.admitted = false;
                return hip_fail(e, "hipMemsetAsync");
            }
        }
        s->cv_slot.wait(lk, [&] { return !s->free_slots.empty() || s->stop; });
        if (s->stop)
            return fail(AUV_ERR_STATE, "session is shutting down");
        slot = s->free_slots.back();
        s->free_slots.pop_back();
        V.submitted += 1;
    }
    // stage: bounding-box seed, then x, y, z back to back
    char *h = s->slot_host[slot];
    int32_t seed[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    std::memcpy(h, seed, sizeof(seed));
    if (n > 0) {
        std::memcpy(h + kSlotHeader, x, 8 * (size_t)n);
        std::memcpy(h + kSlotHeader + 8 * (size_t)n, y, 8 * (size_t)n);
        std::memcpy(h + kSlotHeader + 16 * (size_t)n, z, 8 * (size_t)n);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        Ticket tk{AUV_T_QUEUED, vehicle, slot, n, t_arrival, 0.0, 0.0};
        s->tickets.push_back(tk);
        const uint64_t id = s->tickets.size();
        s->pending.push_back(Pick{id, vehicle, slot, n});
        s->n_queued.fetch_add(1, std::memory_order_release);
        *ticket = id;
    }
    s->cv_work.notify_one();
    return AUV_OK;
}

auv_status auv_session_poll(auv_session *s, uint64_t ticket, auv_ticket_info *info)
{
    if (!s || !info)
        return fail(AUV_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket < 1 || ticket > s->tickets.size())
        return fail(AUV_ERR_INVALID, "unknown ticket");
    const Ticket &t = s->tickets[ticket - 1];
    info->state = t.state;
    info->vehicle = t.vehicle;
    info->n = t.n;
    info->t_arrival = t.t_arrival;
    info->t_launch = t.t_launch;
    info->t_done = t.t_done;
    return AUV_OK;
}

auv_status auv_session_drain(auv_session *s)
{
    if (!s)
        return fail(AUV_ERR_INVALID, "session is null");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->inflight.empty(); });
    if (s->failed)
        return fail(AUV_ERR_HIP, s->error);
    return AUV_OK;
}

static auv_status wait_vehicle(auv_session *s, int32_t vehicle, std::unique_lock<std::mutex> &lk)
{
    Vehicle &V = s->veh[vehicle];
    s->cv_done.wait(lk, [&] { return V.done == V.submitted; });
    if (s->failed)
        return fail(AUV_ERR_HIP, s->error);
    return AUV_OK;
}

auv_status auv_session_read_grid(auv_session *s, int32_t vehicle, float *z_out, int32_t *cnt_out,
                                 auv_stream stream)
{
    if (!s || !z_out)
        return fail(AUV_ERR_INVALID, "null session or z_out");
    if (vehicle < 0 || vehicle >= (int32_t)s->veh.size())
        return fail(AUV_ERR_INVALID, "vehicle out of range");
    std::unique_lock<std::mutex> lk(s->mu);
    AUV_TRY_S(wait_vehicle(s, vehicle, lk));
    const Vehicle &V = s->veh[vehicle];
    if (!V.admitted)
        return fail(AUV_ERR_STATE, "vehicle has no grid (never admitted or retired)");
    const float *acc = reinterpret_cast<const float *>(s->arena + V.off);
    const size_t plane = align256(4 * (size_t)V.nodes) / 4;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t blocks = std::min<int64_t>((V.nodes + 255) / 256, 8192);
    k_serve_read<<<(unsigned)std::max<int64_t>(blocks, 1), 256, 0, st>>>(
        acc, acc + plane, reinterpret_cast<const int32_t *>(acc + 2 * plane), acc + 3 * plane,
        acc + 4 * plane, V.nodes, V.zref, s->desc.params.min_pts, z_out, cnt_out);
    AUV_HIP(hipGetLastError());
    // later launches (picked after this point, the lock held) wait for the read
    AUV_HIP(hipEventRecord(s->read_ev, st));
    AUV_HIP(hipStreamWaitEvent(s->stream, s->read_ev, 0));
    return AUV_OK;
}

auv_status auv_session_retire(auv_session *s, int32_t vehicle)
{
    if (!s)
        return fail(AUV_ERR_INVALID, "session is null");
    if (vehicle < 0 || vehicle >= (int32_t)s->veh.size())
        return fail(AUV_ERR_INVALID, "vehicle out of range");
    std::unique_lock<std::mutex> lk(s->mu);
    AUV_TRY_S(wait_vehicle(s, vehicle, lk));
    Vehicle &V = s->veh[vehicle];
    if (!V.admitted)
        return fail(AUV_ERR_STATE, "vehicle is not admitted");
    s->alloc.release(V.off, s->per_vehicle);
    V.admitted = false;
    return AUV_OK;
}

double auv_session_now(const auv_session *s) { return s ? s->now() : 0.0; }

void auv_session_destroy(auv_session *s)
{
    if (!s)
        return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->cv_slot.notify_all();
        s->worker.join();
    }
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->all_events)
        (void)hipEventDestroy(e);
    if (s->read_ev)
        (void)hipEventDestroy(s->read_ev);
    for (char *h : s->slot_host)
        (void)hipHostFree(h);
    for (char *h : s->table_host)
        (void)hipHostFree(h);
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
