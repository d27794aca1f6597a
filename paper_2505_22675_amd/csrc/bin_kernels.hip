// Binning of soundings into a cell hash: a stable counting sort on gfx950.
//
//   k_rebase_count   FP64 rebase of each sounding onto the 2^-16 m lattice of
//                    the grid, validity / domain test, bin id, atomic
//                    histogram (the atomic's return value is the arrival slot)
//   k_scan_*         exclusive prefix sum of the histogram -> cell_start
//   k_scatter        position = cell_start[bin] + slot  (unordered in a bin)
//   k_stabilise_*    rank every bin's members by original index and write the
//                    binned structure-of-arrays in (bin, original index) order
//
// The result is deterministic although the histogram uses atomics: the slot
// order inside a bin is discarded by the ranking step.
#include "auv_internal.hpp"

#include <algorithm>
#include <climits>
#include <cmath>

// Discrete decisions below depend on exact FP64 rounding: no contraction.
#pragma clang fp contract(off)

namespace auv {

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;  // 2048 bins per scan block
constexpr int kSmallBin = 48;                      // bins ranked by one thread
constexpr int kBigBinLds = 8192;                   // members staged in LDS

__device__ inline int lane_id() { return __lane_id(); }

// Inclusive scan of one value per lane across a 64-wide wavefront.
__device__ inline int wave_inclusive_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d)
            v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across a 256-thread block; also
// returns the block total.  Uses `lds` (4 ints).
__device__ inline int block_exclusive_scan(int v, int *lds, int *total)
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
    int inc = wave_inclusive_scan(v);
    if (lane == 63)
        lds[wave] = inc;
    __syncthreads();
    int base = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        int t = lds[w];
        base += (w < wave) ? t : 0;
        sum += t;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int n)
{
    if ((int)threadIdx.x < n)
        p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads) void k_rebase_count(
    const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, int64_t n, double x0, double y0, int32_t s,
    int32_t hB, int32_t nbx, double lo, double hix, double hiy,
    int32_t *__restrict__ counts, int32_t *__restrict__ key,
    int32_t *__restrict__ slot, int4 *__restrict__ rec,
    unsigned long long *__restrict__ stats)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int bad = 0, out = 0;
    if (i < n) {
        const double xi = x[i], yi = y[i], zi = z[i];
        int k = -1, sl = 0;
        if (!(isfinite(xi) && isfinite(yi) && isfinite(zi))) {
            bad = 1;  // NaN / infinite samples are invalid candidates
        } else {
            const double tx = (xi - x0) * kLatticePerMetre;
            const double ty = (yi - y0) * kLatticePerMetre;
            const double rx = rint(tx), ry = rint(ty);  // nearest-even
            if (rx >= lo && rx < hix && ry >= lo && ry < hiy) {
                const int X = (int)rx, Y = (int)ry;
                k = ((Y + hB) >> s) * nbx + ((X + hB) >> s);
                sl = atomicAdd(&counts[k], 1);
                // residual in [-1/2, 1/2] lattice units, exact in FP64, kept
                // as 16-bit fixed point of 2^-15 lattice units
                const int qx = (int)rint((tx - rx) * 32768.0);
                const int qy = (int)rint((ty - ry) * 32768.0);
                const uint32_t r = ((uint32_t)qx & 0xffffu) | ((uint32_t)qy << 16);
                rec[i] = make_int4(X, Y, (int)r, __float_as_int((float)zi));
            } else {
                out = 1;  // cannot reach any node
            }
        }
        key[i] = k;
        slot[i] = sl;
    }
    const unsigned long long mb = __ballot(bad), mo = __ballot(out);
    if (lane_id() == 0) {
        if (mb)
            atomicAdd(&stats[1], (unsigned long long)__popcll(mb));
        if (mo)
            atomicAdd(&stats[2], (unsigned long long)__popcll(mo));
    }
}

// Phase 1 of the scan: one partial sum per tile of kScanTile bins.
__global__ __launch_bounds__(kThreads) void k_scan_reduce(
    const int32_t *__restrict__ in, int64_t nb, int32_t *__restrict__ partials)
{
    __shared__ int lds[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < nb)
            v += in[base + j];
    int total;
    block_exclusive_scan(v, lds, &total);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = total;
}

// Phase 2: exclusive scan of the partials by a single block.
__global__ __launch_bounds__(kThreads) void k_scan_partials(int32_t *partials, int64_t np)
{
    __shared__ int lds[kThreads / 64];
    int carry = 0;
    for (int64_t c = 0; c < np; c += kThreads) {
        const int64_t i = c + threadIdx.x;
        const int v = i < np ? partials[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, lds, &total);
        if (i < np)
            partials[i] = carry + ex;
        carry += total;
    }
}

// Phase 3: scan each tile and add its offset; the block holding the last bin
// also writes cell_start[nb] = number of binned soundings.
__global__ __launch_bounds__(kThreads) void k_scan_down(
    const int32_t *__restrict__ in, int64_t nb, const int32_t *__restrict__ partials,
    int32_t *__restrict__ out, unsigned long long *__restrict__ stats)
{
    __shared__ int lds[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + j < nb ? in[base + j] : 0;
        sum += v[j];
    }
    int total;
    int run = block_exclusive_scan(sum, lds, &total) + partials[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < nb)
            out[base + j] = run;
        run += v[j];
        if (base + j == nb - 1) {
            out[nb] = run;
            stats[0] = (unsigned long long)run;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_scatter(
    const int32_t *__restrict__ key, const int32_t *__restrict__ slot, int64_t n,
    const int32_t *__restrict__ cell_start, int32_t *__restrict__ perm_tmp)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) {
        const int k = key[i];
        if (k >= 0)
            perm_tmp[cell_start[k] + slot[i]] = (int32_t)i;
    }
}

struct SoA {
    int32_t *X, *Y;
    uint32_t *res;
    float *z;
    int32_t *idx;
};

__device__ inline void emit(const SoA &o, int pos, int orig, const int4 *rec)
{
    const int4 r = rec[orig];
    o.X[pos] = r.x;
    o.Y[pos] = r.y;
    o.res[pos] = (uint32_t)r.z;
    o.z[pos] = __int_as_float(r.w);
    o.idx[pos] = orig;
}

// One thread per bin: rank each member by original index (members are
// distinct indices, so rank = number of smaller ones) and write it there.
// Longer bins are queued for k_stabilise_big.
__global__ __launch_bounds__(kThreads) void k_stabilise_small(
    const int32_t *__restrict__ cell_start, int64_t nb,
    const int32_t *__restrict__ perm_tmp, const int4 *__restrict__ rec, SoA o,
    int32_t *__restrict__ big_list, unsigned long long *__restrict__ stats)
{
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= nb)
        return;
    const int s = cell_start[b], e = cell_start[b + 1];
    const int len = e - s;
    if (len == 0)
        return;
    if (len > kSmallBin) {
        const unsigned long long q = atomicAdd(&stats[3], 1ull);
        big_list[q] = (int32_t)b;
        return;
    }
    for (int j = s; j < e; ++j) {
        const int v = perm_tmp[j];
        int rank = 0;
        for (int k = s; k < e; ++k)
            rank += perm_tmp[k] < v ? 1 : 0;
        emit(o, s + rank, v, rec);
    }
}

// One block per long bin (grid-stride over the queue whose length the
// device wrote); members staged in LDS when they fit.
__global__ __launch_bounds__(kThreads) void k_stabilise_big(
    const int32_t *__restrict__ cell_start, const int32_t *__restrict__ perm_tmp,
    const int4 *__restrict__ rec, SoA o, const int32_t *__restrict__ big_list,
    const unsigned long long *__restrict__ stats)
{
    __shared__ int lds[kBigBinLds];
    const long long nbig = (long long)stats[3];
    for (long long q = blockIdx.x; q < nbig; q += gridDim.x) {
        const int b = big_list[q];
        const int s = cell_start[b], e = cell_start[b + 1];
        const int len = e - s;
        if (len <= kBigBinLds) {
            for (int t = threadIdx.x; t < len; t += kThreads)
                lds[t] = perm_tmp[s + t];
            __syncthreads();
            for (int t = threadIdx.x; t < len; t += kThreads) {
                const int v = lds[t];
                int rank = 0;
                for (int k = 0; k < len; ++k)
                    rank += lds[k] < v ? 1 : 0;
                emit(o, s + rank, v, rec);
            }
            __syncthreads();
        } else {
            for (int t = threadIdx.x; t < len; t += kThreads) {
                const int v = perm_tmp[s + t];
                int rank = 0;
                for (int k = 0; k < len; ++k)
                    rank += perm_tmp[s + k] < v ? 1 : 0;
                emit(o, s + rank, v, rec);
            }
        }
    }
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline unsigned grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)std::max<int64_t>(g, 1);
}

}  // namespace

int32_t default_bin_log2(int32_t R)
{
    int s = 31 - __builtin_clz((unsigned)std::max(R, 1));
    return std::min(26, std::max(12, s));
}

auv_status bin_geometry(const auv_grid *g, double radius, int32_t bin_log2,
                        BinGeom *out)
{
    if (!g || !out)
        return fail(AUV_ERR_INVALID, "null grid or output");
    if (!(radius > 0.0) || !(radius <= 256.0))
        return fail(AUV_ERR_INVALID, "radius must be in (0, 256] metres");
    const double Rd = std::rint(radius * kLatticePerMetre);
    if (Rd < 1.0)
        return fail(AUV_ERR_INVALID, "radius below one lattice unit");
    const int32_t R = (int32_t)Rd;
    const int32_t s = bin_log2 == 0 ? default_bin_log2(R) : bin_log2;
    if (s < 12 || s > 26)
        return fail(AUV_ERR_INVALID, "bin_log2 must be 0 or in [12, 26]");
    const int64_t B = int64_t(1) << s;
    const int64_t h = (R + B - 1) / B;
    const int64_t bx = (g->x_last + R + h * B) / B + 1;
    const int64_t by = (g->y_last + R + h * B) / B + 1;
    if (bx * B >= (int64_t(1) << 31) || by * B >= (int64_t(1) << 31) ||
        bx * by >= INT32_MAX)
        return fail(AUV_ERR_RANGE, "grid grown by the radius exceeds the lattice");
    out->R = R;
    out->s = s;
    out->halo = (int32_t)h;
    out->nbx = (int32_t)bx;
    out->nby = (int32_t)by;
    return AUV_OK;
}

size_t bin_workspace_layout(int64_t n, const BinGeom &g, char *base, BinWorkspace *w)
{
    const int64_t nb = (int64_t)g.nbx * g.nby;
    const int64_t np = (nb + kScanTile - 1) / kScanTile;
    const size_t m = (size_t)std::max<int64_t>(n, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    BinWorkspace t{};
    t.stats = (int64_t *)take(4 * sizeof(int64_t));
    t.counts = (int32_t *)take(sizeof(int32_t) * nb);
    t.cell_start = (int32_t *)take(sizeof(int32_t) * (nb + 1));
    t.partials = (int32_t *)take(sizeof(int32_t) * std::max<int64_t>(np, 1));
    t.big_list = (int32_t *)take(sizeof(int32_t) * nb);
    t.key = (int32_t *)take(sizeof(int32_t) * m);
    t.slot = (int32_t *)take(sizeof(int32_t) * m);
    t.rec = (int4 *)take(sizeof(int4) * m);
    t.perm_tmp = (int32_t *)take(sizeof(int32_t) * m);
    t.X = (int32_t *)take(sizeof(int32_t) * m);
    t.Y = (int32_t *)take(sizeof(int32_t) * m);
    t.res = (uint32_t *)take(sizeof(uint32_t) * m);
    t.z = (float *)take(sizeof(float) * m);
    t.idx = (int32_t *)take(sizeof(int32_t) * m);
    t.bytes = off;
    if (w)
        *w = t;
    return off;
}

auv_status launch_binning(const auv_grid *g, const BinGeom &geom, const double *x,
                          const double *y, const double *z, int64_t n,
                          const BinWorkspace &w, hipStream_t st)
{
    const int64_t nb = (int64_t)geom.nbx * geom.nby;
    const int64_t np = (nb + kScanTile - 1) / kScanTile;
    const int32_t hB = geom.halo << geom.s;
    const double lo = -(double)hB;
    const double hix = (double)(((int64_t)geom.nbx << geom.s) - hB);
    const double hiy = (double)(((int64_t)geom.nby << geom.s) - hB);
    auto *stats = reinterpret_cast<unsigned long long *>(w.stats);

    k_fill_i64<<<1, 64, 0, st>>>(w.stats, 4);
    k_fill_i32<<<(unsigned)std::min<int64_t>(grid_for(nb, kThreads), 4096), kThreads, 0, st>>>(
        w.counts, nb, 0);
    if (n > 0)
        k_rebase_count<<<grid_for(n, kThreads), kThreads, 0, st>>>(
            x, y, z, n, g->d.x0, g->d.y0, geom.s, hB, geom.nbx, lo, hix, hiy,
            w.counts, w.key, w.slot, w.rec, stats);
    k_scan_reduce<<<(unsigned)np, kThreads, 0, st>>>(w.counts, nb, w.partials);
    k_scan_partials<<<1, kThreads, 0, st>>>(w.partials, np);
    k_scan_down<<<(unsigned)np, kThreads, 0, st>>>(w.counts, nb, w.partials,
                                                   w.cell_start, stats);
    if (n > 0) {
        k_scatter<<<grid_for(n, kThreads), kThreads, 0, st>>>(w.key, w.slot, n,
                                                             w.cell_start, w.perm_tmp);
        SoA o{w.X, w.Y, w.res, w.z, w.idx};
        k_stabilise_small<<<grid_for(nb, kThreads), kThreads, 0, st>>>(
            w.cell_start, nb, w.perm_tmp, w.rec, o, w.big_list, stats);
        k_stabilise_big<<<(unsigned)std::min<int64_t>(std::max<int64_t>(nb, 1), 1024),
                          kThreads, 0, st>>>(w.cell_start, w.perm_tmp, w.rec, o,
                                             w.big_list, stats);
    }
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
