// Binning of soundings into a cell hash: a stable counting sort on gfx950.
// Two paths give the same result (bins in id order, each bin's members in
// original index order): the row path further below, for bin domains of at
// most 8192 rows and columns (its histograms live in LDS), and this general
// path for larger ones:
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
    int32_t *__restrict__ slot, int4 *__restrict__ rec, int32_t *__restrict__ drops)
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
    int tb, tob;
    {
        __shared__ int lds_b[kThreads / 64];
        block_exclusive_scan(bad, lds_b, &tb);
        block_exclusive_scan(out, lds_b, &tob);
    }
    if (threadIdx.x == 0) {
        drops[2 * blockIdx.x] = tb;
        drops[2 * blockIdx.x + 1] = tob;
    }
}

// Sum of the per-block drop counters of k_rebase_count (one block).
__global__ __launch_bounds__(kThreads) void k_sum_drops(const int32_t *__restrict__ drops,
                                                        int32_t nblk,
                                                        unsigned long long *__restrict__ stats)
{
    long long nbad = 0, nout = 0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        nbad += drops[2 * b];
        nout += drops[2 * b + 1];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        nbad += __shfl_xor(nbad, d, 64);
        nout += __shfl_xor(nout, d, 64);
    }
    if (lane_id() == 0) {
        atomicAdd(&stats[1], (unsigned long long)nbad);
        atomicAdd(&stats[2], (unsigned long long)nout);
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

// ----------------------------------------------------------- row path ----
//
// Two-level counting sort used when the bin rows fit an LDS histogram:
//   k_row_hist    rebase + per-block LDS histogram over bin rows; one global
//                 atomic per (block, non-empty row) reserves the block's range
//   k_row_scatter every block scans the row counts in LDS (block 0 publishes
//                 the row starts and the drop totals), then writes each
//                 sounding's (column, index) key into its row's range
//   k_row_sort    one block per bin row: counting sort by bin column in LDS
//                 (which also yields the row's cell_start entries), then rank
//                 each bin's members by original index; write the binned SoA.
// Device-scope atomics drop from one per sounding to one per block and row.
// LDS is sized per launch from the bin domain (rows, columns), so small
// domains keep many blocks resident.

constexpr int kRowChunk = 1024;          // soundings per block in k_row_hist
constexpr int kRowPerThread = kRowChunk / kThreads;
constexpr int kMaxRowsLds = 8192;        // bin rows in the LDS histogram
constexpr int kScatterPer = 4;           // soundings per thread in k_row_scatter
constexpr int kRunsMax = 8;              // row runs per wave for the grouped reservation

__device__ void row_hist_block(const RowItem &it, int blk, int *s_cnt)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const auto x = gmem(it.x);
    const auto y = gmem(it.y);
    const auto z = gmem(it.z);
    const int64_t n = it.n;
    const double x0 = it.x0, y0 = it.y0, lo = it.lo, hix = it.hix, hiy = it.hiy;
    const int32_t s = it.s, hB = it.hB, nby = it.nby;
    const auto row_count = gmem(it.row_count);
    const auto rowid = gmem(it.rowid);
    const auto pos = gmem(it.pos);
    const auto colkey = gmem(it.colkey);
    const auto rec = gmem(reinterpret_cast<v4i *>(it.rec));
    const auto drops = gmem(it.drops);
    for (int r = threadIdx.x; r < nby; r += kThreads)
        s_cnt[r] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blk * kRowChunk + threadIdx.x;
    int row[kRowPerThread], lr[kRowPerThread];
    int bad = 0, out = 0;
    int blx = INT_MAX, bly = INT_MAX, bhx = INT_MIN, bhy = INT_MIN;  // box of the binned
#pragma unroll
    for (int j = 0; j < kRowPerThread; ++j) {
        const int64_t i = base + (int64_t)j * kThreads;
        row[j] = -1;
        lr[j] = 0;
        if (i < n) {
            const double xi = x[i], yi = y[i], zi = z[i];
            if (!(isfinite(xi) && isfinite(yi) && isfinite(zi))) {
                bad += 1;  // NaN / infinite samples are invalid candidates
            } else {
                const double tx = (xi - x0) * kLatticePerMetre;
                const double ty = (yi - y0) * kLatticePerMetre;
                const double rx = rint(tx), ry = rint(ty);
                if (rx >= lo && rx < hix && ry >= lo && ry < hiy) {
                    const int X = (int)rx, Y = (int)ry;
                    const int qx = (int)rint((tx - rx) * 32768.0);
                    const int qy = (int)rint((ty - ry) * 32768.0);
                    const uint32_t rr = ((uint32_t)qx & 0xffffu) | ((uint32_t)qy << 16);
                    rec[i] = v4i{X, Y, (int)rr, __float_as_int((float)zi)};
                    colkey[i] = (X + hB) >> s;
                    row[j] = (Y + hB) >> s;
                    blx = min(blx, X);
                    bhx = max(bhx, X);
                    bly = min(bly, Y);
                    bhy = max(bhy, Y);
                } else {
                    out += 1;
                }
            }
        }
        // Reserve slots in the block's row counters, one LDS atomic per
        // distinct row in the wave (a ping's beams share a bin row, so
        // per-lane atomics would serialise on one address) -- unless the
        // wave's rows change more than kRunsMax times (soundings in no
        // particular order): then one LDS atomic per lane, on mostly
        // distinct addresses.  Positions inside a row are arbitrary either
        // way; the row sort orders every row by (bin, original index).
        const int rj = row[j];
        const int rprev = __shfl_up(rj, 1, 64);
        const int runs = __popcll(__ballot(rj >= 0 && (lane_id() == 0 || rprev != rj)));
        unsigned long long pending = __ballot(rj >= 0);
        if (runs > kRunsMax) {
            if (rj >= 0)
                lr[j] = atomicAdd(&s_cnt[rj], 1);
            pending = 0ull;
        }
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int r = __shfl(rj, leader, 64);
            const unsigned long long grp = __ballot(rj == r) & pending;
            int b = 0;
            if (lane_id() == leader)
                b = atomicAdd(&s_cnt[r], __popcll(grp));
            b = __shfl(b, leader, 64);
            if ((grp >> lane_id()) & 1ull)
                lr[j] = b + __popcll(grp & ((1ull << lane_id()) - 1ull));
            pending &= ~grp;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nby; r += kThreads) {
        const int c = s_cnt[r];
        if (c)
            s_cnt[r] = __hip_atomic_fetch_add(&row_count[r], c, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRowPerThread; ++j) {
        const int64_t i = base + (int64_t)j * kThreads;
        if (i < n) {
            rowid[i] = row[j];
            pos[i] = row[j] >= 0 ? s_cnt[row[j]] + lr[j] : 0;
        }
    }
    if (it.bbox) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            blx = min(blx, __shfl_xor(blx, d, 64));
            bly = min(bly, __shfl_xor(bly, d, 64));
            bhx = max(bhx, __shfl_xor(bhx, d, 64));
            bhy = max(bhy, __shfl_xor(bhy, d, 64));
        }
        if (lane_id() == 0 && blx <= bhx) {
            atomicMin(&it.bbox[0], blx);
            atomicMin(&it.bbox[1], bly);
            atomicMax(&it.bbox[2], bhx);
            atomicMax(&it.bbox[3], bhy);
        }
    }
    // per-block drop counters (summed by block 0 of k_row_scatter: a device-wide atomic on
    // one address per wave would serialise at the memory side)
    int tb, tob;
    {
        __shared__ int lds_b[kThreads / 64];
        block_exclusive_scan(bad, lds_b, &tb);
        block_exclusive_scan(out, lds_b, &tob);
    }
    if (threadIdx.x == 0) {
        drops[2 * blk] = tb;
        drops[2 * blk + 1] = tob;
    }
}

// Row starts (exclusive scan of the row counts) into LDS, by every scatter
// block; block 0 also publishes them with the binned total and the drop
// counts summed over the k_row_hist blocks.  Then the block's soundings go to
// their rows: key = bin column << 32 | original index.
__device__ void row_scatter_block(const RowItem &it, int blk, int *s_rs, int *lds)
{
    const auto cnt = gmem(it.row_count);
    const int32_t nby = it.nby;
    // row starts: each thread sums a run of consecutive rows, one block scan
    // of the run sums, then each thread writes its run's starts
    const int per = (nby + kThreads - 1) / kThreads;
    const int r0 = min(nby, (int)threadIdx.x * per), r1 = min(nby, r0 + per);
    int sum = 0;
    for (int r = r0; r < r1; ++r)
        sum += cnt[r];
    int carry;
    int run = block_exclusive_scan(sum, lds, &carry);
    for (int r = r0; r < r1; ++r) {
        s_rs[r] = run;
        run += cnt[r];
    }
    __syncthreads();
    if (blk == 0) {
        const auto start = gmem(it.row_start);
        for (int i = threadIdx.x; i < nby; i += kThreads)
            start[i] = s_rs[i];
        const auto drops = gmem(it.drops);
        long long nbad = 0, nout = 0;
        for (int b = threadIdx.x; b < it.nblk; b += kThreads) {
            nbad += drops[2 * b];
            nout += drops[2 * b + 1];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            nbad += __shfl_xor(nbad, d, 64);
            nout += __shfl_xor(nout, d, 64);
        }
        if (lane_id() == 0) {
            atomicAdd(&it.stats[1], (unsigned long long)nbad);
            atomicAdd(&it.stats[2], (unsigned long long)nout);
        }
        if (threadIdx.x == 0) {
            start[nby] = carry;
            it.stats[0] = (unsigned long long)carry;
        }
    }
    const auto rowid = gmem(it.rowid);
    const auto pos = gmem(it.pos);
    const auto colkey = gmem(it.colkey);
    const auto keys = gmem(it.keys);
    const int64_t base = (int64_t)blk * (kThreads * kScatterPer) + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kScatterPer; ++j) {
        const int64_t i = base + (int64_t)j * kThreads;
        if (i < it.n) {
            const int r = rowid[i];
            if (r >= 0)
                keys[s_rs[r] + pos[i]] =
                    ((unsigned long long)(uint32_t)colkey[i] << 32) | (uint32_t)i;
        }
    }
}

// Ascending bitonic sort of a[0, n) for any n: the sequence is treated as
// padded with +inf up to a power of two, and pairs whose upper element lies in
// the padding are skipped (the mirrored first step of each merge keeps every
// comparison ascending, so padding never moves).  Whole block, any memory.
template <class P>
__device__ void block_bitonic_sort(P a, int n)
{
    using T = unsigned long long;
    int npow = 1;
    while (npow < n)
        npow <<= 1;
    const int pairs = npow >> 1;
    for (int size = 2; size <= npow; size <<= 1) {
        const int half = size >> 1;
        for (int t = threadIdx.x; t < pairs; t += kThreads) {
            const int blk = t / half, off = t - blk * half;
            const int i = blk * size + off, j = blk * size + size - 1 - off;
            if (j < n) {
                const T u = a[i], v = a[j];
                if (v < u) {
                    a[i] = v;
                    a[j] = u;
                }
            }
        }
        __threadfence_block();
        __syncthreads();
        for (int stride = size >> 2; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < pairs; t += kThreads) {
                const int blk = t / stride, off = t - blk * stride;
                const int i = blk * 2 * stride + off, j = i + stride;
                if (j < n) {
                    const T u = a[i], v = a[j];
                    if (v < u) {
                        a[i] = v;
                        a[j] = u;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
}

// One block per bin row: counting sort of the row's soundings by bin column
// (LDS histogram -> exclusive scan = the row's cell_start entries).  Inside a
// bin, members are ordered by original index: by ranking (rank = number of
// members with a smaller index) when every bin of the row is small, else by
// a bitonic sort of the row's (column, index) keys (in LDS when they fit,
// otherwise in place in the key array).  Rows of up to kRowLds keys rank in
// LDS: the keys are re-read (coalesced) from global memory in each pass and
// only the indices are scattered into their bins in LDS; longer rows rank
// through tmp_keys.  (Swath data gives lumpy rows: a ping line spans a bin
// row, so a row holds zero, one or two pings' worth of soundings.)
constexpr int kColsLds = 8192;
constexpr int kSmallRank = 64;     // largest bin ranked member by member
constexpr int kRowU = 8;           // keys per thread per pass: loads kept in flight
// The sort's LDS key area holds kKA u64 keys: rows of up to kKA keys are
// bitonic-sorted there, rows of up to 2 kKA keys rank there (as u32
// indices), and rows of up to kThreads * kSU keys are ranked in registers
// (kSU per thread) and written out through two LDS arrays of that length
// carved from it.  Longer rows take the global-memory paths.  Three sizes:
// a smaller area and fewer staged keys per thread let more blocks share a
// CU (registers and LDS), for rows that are short on average.
template <int kKA, int kSU>
struct SortCfg {
    static constexpr int kBitonic = kKA, kRank = 2 * kKA, kStage = kThreads * kSU;
    static_assert(2 * kThreads * kSU * sizeof(int32_t) <= kKA * sizeof(unsigned long long),
                  "row staging does not fit the key area");
    static_assert(kThreads * kSU <= 2 * kKA, "staged rows must take the LDS ranking");
};

// for (k = threadIdx.x; k < n; k += kThreads) f(k, keys[r0 + k]), with kRowU
// key loads issued before any is used
template <class KP, class F>
__device__ inline void for_row_keys(KP keys, int r0, int n, F f)
{
    for (int k0 = threadIdx.x; k0 < n; k0 += kThreads * kRowU) {
        unsigned long long kk[kRowU];
#pragma unroll
        for (int j = 0; j < kRowU; ++j) {
            const int k = k0 + j * kThreads;
            kk[j] = k < n ? keys[r0 + k] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kRowU; ++j) {
            const int k = k0 + j * kThreads;
            if (k < n)
                f(k, kk[j]);
        }
    }
}

template <int kKA, int kSU>
__device__ void row_sort_block(const RowItem &it, int row, int *s_h,
                               unsigned long long *s_k, int *lds)
{
    using C = SortCfg<kKA, kSU>;
    typedef int v4i __attribute__((ext_vector_type(4)));
    const auto keys = gmem(it.keys);
    const auto row_start = gmem(it.row_start);
    const int32_t nby = it.nby, nbx = it.nbx;
    const auto recv = gmem(reinterpret_cast<const v4i *>(it.rec));
    const auto oX = gmem(it.o.X), oY = gmem(it.o.Y), oIdx = gmem(it.o.idx);
    const auto oRes = gmem(it.o.res);
    const auto oZ = gmem(it.o.z);
    const auto cell_start = gmem(it.cell_start);
    auto load_rec = [&](uint32_t i) {
        const v4i q = recv[i];
        return make_int4(q.x, q.y, q.z, q.w);
    };
    auto emit_g = [&](int pos, int orig) {
        const int4 r = load_rec((uint32_t)orig);
        oX[pos] = r.x;
        oY[pos] = r.y;
        oRes[pos] = (uint32_t)r.z;
        oZ[pos] = __int_as_float(r.w);
        oIdx[pos] = orig;
    };
    const int r0 = row_start[row], n = row_start[row + 1] - r0;
    for (int bx = threadIdx.x; bx < nbx; bx += kThreads)
        s_h[bx] = 0;
    __syncthreads();
    for_row_keys(keys, r0, n, [&](int, unsigned long long key) {
        atomicAdd(&s_h[(int)(key >> 32)], 1);
    });
    __syncthreads();
    const auto cs = cell_start + (int64_t)row * nbx;
    // bin starts within the row: each thread sums a run of consecutive
    // columns, one block scan of the run sums, then each thread writes its
    // run's starts into s_h; cell_start is written from s_h, coalesced
    int big = 0;
    {
        const int per = (nbx + kThreads - 1) / kThreads;
        const int c0 = min(nbx, (int)threadIdx.x * per), c1 = min(nbx, c0 + per);
        int sum = 0;
        for (int bx = c0; bx < c1; ++bx) {
            const int v = s_h[bx];
            sum += v;
            big |= v > kSmallRank ? 1 : 0;
        }
        int total;
        int run = block_exclusive_scan(sum, lds, &total);
        for (int bx = c0; bx < c1; ++bx) {
            const int v = s_h[bx];
            s_h[bx] = run;
            run += v;
        }
        __syncthreads();
        for (int bx = threadIdx.x; bx < nbx; bx += kThreads)
            cs[bx] = r0 + s_h[bx];
    }
    if (row == nby - 1 && threadIdx.x == 0)
        cell_start[(int64_t)nby * nbx] = row_start[nby];
    if (__syncthreads_or(big)) {
        if (n <= C::kBitonic) {
            for (int k = threadIdx.x; k < n; k += kThreads)
                s_k[k] = keys[r0 + k];
            __syncthreads();
            block_bitonic_sort(s_k, n);
            for (int k = threadIdx.x; k < n; k += kThreads)
                emit_g(r0 + k, (int)(uint32_t)(s_k[k] & 0xffffffffull));
        } else {
            const auto a = keys + r0;
            block_bitonic_sort(a, n);
            for (int k = threadIdx.x; k < n; k += kThreads)
                emit_g(r0 + k, (int)(uint32_t)(a[k] & 0xffffffffull));
        }
        return;
    }
    if (n <= C::kRank) {
        // scatter the indices into their bins (unordered inside a bin);
        // afterwards s_h[bx] is the end of bin bx, i.e. the start of bx + 1
        uint32_t *s_i = reinterpret_cast<uint32_t *>(s_k);
        for_row_keys(keys, r0, n, [&](int, unsigned long long key) {
            const int p = atomicAdd(&s_h[(int)(key >> 32)], 1);
            s_i[p] = (uint32_t)key;
        });
        __syncthreads();
        if (n <= C::kStage) {
            // one pass: ranks and gathers in registers, then the records are
            // placed at their sorted slots in LDS (the index list is dead by
            // then) and written out contiguously, two arrays at a time
            const int k0 = threadIdx.x;
            uint32_t ix[kSU];
            int pos[kSU];
            int4 rr[kSU];
#pragma unroll
            for (int j = 0; j < kSU; ++j) {
                const int k = k0 + j * kThreads;
                const unsigned long long key = k < n ? keys[r0 + k] : 0ull;
                ix[j] = (uint32_t)key;
                pos[j] = k < n ? (int)(key >> 32) : -1;  // bin column until ranked
            }
#pragma unroll
            for (int j = 0; j < kSU; ++j) {
                if (pos[j] >= 0) {
                    const int bx = pos[j];
                    const int b0 = bx == 0 ? 0 : s_h[bx - 1], b1 = s_h[bx];
                    int rank = 0;
                    for (int q = b0; q < b1; ++q)
                        rank += s_i[q] < ix[j] ? 1 : 0;
                    pos[j] = b0 + rank;
                }
            }
#pragma unroll
            for (int j = 0; j < kSU; ++j)
                if (pos[j] >= 0)
                    rr[j] = load_rec(ix[j]);
            int32_t *s_a = reinterpret_cast<int32_t *>(s_k);
            int32_t *s_b = s_a + kThreads * kSU;
            __syncthreads();  // every rank is read: the index list is free
#pragma unroll
            for (int j = 0; j < kSU; ++j)
                if (pos[j] >= 0) {
                    s_a[pos[j]] = rr[j].x;
                    s_b[pos[j]] = rr[j].y;
                }
            __syncthreads();
            for (int k = threadIdx.x; k < n; k += kThreads) {
                oX[r0 + k] = s_a[k];
                oY[r0 + k] = s_b[k];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kSU; ++j)
                if (pos[j] >= 0) {
                    s_a[pos[j]] = rr[j].z;
                    s_b[pos[j]] = rr[j].w;
                }
            __syncthreads();
            for (int k = threadIdx.x; k < n; k += kThreads) {
                oRes[r0 + k] = (uint32_t)s_a[k];
                oZ[r0 + k] = __int_as_float(s_b[k]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kSU; ++j)
                if (pos[j] >= 0)
                    s_a[pos[j]] = (int)ix[j];
            __syncthreads();
            for (int k = threadIdx.x; k < n; k += kThreads)
                oIdx[r0 + k] = s_a[k];
            return;
        }
        // ranks first (LDS), then the kRowU record gathers in flight together
        for (int k0 = threadIdx.x; k0 < n; k0 += kThreads * kRowU) {
            unsigned long long kk[kRowU];
            int pos[kRowU];
            int4 rr[kRowU];
#pragma unroll
            for (int j = 0; j < kRowU; ++j) {
                const int k = k0 + j * kThreads;
                kk[j] = k < n ? keys[r0 + k] : 0ull;
            }
#pragma unroll
            for (int j = 0; j < kRowU; ++j) {
                pos[j] = -1;
                if (k0 + j * kThreads < n) {
                    const int bx = (int)(kk[j] >> 32);
                    const uint32_t v = (uint32_t)kk[j];
                    const int b0 = bx == 0 ? 0 : s_h[bx - 1], b1 = s_h[bx];
                    int rank = 0;
                    for (int q = b0; q < b1; ++q)
                        rank += s_i[q] < v ? 1 : 0;
                    pos[j] = r0 + b0 + rank;
                }
            }
#pragma unroll
            for (int j = 0; j < kRowU; ++j)
                if (pos[j] >= 0)
                    rr[j] = load_rec((uint32_t)kk[j]);
#pragma unroll
            for (int j = 0; j < kRowU; ++j)
                if (pos[j] >= 0) {
                    oX[pos[j]] = rr[j].x;
                    oY[pos[j]] = rr[j].y;
                    oRes[pos[j]] = (uint32_t)rr[j].z;
                    oZ[pos[j]] = __int_as_float(rr[j].w);
                    oIdx[pos[j]] = (int)(uint32_t)kk[j];
                }
        }
        return;
    }
    const auto tmp_keys = gmem(it.keys2);
    for (int k = threadIdx.x; k < n; k += kThreads) {
        const unsigned long long key = keys[r0 + k];
        const int p = atomicAdd(&s_h[(int)(key >> 32)], 1);
        tmp_keys[r0 + p] = key;
    }
    __threadfence_block();
    __syncthreads();
    // one thread per sounding: its rank among its bin's members
    for (int p = threadIdx.x; p < n; p += kThreads) {
        const unsigned long long key = tmp_keys[r0 + p];
        const int bx = (int)(key >> 32);
        const int b0 = bx == 0 ? 0 : s_h[bx - 1], b1 = s_h[bx];
        int rank = 0;
        for (int q = b0; q < b1; ++q)
            rank += tmp_keys[r0 + q] < key ? 1 : 0;
        emit_g(r0 + b0 + rank, (int)(uint32_t)(key & 0xffffffffull));
    }
}

// LDS bytes of the row-path kernels for a bin domain of nby rows, nbx columns.
inline size_t row_hist_lds(int nby) { return sizeof(int) * (size_t)nby; }
inline size_t row_scatter_lds(int nby) { return sizeof(int) * (size_t)nby; }
inline size_t row_sort_lds(int ka, int nbx)
{
    return sizeof(unsigned long long) * (size_t)ka + sizeof(int) * (size_t)nbx;
}

// Key-area configuration of the sort for rows averaging `keys_per_row`
// input soundings: 0 (1024 keys, 4 staged per thread), 1 (2048, 8), 2 (4096, 12).
inline int sort_config(double keys_per_row)
{
    return keys_per_row <= 256.0 ? 0 : keys_per_row <= 1024.0 ? 1 : 2;
}
inline int sort_config_ka(int c) { return c == 0 ? 1024 : c == 1 ? 2048 : 4096; }

// Single-item kernels.  Dynamic LDS: 8-byte aligned base.
__global__ __launch_bounds__(kThreads) void k_row_fill(RowItem it)
{
    for (int r = threadIdx.x; r < it.nby; r += kThreads)
        it.row_count[r] = 0;
    if (threadIdx.x < 4)
        it.stats[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads) void k_row_hist(RowItem it)
{
    extern __shared__ unsigned long long s_dyn[];
    row_hist_block(it, blockIdx.x, reinterpret_cast<int *>(s_dyn));
}

__global__ __launch_bounds__(kThreads) void k_row_scatter(RowItem it)
{
    extern __shared__ unsigned long long s_dyn[];
    __shared__ int lds[kThreads / 64];
    row_scatter_block(it, blockIdx.x, reinterpret_cast<int *>(s_dyn), lds);
}

template <int kKA, int kSU>
__global__ __launch_bounds__(kThreads) void k_row_sort(RowItem it)
{
    extern __shared__ unsigned long long s_dyn[];
    __shared__ int lds[kThreads / 64];
    row_sort_block<kKA, kSU>(it, blockIdx.x, reinterpret_cast<int *>(s_dyn + kKA), s_dyn, lds);
}

// Batched kernels: block b belongs to item item_of(off, count, b); the LDS is
// sized for the largest bin domain of the batch.

__global__ __launch_bounds__(kThreads) void k_row_fill_batch(const RowItem *items)
{
    const RowItem &it = items[blockIdx.x];
    for (int r = threadIdx.x; r < it.nby; r += kThreads)
        it.row_count[r] = 0;
    if (threadIdx.x < 4)
        it.stats[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads) void k_row_hist_batch(const RowItem *items,
                                                             const int32_t *off, int count)
{
    extern __shared__ unsigned long long s_dyn[];
    const int i = item_of(off, count, blockIdx.x);
    row_hist_block(items[i], blockIdx.x - off[i], reinterpret_cast<int *>(s_dyn));
}

__global__ __launch_bounds__(kThreads) void k_row_scatter_batch(const RowItem *items,
                                                                const int32_t *off, int count)
{
    extern __shared__ unsigned long long s_dyn[];
    __shared__ int lds[kThreads / 64];
    const int i = item_of(off, count, blockIdx.x);
    row_scatter_block(items[i], blockIdx.x - off[i], reinterpret_cast<int *>(s_dyn), lds);
}

template <int kKA, int kSU>
__global__ __launch_bounds__(kThreads) void k_row_sort_batch(const RowItem *items,
                                                             const int32_t *off, int count)
{
    extern __shared__ unsigned long long s_dyn[];
    __shared__ int lds[kThreads / 64];
    const int i = item_of(off, count, blockIdx.x);
    row_sort_block<kKA, kSU>(items[i], blockIdx.x - off[i],
                             reinterpret_cast<int *>(s_dyn + kKA), s_dyn, lds);
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
    // smallest power of two not below R: a node's disk meets at most 3 bins
    // per axis, and bin rows stay few for the row-wise counting sort
    int s = 0;
    while (s < 31 && (int64_t(1) << s) < R)
        ++s;
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
    t.partials = (int32_t *)take(
        sizeof(int32_t) * std::max<int64_t>(std::max<int64_t>(np, 2 * ((n + 1023) / 1024)), 2));
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
    t.row_count = (int32_t *)take(sizeof(int32_t) * g.nby);
    t.row_start = (int32_t *)take(sizeof(int32_t) * (g.nby + 1));
    t.rowid = (int32_t *)take(sizeof(int32_t) * m);
    t.keys = (unsigned long long *)take(sizeof(unsigned long long) * m);
    t.keys2 = (unsigned long long *)take(sizeof(unsigned long long) * m);
    t.drops = (int32_t *)take(sizeof(int32_t) * 2 * ((m + kThreads - 1) / kThreads + 1));
    t.bytes = off;
    if (w)
        *w = t;
    return off;
}

bool row_path_ok(const BinGeom &geom)
{
    return geom.nby <= kMaxRowsLds && geom.nbx <= kColsLds;
}

RowItem make_row_item(const auv_grid *g, const BinGeom &geom, const double *x,
                      const double *y, const double *z, int64_t n, const BinWorkspace &w)
{
    RowItem it{};
    it.x = x;
    it.y = y;
    it.z = z;
    it.n = n;
    it.x0 = g->d.x0;
    it.y0 = g->d.y0;
    it.hB = geom.halo << geom.s;
    it.lo = -(double)it.hB;
    it.hix = (double)(((int64_t)geom.nbx << geom.s) - it.hB);
    it.hiy = (double)(((int64_t)geom.nby << geom.s) - it.hB);
    it.s = geom.s;
    it.nbx = geom.nbx;
    it.nby = geom.nby;
    it.nblk = n > 0 ? (int32_t)grid_for(n, kRowChunk) : 0;
    it.bbox = nullptr;
    it.row_count = w.row_count;
    it.row_start = w.row_start;
    it.rowid = w.rowid;
    it.pos = w.slot;
    it.colkey = w.key;
    it.drops = w.partials;
    it.cell_start = w.cell_start;
    it.rec = w.rec;
    it.keys = w.keys;
    it.keys2 = w.keys2;
    it.stats = reinterpret_cast<unsigned long long *>(w.stats);
    it.o = SoA{w.X, w.Y, w.res, w.z, w.idx};
    return it;
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

    if (row_path_ok(geom)) {
        const RowItem it = make_row_item(g, geom, x, y, z, n, w);
        k_row_fill<<<1, kThreads, 0, st>>>(it);
        if (n > 0)
            k_row_hist<<<it.nblk, kThreads, row_hist_lds(geom.nby), st>>>(it);
        k_row_scatter<<<row_scatter_blocks(n), kThreads, row_scatter_lds(geom.nby), st>>>(it);
        const int sc = sort_config((double)n / std::max(1, geom.nby));
        const size_t sl = row_sort_lds(sort_config_ka(sc), geom.nbx);
        const unsigned sb = (unsigned)geom.nby;
        if (sc == 0)
            k_row_sort<1024, 4><<<sb, kThreads, sl, st>>>(it);
        else if (sc == 1)
            k_row_sort<2048, 8><<<sb, kThreads, sl, st>>>(it);
        else
            k_row_sort<4096, 12><<<sb, kThreads, sl, st>>>(it);
        AUV_HIP(hipGetLastError());
        return AUV_OK;
    }
    k_fill_i64<<<1, 64, 0, st>>>(w.stats, 4);
    k_fill_i32<<<(unsigned)std::min<int64_t>(grid_for(nb, kThreads), 4096), kThreads, 0, st>>>(
        w.counts, nb, 0);
    if (n > 0) {
        k_rebase_count<<<grid_for(n, kThreads), kThreads, 0, st>>>(
            x, y, z, n, g->d.x0, g->d.y0, geom.s, hB, geom.nbx, lo, hix, hiy,
            w.counts, w.key, w.slot, w.rec, w.drops);
        k_sum_drops<<<1, kThreads, 0, st>>>(w.drops, (int)grid_for(n, kThreads), stats);
    }
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


int32_t row_hist_blocks(int64_t n) { return n > 0 ? (int32_t)grid_for(n, kRowChunk) : 0; }
// at least one block: block 0 publishes the row starts even for no soundings
int32_t row_scatter_blocks(int64_t n) { return (int32_t)grid_for(n, kThreads * kScatterPer); }

auv_status launch_binning_batch(const RowItem *d_items, const int32_t *d_hist_off,
                                const int32_t *d_scatter_off, const int32_t *d_sort_off,
                                int32_t count, int32_t hist_blocks, int32_t scatter_blocks,
                                int32_t sort_blocks, int32_t max_nbx, int32_t max_nby,
                                double keys_per_row, hipStream_t st)
{
    if (count <= 0)
        return AUV_OK;
    if (max_nbx > kColsLds || max_nby > kMaxRowsLds)
        return fail(AUV_ERR_INVALID, "bin domain too large for the row path");
    k_row_fill_batch<<<count, kThreads, 0, st>>>(d_items);
    if (hist_blocks > 0)
        k_row_hist_batch<<<hist_blocks, kThreads, row_hist_lds(max_nby), st>>>(d_items,
                                                                             d_hist_off, count);
    k_row_scatter_batch<<<scatter_blocks, kThreads, row_scatter_lds(max_nby), st>>>(
        d_items, d_scatter_off, count);
    const int sc = sort_config(keys_per_row);
    const size_t sl = row_sort_lds(sort_config_ka(sc), max_nbx);
    if (sc == 0)
        k_row_sort_batch<1024, 4><<<sort_blocks, kThreads, sl, st>>>(d_items, d_sort_off, count);
    else if (sc == 1)
        k_row_sort_batch<2048, 8><<<sort_blocks, kThreads, sl, st>>>(d_items, d_sort_off, count);
    else
        k_row_sort_batch<4096, 12><<<sort_blocks, kThreads, sl, st>>>(d_items, d_sort_off, count);
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
