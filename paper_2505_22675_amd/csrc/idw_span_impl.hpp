// Radius-limited IDW and nearest pick, span form (gfx950): the window form's
// scatter from soundings to the nodes of a tile, with the work of several
// soundings packed into each instruction.
//
// One 64-lane wavefront owns a kTW x kTH tile of grid nodes; its per-node
// accumulators (weighted depth, weight, count, smallest and largest depth,
// packed (D^2, index) key) live in LDS.  For each batch of 64 candidate
// soundings (the binned soundings of the bin rows that meet the tile grown by
// the radius) the wave
//   1. keeps those whose node window meets the tile and writes their records
//      to LDS;
//   2. cuts each kept sounding's disk into one column span per tile row it
//      reaches (lane-parallel over (sounding, row)): the columns whose node
//      lies within the radius, from an FP32 bound with a safety margin, so the
//      span is a superset of the disk's nodes in that row;
//   3. expands the spans into (sounding, node) pairs in an LDS ring;
//   4. takes the pairs 64 at a time, one per lane: the exact lattice D^2
//      decides membership (the margin's extra nodes drop out here), and the
//      members' weights, depths, counts and keys go into the accumulators
//      through LDS atomics (pairs of one instruction may share a node).
// A 16 x 16 tile has about 16 in-disk, in-tile nodes per sounding visit at
// cfg2 (6 m radius, 2 m nodes): one lane per window cell, as in the window
// form, would leave three lanes in four idle.
//
// Exactness: membership, ranking, hits and the nearest pick on the exact
// lattice D^2 (64-bit integers); FP32 distances and weights from the lattice
// offsets plus the residuals; the quotient, the return to absolute depth and
// the clamp to the members' depth range in FP64, rounded once to FP32.  The
// wave's LDS atomics complete in instruction order and the lanes of one
// instruction in a fixed order, so the sums do not depend on timing.  Nodes
// with more than max_pts members are re-done exactly (exact_node).
//
// kPmode: 1, 2, 3 for a compile-time power, -1 for the power of a.pmode.
// Used for the exact lattice contract with an integer power (1, 2, 3), a key
// that fits 64 bits, node spacings below 2^22 lattice units and a window of
// at most 31 columns; every other case takes the window form.
#pragma once
#include "idw_window_impl.hpp"

namespace auv {
namespace span {

constexpr int kRing = 1024;          // pair ring (16-bit entries)
constexpr int kMaxRows = 64;         // bin rows per staging pass

template <int kTW, int kTH>
struct Shape {
    static constexpr int RS = kTW + 1;            // padded row stride (odd)
    static constexpr int NA = kTH * RS;           // accumulator slots
    static constexpr int kColBits = kTW <= 16 ? 4 : 5;
    static constexpr int kRowBits = kTH <= 16 ? 4 : 5;
    static_assert(kTW <= 32 && kTH <= 32, "pair entries hold 5-bit rows and columns");
    static_assert(6 + kColBits + kRowBits <= 16, "pair entries are 16 bits");
};

template <int kTW, int kTH>
struct Smem {
    float num[Shape<kTW, kTH>::NA];
    float den[Shape<kTW, kTH>::NA];
    int cnt[Shape<kTW, kTH>::NA];
    float lo[Shape<kTW, kTH>::NA];
    float hi[Shape<kTW, kTH>::NA];
    unsigned long long key[Shape<kTW, kTH>::NA];
    int beg[kMaxRows];
    int off[kMaxRows + 1];
    int4 r0[64];        // kept sounding: X - Xt0, Y - Yt0, first window row, index
    float4 r1[64];      //                residual x, residual y, depth - zref, depth
    unsigned short ring[kRing];  // (sounding << (r + c)) | (row << c) | column
};

// Span of tile columns of one (sounding, tile row): the nodes of the row that
// can lie within the radius.  dY is the exact lattice offset of the row from
// the sounding, px the sounding's lattice offset from column 0.  FP32 with a
// margin: R^2 (1 + 2^-20) bounds the FP32 rounding of R^2 - dY^2, and 1e-4 of
// a column bounds the rounding of the column quotients, so every node within
// the radius is inside [jlo, jhi].
__device__ inline void row_span(int px, int dY, float R2f, float invDX, int tw, int *jlo,
                                int *cnt)
{
    const float fy = (float)dY;
    const float h2 = fmaf(-fy, fy, R2f * (1.0f + 0x1p-20f));
    if (!(h2 >= 0.0f)) {
        *jlo = 0;
        *cnt = 0;
        return;
    }
    const float s = __builtin_sqrtf(h2);
    const float fx = (float)px;
    int a = (int)ceilf(fmaf(fx - s, invDX, -1e-4f));
    int b = (int)floorf(fmaf(fx + s, invDX, 1e-4f));
    a = max(a, 0);
    b = min(b, tw - 1);
    *jlo = a;
    *cnt = max(b - a + 1, 0);
}

template <int kMode, int kPmode, int kTW, int kTH>
__device__ void span_tile(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int tile,
                          int ntx, Smem<kTW, kTH> &sm)
{
    using S = Shape<kTW, kTH>;
    constexpr bool kIdw = (kMode & 1) != 0;
    constexpr bool kKey = (kMode & 2) != 0;  // the key serves the nearest outputs and hits
    constexpr int kCB = S::kColBits, kRB = S::kRowBits;
    const int lane = threadIdx.x & 63;
    const int tx = tile % ntx, ty = tile / ntx;
    const int tb0 = tx * kTW, ta0 = ty * kTH;
    const int tw = min(kTW, a.nx - tb0), th = min(kTH, a.ny - ta0);
    const int Xt0 = g.X0 + tb0 * g.DXl, Yt0 = g.Y0 + ta0 * g.DYl;
    const int R = a.R_stage;
    const long long R2 = (long long)a.R * a.R;
    const float R2f = (float)R2;
    const int kb = bv.idx_bits;
    // estimates with margins (row_span) or corrected exactly in integers
    const float invDX = __builtin_amdgcn_rcpf((float)g.DXl),
                invDY = __builtin_amdgcn_rcpf((float)g.DYl);
    // spans per sounding: the window rows padded to a power of two
    int wy_log = 0;
    while ((1 << wy_log) < g.Wy)
        ++wy_log;
    // spans per pass: the ring must hold one pass's pairs plus a partial chunk
    // (a span's FP32 margin can add one column to the window's Wx)
    const int span_lanes = min(64, (kRing - 64) / min(g.Wx + 1, kTW));

    for (int q = lane; q < S::NA; q += 64) {
        if constexpr (kIdw) {
            sm.num[q] = 0.0f;
            sm.den[q] = 0.0f;
        }
        sm.cnt[q] = 0;
        sm.lo[q] = INFINITY;
        sm.hi[q] = -INFINITY;
        if constexpr (kKey)
            sm.key[q] = ~0ull;
    }

    // bins covering the tile grown by R
    const int hB = bv.halo << bv.bin_log2;
    const int s = bv.bin_log2;
    const int bx_lo = max(0, (Xt0 - R + hB) >> s);
    const int nbx_row = min(bv.nbx - 1, (Xt0 + (tw - 1) * g.DXl + R + hB) >> s) - bx_lo + 1;
    const int by_lo = max(0, (Yt0 - R + hB) >> s);
    const int nrows = min(bv.nby - 1, (Yt0 + (th - 1) * g.DYl + R + hB) >> s) - by_lo + 1;

    float zref = 0.0f;
    bool have_ref = false;
    unsigned prod = 0, cons = 0;  // pairs written to / taken from the ring (wave-uniform)

    // take 64 pairs (or the last partial chunk) from the ring, one per lane
    auto consume = [&](unsigned upto) {
        while (cons < upto) {
            const unsigned p = cons + (unsigned)lane;
            if (p < upto) {
                const unsigned e = sm.ring[p & (kRing - 1)];
                const int j = (int)(e & ((1u << kCB) - 1u));
                const int r = (int)((e >> kCB) & ((1u << kRB) - 1u));
                const int k = (int)(e >> (kCB + kRB));
                const int4 v0 = sm.r0[k];
                const float4 v1 = sm.r1[k];
                const int dX = win::sext23(v0.x - j * g.DXl);
                const int dY = win::sext23(v0.y - r * g.DYl);
                const long long D2 = (long long)dX * dX + (long long)dY * dY;  // exact
                if (D2 <= R2) {
                    const int q = r * S::RS + j;
                    atomicAdd(&sm.cnt[q], 1);
                    __hip_atomic_fetch_min(&sm.lo[q], v1.w, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_max(&sm.hi[q], v1.w, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    if constexpr (kKey)
                        atomicMin(&sm.key[q],
                                  ((unsigned long long)D2 << kb) | (unsigned)v0.w);
                    if constexpr (kIdw) {
                        const float fx = (float)dX + v1.x, fy = (float)dY + v1.y;
                        const float d2f = fx * fx + fy * fy;
                        const float w =
                            D2 == 0 ? win::kHitW
                                    : win::weight_nonhit(d2f, kPmode > 0 ? kPmode : a.pmode);
                        atomicAdd(&sm.num[q], w * v1.z);
                        atomicAdd(&sm.den[q], w);
                    }
                }
            }
            cons = min(cons + 64u, upto);
        }
    };

    __syncthreads();  // accumulators cleared
    for (int r0 = 0; r0 < nrows; r0 += kMaxRows) {
        const int nr = min(kMaxRows, nrows - r0);
        int beg = 0, len = 0;
        if (lane < nr) {
            const int id0 = (by_lo + r0 + lane) * bv.nbx + bx_lo;
            beg = bv.cell_start[id0];
            len = bv.cell_start[id0 + nbx_row] - beg;
        }
        int inc = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(inc, d, 64);
            if (lane >= d)
                inc += u;
        }
        const int total = __shfl(inc, 63, 64);
        __syncthreads();
        if (lane < nr) {
            sm.beg[lane] = beg;
            sm.off[lane] = inc - len;
        }
        if (lane == 0)
            sm.off[nr] = total;
        __syncthreads();
        for (int c0 = 0; c0 < total; c0 += 64) {
            const int gi = c0 + lane;
            bool keep = false;
            int xr = 0, yr = 0, ia = 0, idx = 0;
            float rx = 0.0f, ry = 0.0f, z = 0.0f;
            if (gi < total) {
                int lo = 0, hi = nr - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sm.off[mid] <= gi)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const int k = sm.beg[lo] + (gi - sm.off[lo]);
                xr = bv.X[k] - Xt0;
                yr = bv.Y[k] - Yt0;
                // first window column / row: ceil((xr - R) / DX), from a float
                // estimate corrected exactly in integers
                int jb = (int)ceilf((float)(xr - R) * invDX);
                jb += (jb - 1) * g.DXl >= xr - R ? -1 : 0;
                jb += jb * g.DXl < xr - R ? 1 : 0;
                ia = (int)ceilf((float)(yr - R) * invDY);
                ia += (ia - 1) * g.DYl >= yr - R ? -1 : 0;
                ia += ia * g.DYl < yr - R ? 1 : 0;
                keep = jb <= tw - 1 && jb + g.Wx - 1 >= 0 && ia <= th - 1 && ia + g.Wy - 1 >= 0;
                const uint32_t res = bv.res[k];
                rx = (float)(int16_t)(res & 0xffffu) * kResidualUnit;
                ry = (float)(int16_t)(res >> 16) * kResidualUnit;
                z = bv.z[k];
                idx = bv.idx[k];
            }
            const unsigned long long m = __ballot(keep);
            if (m == 0ull)
                continue;
            if (!have_ref) {
                // the depth of the first kept sounding is the tile's reference
                zref = __shfl(z, __ffsll((long long)m) - 1, 64);
                have_ref = true;
            }
            const int nkept = __popcll(m);
            if (keep) {
                const int slot = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                sm.r0[slot] = make_int4(xr, yr, ia, idx);
                sm.r1[slot] = make_float4(rx, ry, z - zref, z);
            }
            __builtin_amdgcn_wave_barrier();
            // spans: lane -> (sounding k, window row i)
            const int nspans = nkept << wy_log;
            for (int s0 = 0; s0 < nspans; s0 += span_lanes) {
                const int si = s0 + lane;
                int jlo = 0, c = 0, row = 0, k = 0;
                if (lane < span_lanes && si < nspans) {
                    k = si >> wy_log;
                    const int i = si & ((1 << wy_log) - 1);
                    const int4 v0 = sm.r0[k];
                    row = v0.z + i;
                    if (i < g.Wy && row >= 0 && row < th)
                        row_span(v0.x, v0.y - row * g.DYl, R2f, invDX, tw, &jlo, &c);
                }
                int incl = c;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int u = __shfl_up(incl, d, 64);
                    if (lane >= d)
                        incl += u;
                }
                const unsigned base = prod + (unsigned)(incl - c);
                const unsigned e0 = ((unsigned)k << (kCB + kRB)) | ((unsigned)row << kCB) |
                                    (unsigned)jlo;
                for (int t = 0; __ballot(t < c); ++t)
                    if (t < c)
                        sm.ring[(base + (unsigned)t) & (kRing - 1)] =
                            (unsigned short)(e0 + (unsigned)t);
                prod += (unsigned)__shfl(incl, 63, 64);
                __builtin_amdgcn_wave_barrier();
                consume(cons + ((prod - cons) & ~63u));
            }
            consume(prod);  // the records are rewritten by the next batch
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();

    // finalize: one node per lane
    const int kcap = a.max_pts;
    const unsigned long long imask = (1ull << kb) - 1ull;
    for (int q0 = 0; q0 < kTW * kTH; q0 += 64) {
        const int qq = q0 + lane;
        const int la = qq / kTW, lb = qq - la * kTW;
        const int q = la * S::RS + lb;
        const bool act = la < th && lb < tw;
        const int cnt = sm.cnt[q];
        const bool over = act && kcap > 0 && cnt > kcap;
        if (act && !over) {
            const int64_t o = (int64_t)(ta0 + la) * a.nx + tb0 + lb;
            bool hit;
            if constexpr (kKey) {
                const unsigned long long key = sm.key[q];
                const int bi = (int)(key & imask);
                hit = cnt > 0 && (key >> kb) == 0ull;
                if (a.nn_idx_out)
                    a.nn_idx_out[o] = cnt > 0 ? bi : -1;
                if (a.nn_z_out)
                    a.nn_z_out[o] = cnt > 0 ? __int_as_float(bv.rec[bi].w) : NAN;
            } else {
                hit = kIdw && sm.den[q] >= win::kHitW;
            }
            if constexpr (kIdw) {
                if (a.cnt_out)
                    a.cnt_out[o] = cnt;
                // a hit carries a dominant weight, so the ratio is the mean of
                // the hits, and it beats min_pts
                const bool hole = cnt == 0 || (cnt < a.min_pts && !hit);
                const double v = (double)zref + (double)sm.num[q] / (double)sm.den[q];
                a.z_out[o] = hole ? NAN
                                  : (float)fmin(fmax(v, (double)sm.lo[q]), (double)sm.hi[q]);
            }
        }
        unsigned long long om = __ballot(over);
        while (om) {
            const int l = __ffsll((long long)om) - 1;
            om &= om - 1;
            const int qn = q0 + l;
            win::exact_node<kMode, kPmode, AUV_P_FP32_REBASE>(bv, a, g.X0, g.Y0, g.DXl, g.DYl,
                                                              ta0 + qn / kTW, tb0 + qn % kTW,
                                                              zref);
        }
    }
}

template <int kMode, int kPmode, int kTW, int kTH>
__global__ __launch_bounds__(64) void k_idw_span(auv_bin_view bv, IdwArgs a, WinGeom g, int ntx,
                                                  int nty)
{
    __shared__ Smem<kTW, kTH> sm;
    span_tile<kMode, kPmode, kTW, kTH>(bv, a, g, win::xcd_tile(blockIdx.x, ntx * nty), ntx, sm);
}

// Whether the span form covers this launch (see the header comment).
inline bool span_ok(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int pmode)
{
    if (a.precision != AUV_P_FP32_REBASE || pmode < 1 || pmode > 3 || a.mode < 1 || a.mode > 3)
        return false;
    if (g.DXl >= (1 << 22) || g.DYl >= (1 << 22) || g.Wx > 31)
        return false;
    const unsigned __int128 top = (unsigned __int128)((unsigned long long)a.R * a.R)
                                  << bv.idx_bits;
    return top < ((unsigned __int128)1 << 64);
}

template <int kMode, int kTW, int kTH>
void launch_shape(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int pmode,
                  hipStream_t st)
{
    const int ntx = (a.nx + kTW - 1) / kTW, nty = (a.ny + kTH - 1) / kTH;
    const dim3 grid((unsigned)(ntx * nty)), block(64);
    switch (pmode) {
    case 1: k_idw_span<kMode, 1, kTW, kTH><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    case 2: k_idw_span<kMode, 2, kTW, kTH><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    default: k_idw_span<kMode, 3, kTW, kTH><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    }
}

}  // namespace span
}  // namespace auv
