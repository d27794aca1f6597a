// Radius-limited IDW and nearest pick, window form (gfx950).
//
// One 64-lane wavefront owns a 16 x 16 tile of grid nodes whose accumulators
// live in LDS.  The binned soundings of the bin rows meeting the tile grown by
// the radius are read and compacted to those whose node window meets the
// tile.  For each of those, the 64 lanes cover its window of nodes
// (the nodes within +-R of it: at most floor(2R/dX)+1 per axis, <= 64 cells
// per pass), test membership exactly and update the member nodes'
// accumulators.  Within one instruction every lane owns a distinct node and
// soundings are applied in staging order, so the read-modify-write needs no
// atomics and the result is deterministic.
//
// Used when the node lattice is linear (dx * 2^15 and dy * 2^15 integers, so
// X_b = X_0 + b*DX exactly) and the window has at most 256 cells; the tile
// kernel in idw_kernels.hip covers every other grid.
//
// Exactness as in the tile kernel: membership, ranking and hits on the exact
// lattice D^2 (64-bit integers), FP32 distances/weights from lattice offsets
// plus residuals, FP64 final quotient, clamped to the smallest and largest
// depth of the node's selected set (tracked beside the sums), so that every
// value lies within its neighbours' depths also after rounding.  Sums are
// relative to one reference depth per tile (a sounding's depth, so a
// constant field stays exact).  A hit (D^2 == 0) enters with a dominant weight, which yields the
// mean of the hits; it is recognised at the end by a best key of D^2 == 0.
// Nodes with more than max_pts members are re-done exactly by the whole wave
// (bisection on the rank-k key over the node's candidates).
#pragma once
#include "auv_internal.hpp"

#include <climits>
#include <cmath>

namespace auv {

namespace win {

// 16 x 16: a wider tile would cross fewer tile edges per sounding but its
// LDS lowers the waves per SIMD, which costs more (measured 16 x 32: +19 %).
constexpr int kTW = 16;              // tile nodes per row (columns)
constexpr int kTH = 16;              // tile rows
constexpr int kNodes = kTW * kTH;    // nodes per wave
constexpr int kMaxRows = 64;         // bin rows per staging pass
constexpr int kMaxChunks = 4;        // window cells <= 64 * kMaxChunks
constexpr float kHitW = 0x1p80f;     // weight of a coincident sounding

// Tile rows of the window form: 16 (default) or 8.
__host__ __device__ inline int tile_rows(const IdwArgs &a) { return a.tile_h == 8 ? 8 : 16; }

__device__ inline int ceil_div(int v, int d)
{
    return v >= 0 ? (v + d - 1) / d : -((-v) / d);
}

__device__ inline int xcd_tile(int bid, int ntiles)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int q = ntiles >> 3, rem = ntiles & 7;
    return xcd * q + min(xcd, rem) + local;
}

// Weights for p = 1, 2, 3 on the squared lattice distance (the common scale
// cancels in num/den).  The floor only guards an exactly-zero fine offset:
// real offsets are at least one residual unit (2^-15 lattice) away, and the
// largest weight (p = 3 at the floor) stays 2^20 below the hit weight.
__device__ inline float weight_fast(float d2n, int pmode)
{
    d2n = fmaxf(d2n, 0x1p-40f);
    if (pmode == 1)
        return __builtin_amdgcn_rsqf(d2n);
    if (pmode == 2)
        return __builtin_amdgcn_rcpf(d2n);
    const float r = __builtin_amdgcn_rsqf(d2n);
    return r * r * r;
}

// Weight of a non-coincident sounding: its squared distance is at least a
// quarter of a lattice unit squared (the exact offsets differ by at least one
// unit and the residuals by less than one), so no clamp is needed.
__device__ inline float weight_nonhit(float d2n, int pmode)
{
    if (pmode == 1)
        return __builtin_amdgcn_rsqf(d2n);
    if (pmode == 2)
        return __builtin_amdgcn_rcpf(d2n);
    const float r = __builtin_amdgcn_rsqf(d2n);
    return r * r * r;
}

// Sign-extend from 23 bits.  Applied to window offsets known to lie within
// +-2^22 it changes nothing, but it tells the compiler that their
// differences fit 24 bits, so exact 64-bit squares use the full-rate 24-bit
// multiplies.
__device__ inline int sext23(int v) { return (int)((unsigned)v << 9) >> 9; }

__device__ inline float log_weight(float d2n, float power)
{
    return -0.5f * power * __builtin_amdgcn_logf(fmaxf(d2n, 0x1p-120f));
}

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline int wave_sum_i(int v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline int wave_count(bool p) { return __popcll(__ballot(p)); }

// p advanced by `bytes` (a 32-bit offset, so that stores and loads take a
// scalar base with a 32-bit vector offset).
template <class T>
__device__ inline T *byte_at(T *p, uint32_t bytes)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(p) + bytes);
}
template <class T>
__device__ inline const T *byte_at(const T *p, uint32_t bytes)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + bytes);
}

// num / den in FP64 from FP32 sums (den > 0): the hardware reciprocal, one
// Newton step, the quotient and one correction by its residual.
__device__ inline double quotient64(float num, float den)
{
    const double n = (double)num, d = (double)den;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// Non-returning LDS atomics (workgroup scope, relaxed): ds_add_u32,
// ds_min_u64, ds_min_f32, ds_max_f32.  Used where lanes of one instruction
// update distinct words, so nothing serialises.
template <class T>
__device__ inline void lds_add(T *p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ inline void lds_min(T *p, T v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ inline void lds_max(T *p, T v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Best key (D^2, index) and its depth, reduced over the wave.
__device__ inline void wave_best(double &d2, int &idx, float &z)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double od = __shfl_xor(d2, d, 64);
        const int oi = __shfl_xor(idx, d, 64);
        const float oz = __shfl_xor(z, d, 64);
        if (od < d2 || (od == d2 && oi < idx)) {
            d2 = od;
            idx = oi;
            z = oz;
        }
    }
}

struct Seg {
    int by_lo, nrows, bx_lo, nbx_row;
};

// Iterate, wave-wide, over every binned sounding of the bin rows [by_lo,
// by_lo+nrows) and columns [bx_lo, bx_lo+nbx_row): f(k) per lane with k the
// binned position, or k = -1 for idle lanes.  Must be called by the whole wave.
template <class F>
__device__ inline void for_each_candidate(const auv_bin_view &bv, const Seg &sg, F &&f)
{
    const int lane = threadIdx.x & 63;  // lane within the wave (blocks may hold several)
    for (int r = 0; r < sg.nrows; ++r) {
        const int id0 = (sg.by_lo + r) * bv.nbx + sg.bx_lo;
        const int s = bv.cell_start[id0], e = bv.cell_start[id0 + sg.nbx_row];
        for (int k0 = s; k0 < e; k0 += 64) {
            const int k = k0 + lane;
            f(k < e ? k : -1);
        }
    }
}

// Coordinates of a sounding and of a node under the precision variants, in
// metres: AUV_P_FP16_OFFSETS rounds offsets from the tile centre to FP16;
// AUV_P_FP32_ABSOLUTE rounds absolute coordinates to FP32 (no rebase).  The
// sounding's position is rebuilt from its lattice point and residual.
__device__ inline void variant_point(const IdwArgs &a, int X, int Y, float rx, float ry,
                                     int tb0, int ta0, int X0, int Y0, int DXl, int DYl,
                                     int prec, float *px, float *py)
{
    if (prec == AUV_P_FP16_OFFSETS) {
        // tile centre between its nodes 7 and 8 (DX is even)
        const int Xc = X0 + tb0 * DXl + (kTW - 1) * (DXl / 2);
        const int Yc = Y0 + ta0 * DYl + (kTH - 1) * (DYl / 2);
        *px = (float)(_Float16)(((float)(X - Xc) + rx) * 0x1p-16f);
        *py = (float)(_Float16)(((float)(Y - Yc) + ry) * 0x1p-16f);
    } else {
        *px = (float)(a.x0 + ((double)X + (double)rx) * 0x1p-16);
        *py = (float)(a.y0 + ((double)Y + (double)ry) * 0x1p-16);
    }
}

__device__ inline void variant_node(const IdwArgs &a, int bl, int al, int tb0, int ta0,
                                    int prec, float *qx, float *qy)
{
    if (prec == AUV_P_FP16_OFFSETS) {
        *qx = (float)(_Float16)(((float)bl - 0.5f * (kTW - 1)) * (float)a.dx);
        *qy = (float)(_Float16)(((float)al - 0.5f * (kTH - 1)) * (float)a.dy);
    } else {
        *qx = (float)(a.x0 + ((double)(tb0 + bl) + 0.5) * a.dx);
        *qy = (float)(a.y0 + ((double)(ta0 + al) + 0.5) * a.dy);
    }
}

// Distance of binned sounding k from node (na, nb) under precision variant
// kPrec.  Returns the ranking key (exact lattice D^2, or the bit pattern of
// the variant's FP32 squared distance, both order-preserving and held exactly
// in a double) and the squared distance in lattice units for the weight.
template <int kPrec>
__device__ inline double cand_key(const auv_bin_view &bv, const IdwArgs &a, int k, int Xn,
                                  int Yn, int na, int nb, int X0, int Y0, int DXl, int DYl,
                                  float *d2w)
{
    const uint32_t res = bv.res[k];
    const float rx = (float)(int16_t)(res & 0xffffu) * kResidualUnit;
    const float ry = (float)(int16_t)(res >> 16) * kResidualUnit;
    if constexpr (kPrec == AUV_P_FP32_REBASE) {
        const int dX = bv.X[k] - Xn, dY = bv.Y[k] - Yn;
        const float fx = (float)dX + rx, fy = (float)dY + ry;
        *d2w = fx * fx + fy * fy;
        return (double)dX * (double)dX + (double)dY * (double)dY;
    } else {
        float px, py, qx, qy;
        variant_point(a, bv.X[k], bv.Y[k], rx, ry, nb & ~(kTW - 1), na & ~(kTH - 1), X0, Y0,
                      DXl, DYl, kPrec, &px, &py);
        variant_node(a, nb & (kTW - 1), na & (kTH - 1), nb & ~(kTW - 1), na & ~(kTH - 1), kPrec,
                     &qx, &qy);
        const float ex = px - qx, ey = py - qy;
        const float d2 = ex * ex + ey * ey;
        *d2w = d2 * 0x1p32f;
        return (double)__float_as_uint(d2);
    }
}

// Exact value of one over-cap node, computed by the whole wave: find the
// rank-k key (T, J) by bisection over the key and then over the index among
// ties, then accumulate the selected set.  Writes the node's outputs.
template <int kMode, int kPmode, int kPrec>
__device__ void exact_node(const auv_bin_view &bv, const IdwArgs &a, int X0, int Y0,
                           int DXl, int DYl, int na, int nb, float zref)
{
    const int R = a.R_stage;
    const double R2 = kPrec == AUV_P_FP32_REBASE ? (double)a.R * (double)a.R
                                                 : (double)__float_as_uint(a.r2f);
    const int Xn = X0 + nb * DXl, Yn = Y0 + na * DYl;
    const int hB = bv.halo << bv.bin_log2;
    Seg sg;
    sg.bx_lo = max(0, (Xn - R + hB) >> bv.bin_log2);
    sg.nbx_row = min(bv.nbx - 1, (Xn + R + hB) >> bv.bin_log2) - sg.bx_lo + 1;
    sg.by_lo = max(0, (Yn - R + hB) >> bv.bin_log2);
    sg.nrows = min(bv.nby - 1, (Yn + R + hB) >> bv.bin_log2) - sg.by_lo + 1;
    auto key_d2 = [&](int k) {
        float d2w;
        return cand_key<kPrec>(bv, a, k, Xn, Yn, na, nb, X0, Y0, DXl, DYl, &d2w);
    };
    // members only: a key above the radius never counts
    auto member_key = [&](int k) {
        const double kv = key_d2(k);
        return kv <= R2 ? kv : -1.0;
    };
    const int kcap = a.max_pts;
    // accumulate one selected member (per lane, reduced over the wave below)
    float num = 0.0f, den = 0.0f, emax = -INFINITY, zlo = INFINITY, zhi = -INFINITY;
    int cnt = 0, hits = 0;
    double hsum = 0.0, bd2 = 1e300;
    int bidx = INT_MAX;
    float bz = 0.0f;
    auto take = [&](int k, double d2, float d2f, int ci) {
        const float z = bv.z[k];
        cnt += 1;
        zlo = fminf(zlo, z);
        zhi = fmaxf(zhi, z);
        if (d2 < bd2 || (d2 == bd2 && ci < bidx)) {
            bd2 = d2;
            bidx = ci;
            bz = z;
        }
        if constexpr ((kMode & 1) != 0) {
            if (d2 == 0.0) {
                hits += 1;
                hsum += (double)z;
            }
            if constexpr (kPmode != 0) {
                const float w = weight_fast(d2f, kPmode > 0 ? kPmode : a.pmode);
                num += w * (z - zref);
                den += w;
            } else {
                const float e = log_weight(d2f * a.inv_r2, a.power);
                if (e > emax) {
                    const float sc = __builtin_amdgcn_exp2f(emax - e);
                    num *= sc;
                    den *= sc;
                    emax = e;
                }
                const float w = __builtin_amdgcn_exp2f(e - emax);
                num += w * (z - zref);
                den += w;
            }
        }
    };
    // Fast path (exact lattice keys): gather the node's members once into
    // registers, up to kHold per lane, as unique packed keys (D^2 << b | index);
    // find the cap-th smallest key by bisection over the held keys (no memory
    // traffic), then take the members at or below it.
    constexpr int kHold = 4;
    bool done = false;
    if constexpr (kPrec == AUV_P_FP32_REBASE) {
        const int kb = bv.idx_bits;
        const long long R2i = (long long)a.R * a.R;
        if ((unsigned long long)R2i < (1ull << (63 - kb))) {
            unsigned long long mk[kHold];
            int mpos[kHold];
#pragma unroll
            for (int j = 0; j < kHold; ++j) {
                mk[j] = ~0ull;
                mpos[j] = -1;
            }
            int held = 0;
            bool over = false;
            for_each_candidate(bv, sg, [&](int k) {
                if (k < 0)
                    return;
                const long long dX = bv.X[k] - Xn, dY = bv.Y[k] - Yn;
                const long long D2 = dX * dX + dY * dY;
                if (D2 > R2i)
                    return;
                const unsigned long long key = ((unsigned long long)D2 << kb) | (unsigned)bv.idx[k];
#pragma unroll
                for (int j = 0; j < kHold; ++j)
                    if (held == j) {
                        mk[j] = key;
                        mpos[j] = k;
                    }
                over |= held >= kHold;
                held += 1;
            });
            if (!__ballot(over)) {
                unsigned long long lo = 0ull, hi = 0ull;
#pragma unroll
                for (int j = 0; j < kHold; ++j)
                    hi = mpos[j] >= 0 && mk[j] > hi ? mk[j] : hi;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const unsigned long long o = __shfl_xor(hi, d, 64);
                    hi = o > hi ? o : hi;
                }
                // smallest key with at least kcap members at or below it
                while (lo < hi) {
                    const unsigned long long mid = lo + ((hi - lo) >> 1);
                    int c = 0;
#pragma unroll
                    for (int j = 0; j < kHold; ++j)
                        c += mpos[j] >= 0 && mk[j] <= mid ? 1 : 0;
                    if (wave_sum_i(c) >= kcap)
                        hi = mid;
                    else
                        lo = mid + 1ull;
                }
#pragma unroll
                for (int j = 0; j < kHold; ++j) {
                    if (mpos[j] >= 0 && mk[j] <= lo) {
                        float d2f;
                        const double d2 = cand_key<kPrec>(bv, a, mpos[j], Xn, Yn, na, nb, X0, Y0,
                                                          DXl, DYl, &d2f);
                        take(mpos[j], d2, d2f, (int)(mk[j] & ((1ull << kb) - 1ull)));
                    }
                }
                done = true;
            }
        }
    }
    if (!done) {
        // general path: smallest T in [0, R2] with #{D^2 <= T} >= k
        double lo = 0.0, hi = R2;
        while (lo < hi) {
            const double mid = floor((lo + hi) * 0.5);
            int c = 0;
            for_each_candidate(bv, sg, [&](int k) {
                const double kv = k >= 0 ? member_key(k) : -1.0;
                c += wave_count(kv >= 0.0 && kv <= mid);
            });
            if (c >= kcap)
                hi = mid;
            else
                lo = mid + 1.0;
        }
        const double T = lo;
        int clt = 0, ceq = 0;
        for_each_candidate(bv, sg, [&](int k) {
            const double d2 = k >= 0 ? member_key(k) : -1.0;
            clt += wave_count(d2 >= 0.0 && d2 < T);
            ceq += wave_count(d2 >= 0.0 && d2 == T);
        });
        const int need = kcap - clt;
        long long J = INT_MAX;
        if (ceq > need) {
            long long jlo = 0, jhi = INT_MAX;
            while (jlo < jhi) {
                const long long mid = (jlo + jhi) >> 1;
                int c = 0;
                for_each_candidate(bv, sg, [&](int k) {
                    c += wave_count(k >= 0 && member_key(k) == T && bv.idx[k] <= mid);
                });
                if (c >= need)
                    jhi = mid;
                else
                    jlo = mid + 1;
            }
            J = jlo;
        }
        for_each_candidate(bv, sg, [&](int k) {
            if (k < 0)
                return;
            float d2f;
            const double d2 = cand_key<kPrec>(bv, a, k, Xn, Yn, na, nb, X0, Y0, DXl, DYl, &d2f);
            const int ci = bv.idx[k];
            if (!(d2 <= R2) || !(d2 < T || (d2 == T && ci <= J)))
                return;
            take(k, d2, d2f, ci);
        });
    }
    cnt = wave_sum_i(cnt);
    wave_best(bd2, bidx, bz);
    const int64_t o = (int64_t)na * a.nx + nb;
    if constexpr ((kMode & 1) != 0) {
        hits = wave_sum_i(hits);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1)
            hsum += __shfl_xor(hsum, d, 64);
        if constexpr (kPmode == 0) {
            float em = emax;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1)
                em = fmaxf(em, __shfl_xor(em, d, 64));
            const float sc = emax == -INFINITY ? 0.0f : __builtin_amdgcn_exp2f(emax - em);
            num *= sc;
            den *= sc;
        }
        num = wave_sum(num);
        den = wave_sum(den);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            zlo = fminf(zlo, __shfl_xor(zlo, d, 64));
            zhi = fmaxf(zhi, __shfl_xor(zhi, d, 64));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        if (kMode & 2) {
            if (a.nn_idx_out)
                a.nn_idx_out[o] = bidx;
            if (a.nn_z_out)
                a.nn_z_out[o] = bz;
        }
        if constexpr ((kMode & 1) != 0) {
            if (a.cnt_out)
                a.cnt_out[o] = cnt;
            float v;
            if (hits > 0)
                v = (float)(hsum / (double)hits);
            else if (cnt < a.min_pts)
                v = NAN;
            else
                v = (float)fmin(fmax((double)zref + (double)num / (double)den, (double)zlo),
                                (double)zhi);
            a.z_out[o] = v;
        }
    }
}

// LDS accumulators are structure-of-arrays, one row of the tile after the
// other.  Unpadded: a padded stride (18) spreads a sounding's 7-row window
// over more banks, but its 896 more bytes per wave held a CU to 15 waves
// instead of 16 (at the 2M-sounding swath 235 us padded, 216 us unpadded;
// a stride of 17, also 16 waves, 222 us).
constexpr int kRS = kTW;
constexpr int kAcc = kTH * kRS;

// kChunks = window cells / 64 rounded up (compile-time, so the visit loop has
// no per-chunk branches).  A 64-wide batch of candidates is tested
// lane-parallel; the kept ones are compacted into a small LDS record array
// and visited one by one: the window offsets come by readlane (scalar
// registers, where their range is known to the compiler), the rest by
// broadcast LDS reads, which keeps the vector ALU for the per-cell work.
// int4 slots of the kept-sounding records: 64 records of two, and one more
// record that the visit loop's unconditional read-ahead may touch.
constexpr int kRecSlots = 2 * 64 + 2;

// Shared arrays of one window tile (pointers into the caller's LDS).
struct WinSmem {
    float2 *nd;                 // numerator, denominator        [kAcc]
    int *cnt;                   // members                       [kAcc]
    float *lo, *hi;             // smallest, largest member depth [kAcc] each
    unsigned long long *key;    // packed (D^2 << b) | index     [kAcc] (packed)
    double *bd2;                // best D^2                      [kAcc] (unpacked)
    int *bidx;                  // best index                    [kAcc] (unpacked)
    float *bz;                  // best depth                    [kAcc] (unpacked)
    float *emax;                // running log2 weight max       [kAcc] (general p)
    int *beg, *off;             // staging rows                  [kMaxRows(+1)]
    int4 *r0;                   // kept soundings: ia, jb (exact form: depth bits), 8 qb, 4 qb
                                //                                             [64, stride 2]
    int4 *r1;                   //   residual x, y, depth - zref (bits), index  [64, stride 2]
                                // (r1 = r0 + 1: a record's halves are adjacent, so both
                                //  reads of a visit share one LDS address)
    float4 *rv;                 //   variant coordinates, depth   [64] (variants, unpacked)
};

// Where a caller collects a tile's nodes above the cap for a later pass of
// its own (one lane per node) instead of the tile re-doing them one at a
// time: entries (item, row, column, 0) appended at list[*count] while below cap.
struct CapSink {
    int32_t *count = nullptr;  // null: no sink
    int4 *list = nullptr;
    int32_t cap = 0;
    int32_t item = 0;
};

// part / nparts: the wave takes every nparts-th 64-wide chunk of the tile's
// candidates, starting at chunk `part` (several waves can share one tile).
// In accumulate mode with nparts > 1 the wave leaves its partial sums in LDS
// and its reference depth in *zref_out; the caller combines the parts.
template <int kMode, int kPmode, bool kPacked, int kChunks, int kPrec>
__device__ void window_tile(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g,
                            int tile, int ntx, const WinSmem &sm, int part = 0,
                            int nparts = 1, float *zref_out = nullptr,
                            CapSink sink = CapSink{})
{
    constexpr bool kIdw = (kMode & 1) != 0;
    // the nearest key serves the nearest outputs, hits and the cap; the
    // accumulate mode (no cap) recognises hits by their weight instead
    constexpr bool kKey = kPacked && (kMode & 4) == 0;
    // Accumulators are updated by plain LDS read-modify-write: within one
    // instruction every lane owns a distinct node, and a wave's LDS operations
    // complete in order, so no atomics are needed (LDS atomics would serialise
    // per lane).
    float2 *const s_nd = sm.nd;
    int *const s_cnt = sm.cnt;
    float *const s_lo = sm.lo;
    float *const s_hi = sm.hi;
    unsigned long long *const s_key = sm.key;
    double *const s_bd2 = sm.bd2;
    int *const s_bidx = sm.bidx;
    float *const s_bz = sm.bz;
    float *const s_emax = sm.emax;
    int *const s_beg = sm.beg;
    int *const s_off = sm.off;

    const int lane = threadIdx.x & 63;  // lane within the wave (blocks may hold several)
    // tile rows: 16 or 8 (the FP16-offset variant measures offsets from the
    // centre of a 16 x 16 tile, so the variants keep 16)
    const int TH = kPrec == AUV_P_FP32_REBASE ? tile_rows(a) : kTH;
    const int tx = tile % ntx, ty = tile / ntx;
    const int tb0 = tx * kTW, ta0 = ty * TH;
    const int tw = min(kTW, a.nx - tb0), th = min(TH, a.ny - ta0);
    const int Xt0 = g.X0 + tb0 * g.DXl, Yt0 = g.Y0 + ta0 * g.DYl;
    const int R = a.R_stage;          // staging reach (>= the radius)
    const long long R2 = (long long)a.R * a.R;
    const int kb = bv.idx_bits;
    constexpr bool kExact = kPrec == AUV_P_FP32_REBASE;

    // this lane's window cell in each chunk
    int ci[kChunks], cj[kChunks], iD[kChunks], jD[kChunks], qo[kChunks];
    // exact form: (row, column) of the cell as two 16-bit halves; the cell of
    // a record's window lies in the tile when both halves of cell + window
    // origin are in [0, 16) -- one packed add and one mask test.  Edge tiles
    // are treated as whole 16 x 16 tiles: nodes past the grid edge collect
    // sums that are never read (finalisation covers in-grid nodes only).
    static_assert(kTW == 16 && kTH == 16, "the packed tile test assumes 16-wide tiles of "
                                          "at most 16 rows");
    // row half: [0, TH) with TH = 16 or 8; column half: [0, 16)
    const uint32_t tmask = TH == 16 ? 0xfff0fff0u : 0xfff8fff0u;
    uint32_t pc[kChunks];
    // c / Wx for c < 256 by a float product: (c + 1/2) / Wx stays at least
    // 1/512 from an integer, far beyond the reciprocal's rounding
    const float invWx = __builtin_amdgcn_rcpf((float)g.Wx);
#pragma unroll
    for (int t = 0; t < kChunks; ++t) {
        const int c = t * 64 + lane;
        const bool v = c < g.ncells;
        const int cq = (int)(((float)c + 0.5f) * invWx);
        // an unused lane gets a cell far outside any tile
        ci[t] = v ? cq : -100000;
        cj[t] = v ? c - cq * g.Wx : -100000;
        iD[t] = sext23(v ? ci[t] * g.DYl : 0);
        jD[t] = sext23(v ? cj[t] * g.DXl : 0);
        qo[t] = v ? ci[t] * kRS + cj[t] : 0;
        pc[t] = v ? ((uint32_t)ci[t] << 16) | (uint32_t)cj[t] : 0x40004000u;
    }


    // accumulators cleared once the tile is known to have candidates
    auto clear_acc = [&]() {
        __syncthreads();  // the previous tile of this wave is finished with LDS
        for (int q = lane; q < TH * kRS; q += 64) {
            s_nd[q] = make_float2(0.0f, 0.0f);
            s_cnt[q] = 0;
            s_lo[q] = INFINITY;
            s_hi[q] = -INFINITY;
            if constexpr (kPacked) {
                if constexpr (kKey)
                    s_key[q] = ~0ull;
            } else {
                s_bd2[q] = 1e300;
                s_bidx[q] = INT_MAX;
                s_bz[q] = 0.0f;
            }
            if constexpr (kPmode == 0)
                s_emax[q] = -INFINITY;
        }
        __syncthreads();
    };

    // bins covering the tile grown by R
    const int hB = bv.halo << bv.bin_log2;
    const int s = bv.bin_log2;
    const int bx_lo = max(0, (Xt0 - R + hB) >> s);
    const int nbx_row = min(bv.nbx - 1, (Xt0 + (tw - 1) * g.DXl + R + hB) >> s) - bx_lo + 1;
    const int by_lo = max(0, (Yt0 - R + hB) >> s);
    const int nrows = min(bv.nby - 1, (Yt0 + (th - 1) * g.DYl + R + hB) >> s) - by_lo + 1;
    // estimates only (the window origin is corrected exactly in integers)
    const float invDX = __builtin_amdgcn_rcpf((float)g.DXl),
                invDY = __builtin_amdgcn_rcpf((float)g.DYl);
    // squared staging reach, widened by 2^-20 against the FP32 rounding of
    // the squared distances it is compared with
    const float reach2 = (float)R * (float)R * (1.0f + 0x1p-20f);

    float zref = 0.0f;
    bool have_ref = false;

    if (nrows <= 0)
        clear_acc();
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
        if (r0 == 0) {
            if constexpr ((kMode & 4) == 0) {
                if (total == 0 && nrows <= kMaxRows) {
                    // no sounding can reach the tile: its outputs are empty
                    const size_t tbase = (size_t)ta0 * a.nx + tb0;
                    for (int q0 = 0; q0 < kTW * TH; q0 += 64) {
                        const int qq = q0 + lane;
                        const int la = qq / kTW, lb = qq - la * kTW;
                        if (la < th && lb < tw) {
                            const uint32_t ob = (uint32_t)(la * a.nx + lb) << 2;
                            if (kMode & 2) {
                                if (a.nn_idx_out)
                                    *byte_at(a.nn_idx_out + tbase, ob) = -1;
                                if (a.nn_z_out)
                                    *byte_at(a.nn_z_out + tbase, ob) = NAN;
                            }
                            if constexpr (kIdw) {
                                if (a.cnt_out)
                                    *byte_at(a.cnt_out + tbase, ob) = 0;
                                *byte_at(a.z_out + tbase, ob) = NAN;
                            }
                        }
                    }
                    return;
                }
            }
            clear_acc();
        }
        __syncthreads();
        if (lane < nr) {
            s_beg[lane] = beg;
            s_off[lane] = inc - len;
        }
        if (lane == 0)
            s_off[nr] = total;
        __syncthreads();
        for (int c0 = part * 64; c0 < total; c0 += nparts * 64) {
            const int gi = c0 + lane;
            bool keep = false;
            int px = 0, py = 0, pia = 0, pjb = 0, pidx = 0;
            float prx = 0.0f, pry = 0.0f, pz = 0.0f, pvx = 0.0f, pvy = 0.0f;
            if (gi < total) {
                int lo = 0, hi = nr - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= gi)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const int k = s_beg[lo] + (gi - s_off[lo]);
                const int xr = bv.X[k] - Xt0, yr = bv.Y[k] - Yt0;
                // first window column / row: ceil((xr - R) / DX), from a
                // float estimate corrected exactly in integers
                int jb = (int)ceilf((float)(xr - R) * invDX);
                jb += (jb - 1) * g.DXl >= xr - R ? -1 : 0;
                jb += jb * g.DXl < xr - R ? 1 : 0;
                int ia = (int)ceilf((float)(yr - R) * invDY);
                ia += (ia - 1) * g.DYl >= yr - R ? -1 : 0;
                ia += ia * g.DYl < yr - R ? 1 : 0;
                keep = jb <= tw - 1 && jb + g.Wx - 1 >= 0 && ia <= th - 1 && ia + g.Wy - 1 >= 0;
                // and the disk must meet the box of the tile's in-grid nodes
                // (a window can meet the tile with corner cells only): FP32
                // distance to the box against the staging reach with a margin
                // above the rounding, so no sounding that can reach a node is
                // dropped (about one visit in ten goes)
                const float ex = (float)max(max(-xr, xr - (tw - 1) * g.DXl), 0);
                const float ey = (float)max(max(-yr, yr - (th - 1) * g.DYl), 0);
                keep = keep && fmaf(ex, ex, ey * ey) <= reach2;
                const uint32_t res = bv.res[k];
                px = xr - jb * g.DXl;
                py = yr - ia * g.DYl;
                prx = (float)(int16_t)(res & 0xffffu) * kResidualUnit;
                pry = (float)(int16_t)(res >> 16) * kResidualUnit;
                pz = bv.z[k];
                pidx = bv.idx[k];
                if constexpr (!kExact)
                    variant_point(a, bv.X[k], bv.Y[k], prx, pry, tb0, ta0, g.X0, g.Y0, g.DXl,
                                  g.DYl, kPrec, &pvx, &pvy);
                pia = ia;
                pjb = jb;
            }
            unsigned long long m = __ballot(keep);
            if (m == 0ull)
                continue;
            if (!have_ref) {
                // the depth of the first kept sounding is the tile's reference
                zref = __shfl(pz, __ffsll((long long)m) - 1, 64);
                have_ref = true;
            }
            const float pdz = pz - zref;
            if (keep) {
                const int slot = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                const int qb = pia * kRS + pjb;
                // exact form: window origin as packed 16-bit (row, column)
                const int o0 = kExact ? (int)((((uint32_t)pia & 0xffffu) << 16) |
                                              ((uint32_t)pjb & 0xffffu))
                                      : pia;
                sm.r0[2 * slot] = make_int4(o0, kExact && kPacked ? __float_as_int(pz) : pjb,
                                            qb * 8, qb * 4);
                sm.r1[2 * slot] = make_int4(__float_as_int(prx), __float_as_int(pry),
                                        __float_as_int(pdz), pidx);
                if constexpr (!kExact || !kPacked)
                    sm.rv[slot] = make_float4(pvx, pvy, pz, 0.0f);
            }
            // the records are read back by the same wave, in order
            __builtin_amdgcn_wave_barrier();
            // the record address lives in a VGPR (LDS reads take one) and
            // both halves are read from it with an immediate offset
            typedef int v4i __attribute__((ext_vector_type(4)));
            typedef __attribute__((address_space(3))) const v4i lds_v4i;
            lds_v4i *rp0 = (lds_v4i *)sm.r0;
            asm volatile("" : "+v"(rp0));
            const float4 *rpv = sm.rv;
            // Visit of the kept sounding in lane l, whose record is (v0, v1).
            auto visit = [&](int l, const v4i &v0, const v4i &v1) {
                const int sx = sext23(__builtin_amdgcn_readlane(px, l));
                const int sy = sext23(__builtin_amdgcn_readlane(py, l));
                const int4 w0 = make_int4(v0.x, v0.y, v0.z, v0.w);
                const int4 w1 = make_int4(v1.x, v1.y, v1.z, v1.w);
                const int ia = w0.x, jb = w0.y, qb8 = w0.z, qb4 = w0.w;
                const float srx = __int_as_float(w1.x), sry = __int_as_float(w1.y);
                const float sdz = __int_as_float(w1.z);
                const int sidx = w1.w;
                float svx = 0.0f, svy = 0.0f, spz;
                if constexpr (!kExact || !kPacked) {
                    const float4 v = *rpv;
                    svx = v.x;
                    svy = v.y;
                    spz = v.z;
                } else {
                    spz = __int_as_float(w0.y);  // the depth itself (exact form)
                }
                ++rpv;
                const int qb = qb4 >> 2;
#pragma unroll
                for (int t = 0; t < kChunks; ++t) {
                    bool in;
                    if constexpr (kExact) {
                        typedef unsigned short us2 __attribute__((ext_vector_type(2)));
                        const us2 sum = __builtin_bit_cast(us2, pc[t]) +
                                        __builtin_bit_cast(us2, (uint32_t)ia);
                        in = (__builtin_bit_cast(uint32_t, sum) & tmask) == 0u;
                    } else {
                        in = (unsigned)(ia + ci[t]) < (unsigned)th &&
                             (unsigned)(jb + cj[t]) < (unsigned)tw;
                    }
                    const int dX = sx - jD[t], dY = sy - iD[t];
                    // ranking key and member test: exact lattice D^2, or the
                    // variant's FP32 squared distance (bit pattern)
                    long long D2;
                    float d2f;
                    bool mem;
                    if constexpr (kExact) {
                        D2 = (long long)dX * dX + (long long)dY * dY;  // exact
                        mem = in && D2 <= R2;
                        const float fx = (float)dX + srx, fy = (float)dY + sry;
                        d2f = fx * fx + fy * fy;
                    } else {
                        float qx, qy;
                        variant_node(a, jb + cj[t], ia + ci[t], tb0, ta0, kPrec, &qx, &qy);
                        const float ex = svx - qx, ey = svy - qy;
                        const float dv = ex * ex + ey * ey;
                        D2 = (long long)__float_as_uint(dv);
                        mem = in && dv <= a.r2f;
                        d2f = dv * 0x1p32f;
                    }
                    if constexpr (kExact && kKey && kIdw && kPmode != 0) {
                        // The weight, key and addresses for every lane (a masked
                        // VALU instruction costs the same issue slot), so that
                        // the masked block below holds the LDS updates only and
                        // the record's fields are read before it: their wait no
                        // longer sits inside the block, where it had to cover
                        // every LDS operation issued before (the compiler keeps
                        // the jump over a block with LDS operations, so it
                        // counts outstanding operations for the shortest path).
                        const int q8 = qb8 + qo[t] * 8;
                        const int q4 = qb4 + qo[t] * 4;
                        const float w = D2 == 0 ? kHitW
                                                : weight_nonhit(d2f, kPmode > 0 ? kPmode : a.pmode);
                        const unsigned long long key =
                            ((unsigned long long)D2 << kb) | (unsigned)sidx;
                        asm volatile("" ::"v"(w), "v"(key), "v"(q8), "v"(q4));
                        if (mem) {
                            float2 *const pn =
                                reinterpret_cast<float2 *>(reinterpret_cast<char *>(s_nd) + q8);
                            float2 nd = *pn;
                            lds_min(reinterpret_cast<unsigned long long *>(
                                        reinterpret_cast<char *>(s_key) + q8),
                                    key);
                            lds_add(reinterpret_cast<int *>(reinterpret_cast<char *>(s_cnt) + q4), 1);
                            lds_min(reinterpret_cast<float *>(reinterpret_cast<char *>(s_lo) + q4), spz);
                            lds_max(reinterpret_cast<float *>(reinterpret_cast<char *>(s_hi) + q4), spz);
                            nd.x = fmaf(w, sdz, nd.x);
                            nd.y += w;
                            *pn = nd;
                        }
                    } else if (mem) {
                        const int q = qb + qo[t];
                        const int q8 = qb8 + qo[t] * 8;
                        const int q4 = qb4 + qo[t] * 4;
                        int *const pc = reinterpret_cast<int *>(reinterpret_cast<char *>(s_cnt) + q4);
                        float *const pl = reinterpret_cast<float *>(reinterpret_cast<char *>(s_lo) + q4);
                        float *const ph = reinterpret_cast<float *>(reinterpret_cast<char *>(s_hi) + q4);
                        float2 *const pn =
                            reinterpret_cast<float2 *>(reinterpret_cast<char *>(s_nd) + q8);
                        float2 nd = make_float2(0.0f, 0.0f);
                        float em = 0.0f;
                        if constexpr (kIdw) {
                            nd = *pn;
                            if constexpr (kPmode == 0)
                                em = s_emax[q];
                        }
                        float w = 0.0f;
                        if constexpr (kIdw) {
                            if constexpr (kPmode != 0)
                                w = D2 == 0 ? kHitW
                                            : weight_nonhit(d2f, kPmode > 0 ? kPmode : a.pmode);
                            else
                                w = D2 == 0 ? 1e30f : log_weight(d2f * a.inv_r2, a.power);
                        }
                        // count, nearest key and depth range: non-returning LDS
                        // atomics (no read back; lanes of one instruction hit
                        // distinct nodes, and a wave's LDS operations execute
                        // in program order, so the result is deterministic)
                        if constexpr (kKey) {
                            const unsigned long long key =
                                ((unsigned long long)D2 << kb) | (unsigned)sidx;
                            lds_min(reinterpret_cast<unsigned long long *>(
                                        reinterpret_cast<char *>(s_key) + q8),
                                    key);
                        } else if constexpr (!kPacked) {
                            const double d2 = (double)D2, bd = s_bd2[q];
                            if (d2 < bd || (d2 == bd && sidx < s_bidx[q])) {
                                s_bd2[q] = d2;
                                s_bidx[q] = sidx;
                                s_bz[q] = spz;
                            }
                        }
                        lds_add(pc, 1);
                        lds_min(pl, spz);
                        lds_max(ph, spz);
                        if constexpr (kIdw) {
                            if constexpr (kPmode != 0) {
                                nd.x += w * sdz;
                                nd.y += w;
                            } else {
                                // w holds the log2 weight; rescale to the running max
                                if (w > em) {
                                    const float sc = __builtin_amdgcn_exp2f(em - w);
                                    nd.x *= sc;
                                    nd.y *= sc;
                                    em = w;
                                    s_emax[q] = em;
                                }
                                const float lw = __builtin_amdgcn_exp2f(w - em);
                                nd.x += lw * sdz;
                                nd.y += lw;
                            }
                            *pn = nd;
                        }
                    }
                }
            };
            // The next record is read while the current one is applied (two
            // register sets, so the prefetch needs no copies); the records
            // were written before the wave barrier above.  The read-ahead is
            // unconditional (past the last record it reads the spare slot and
            // the value goes unused): issued on every path, it lets the
            // compiler wait for a record's own reads instead of for every LDS
            // operation before them.
            v4i a0 = rp0[0], a1 = rp0[1], b0, b1;
            while (m) {
                int l = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                b0 = rp0[2];
                b1 = rp0[3];
                visit(l, a0, a1);
                rp0 += 2;
                if (!m)
                    break;
                l = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                a0 = rp0[2];
                a1 = rp0[3];
                visit(l, b0, b1);
                rp0 += 2;
            }
        }
    }
    __syncthreads();
    if constexpr ((kMode & 4) != 0) {
        if (nparts > 1) {
            *zref_out = zref;  // partial sums stay in LDS for the caller
            return;
        }
    }

    // finalize: one node per lane, four passes over the tile
    const int kcap = a.max_pts;
    const unsigned long long imask = (1ull << kb) - 1ull;
    if constexpr ((kMode & 4) != 0) {
        for (int q0 = 0; q0 < kTW * TH; q0 += 64) {
            const int qq = q0 + lane;
            const int la = qq / kTW, lb = qq - la * kTW;
            const int q = la * kRS + lb;
            const bool act = la < th && lb < tw;
            const int cnt = s_cnt[q];
            // accumulate mode (no cap): add this tile's sums into the resident
            // per-node accumulators, re-referenced from the tile's depth to
            // the accumulators' depth.  One lane owns each node; the caller
            // guarantees that no other wave updates the same node meanwhile.
            if (act && cnt > 0) {
                const int64_t o = (int64_t)(ta0 + la) * a.nx + tb0 + lb;
                const float2 nd = s_nd[q];
                const double shift = (double)zref - a.zref_acc;
                const float lo = s_lo[q], hi = s_hi[q];
                const int c0 = a.acc_cnt[o];
                a.acc_num[o] += (float)((double)nd.x + (double)nd.y * shift);
                a.acc_den[o] += nd.y;
                a.acc_cnt[o] = c0 + cnt;
                a.acc_lo[o] = c0 > 0 ? fminf(a.acc_lo[o], lo) : lo;
                a.acc_hi[o] = c0 > 0 ? fmaxf(a.acc_hi[o], hi) : hi;
            }
        }
    } else {
        // outputs: the tile's first node as a scalar base, 32-bit byte
        // offsets per lane (rows of the tile lie within 2^30 nodes of it).
        // The nearest depth gathered in one pass is stored in the next, so
        // the gather overlaps a pass of work (the passes are unrolled: in a
        // loop, carrying the gathered value to the next iteration made the
        // compiler wait for it at the end of its own pass).
        constexpr int kPass = kTW * kTH / 64;
        const size_t tbase = (size_t)ta0 * a.nx + tb0;
        unsigned overm = 0u;  // bit p: this lane's node of pass p is over the cap
        float bz_prev = NAN;
        uint32_t ob_prev = 0;
        bool st_prev = false;
#pragma unroll
        for (int p = 0; p < kPass; ++p) {
            const int qq = p * 64 + lane;
            const int la = qq / kTW, lb = qq - la * kTW;
            const int q = la * kRS + lb;
            const bool act = p * 64 < kTW * TH && la < th && lb < tw;
            const int cnt = s_cnt[q];
            // the node's sums and bounds read with its count and key, one
            // wait for all (the reads are in bounds for every lane)
            const float2 ndv = s_nd[q];
            const float lov = s_lo[q], hiv = s_hi[q];
            int bi;
            bool hit;
            if constexpr (kKey) {
                const unsigned long long key = s_key[q];
                asm volatile("" ::"v"(cnt), "v"(key), "v"(ndv.x), "v"(ndv.y), "v"(lov), "v"(hiv));
                bi = (int)(key & imask);
                hit = (key >> kb) == 0ull;
            } else if constexpr (kPacked) {
                bi = 0;
                hit = false;
            } else {
                bi = s_bidx[q];
                hit = s_bd2[q] == 0.0;
            }
            const bool over = act && kcap > 0 && cnt > kcap;
            overm |= over ? 1u << p : 0u;
            const uint32_t ob = (uint32_t)(la * a.nx + lb) << 2;
            float bz = NAN;
            if (act && !over) {
                if (kMode & 2) {
                    if (a.nn_idx_out)
                        *byte_at(a.nn_idx_out + tbase, ob) = cnt > 0 ? bi : -1;
                    if (a.nn_z_out && cnt > 0) {
                        if constexpr (kPacked)
                            bz = __int_as_float(byte_at(bv.rec, (uint32_t)bi << 4)->w);
                        else
                            bz = s_bz[q];
                    }
                }
                if constexpr (kIdw) {
                    if (a.cnt_out)
                        *byte_at(a.cnt_out + tbase, ob) = cnt;
                    // a hit (best D^2 == 0) carries a dominant weight, so the
                    // ratio is the mean of the hits, and it beats min_pts
                    const bool hole = cnt == 0 || (cnt < a.min_pts && !hit);
                    const float2 nd = ndv;
                    // the quotient num / den and the return to absolute depth
                    // in FP64 (the hardware reciprocal refined by a Newton
                    // step, then one residual correction of the quotient),
                    // rounded once to FP32 and clamped to the members' depths
                    // (FP32 values, and rounding is monotonic, so this equals
                    // clamping before the rounding)
                    const float v = (float)((double)zref + quotient64(nd.x, nd.y));
                    *byte_at(a.z_out + tbase, ob) = hole ? NAN : fminf(fmaxf(v, lov), hiv);
                }
            }
            if (kMode & 2) {
                if (a.nn_z_out && st_prev)
                    *byte_at(a.nn_z_out + tbase, ob_prev) = bz_prev;
            }
            bz_prev = bz;
            ob_prev = ob;
            st_prev = act && !over;
        }
        if (kMode & 2) {
            if (a.nn_z_out && st_prev)
                *byte_at(a.nn_z_out + tbase, ob_prev) = bz_prev;
        }
        // nodes above the cap: handed to the caller's sink while it has room
        if (sink.count) {
#pragma unroll 1
            for (int p = 0; p < kPass; ++p) {
                const bool mine = (overm >> p) & 1u;
                const unsigned long long m = __ballot(mine);
                if (m == 0ull)
                    continue;
                int base = 0;
                if (lane == 0)
                    base = atomicAdd(sink.count, __popcll(m));
                base = __shfl(base, 0, 64);
                const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                if (mine && slot < sink.cap) {
                    const int qn = p * 64 + lane;
                    sink.list[slot] = make_int4(sink.item, ta0 + qn / kTW, tb0 + qn % kTW, 0);
                    overm &= ~(1u << p);
                }
            }
        }
        // the others: re-done exactly by the whole wave
#pragma unroll 1
        for (int p = 0; p < kPass; ++p) {
            unsigned long long om = __ballot((overm >> p) & 1u);
            while (om) {
                const int l = __ffsll((long long)om) - 1;
                om &= om - 1;
                const int qn = p * 64 + l;
                exact_node<kMode, kPmode, kPrec>(bv, a, g.X0, g.Y0, g.DXl, g.DYl, ta0 + qn / kTW,
                                                 tb0 + qn % kTW, zref);
            }
        }
    }
}


template <int kMode, int kPmode, bool kPacked, int kChunks, int kPrec>
__global__ __launch_bounds__(64) void k_idw_window(auv_bin_view bv, IdwArgs a, WinGeom g,
                                                    int ntx, int nty)
{
    __shared__ float2 s_nd[kAcc];
    __shared__ int s_cnt[kAcc];
    __shared__ float s_lo[kAcc];
    __shared__ float s_hi[kAcc];
    __shared__ unsigned long long s_key[kPacked ? kAcc : 1];
    __shared__ double s_bd2[kPacked ? 1 : kAcc];
    __shared__ int s_bidx[kPacked ? 1 : kAcc];
    __shared__ float s_bz[kPacked ? 1 : kAcc];
    __shared__ float s_emax[kPmode == 0 ? kAcc : 1];
    __shared__ int s_beg[kMaxRows];
    __shared__ int s_off[kMaxRows + 1];
    __shared__ int4 s_rec[kRecSlots];
    __shared__ float4 s_rv[kPrec == AUV_P_FP32_REBASE && kPacked ? 1 : 64];
    const WinSmem sm{s_nd, s_cnt, s_lo, s_hi, s_key, s_bd2, s_bidx, s_bz, s_emax, s_beg, s_off,
                     s_rec, s_rec + 1, s_rv};
    window_tile<kMode, kPmode, kPacked, kChunks, kPrec>(
        bv, a, g, xcd_tile(blockIdx.x, ntx * nty), ntx, sm);
}

template <int kMode, bool kPacked, int kChunks, int kPrec>
void launch_chunks(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int ntx,
                   int nty, int pmode, hipStream_t st)
{
    const dim3 grid((unsigned)(ntx * nty)), block(64);
    switch (pmode) {
    case 1: k_idw_window<kMode, 1, kPacked, kChunks, kPrec><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    case 2: k_idw_window<kMode, 2, kPacked, kChunks, kPrec><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    case 3: k_idw_window<kMode, 3, kPacked, kChunks, kPrec><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    default: k_idw_window<kMode, 0, kPacked, kChunks, kPrec><<<grid, block, 0, st>>>(bv, a, g, ntx, nty); break;
    }
}

template <int kMode, bool kPacked, int kPrec>
void launch_mode(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int ntx,
                 int nty, int pmode, hipStream_t st)
{
    switch (g.nchunks) {
    case 1: launch_chunks<kMode, kPacked, 1, kPrec>(bv, a, g, ntx, nty, pmode, st); break;
    case 2: launch_chunks<kMode, kPacked, 2, kPrec>(bv, a, g, ntx, nty, pmode, st); break;
    case 3: launch_chunks<kMode, kPacked, 3, kPrec>(bv, a, g, ntx, nty, pmode, st); break;
    default: launch_chunks<kMode, kPacked, 4, kPrec>(bv, a, g, ntx, nty, pmode, st); break;
    }
}

template <int kMode, int kPrec>
void launch_mode(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g, int ntx,
                 int nty, int pmode, hipStream_t st)
{
    // the (D^2, index) key fits 64 bits when R^2 * 2^idx_bits < 2^64
    const unsigned __int128 top = (unsigned __int128)((unsigned long long)a.R * a.R)
                                  << bv.idx_bits;
    if (top < ((unsigned __int128)1 << 64))
        launch_mode<kMode, true, kPrec>(bv, a, g, ntx, nty, pmode, st);
    else
        launch_mode<kMode, false, kPrec>(bv, a, g, ntx, nty, pmode, st);
}

}  // namespace win
}  // namespace auv
