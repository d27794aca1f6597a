// Radius-limited IDW with a small cap k on dense soundings (gfx950).
//
// When a node's disk holds many more soundings than k, the selection dominates.
// Here one lane owns one node (a wave covers an 8x8 node tile) and walks the
// bins in square rings around the node's own bin, nearest ring first, keeping
// the k smallest keys (D^2 << b | original index) in a sorted register list.
// After ring d every unvisited sounding is at least d*B + m0 away (m0: the
// node's distance to the nearest edge of its bin), so the walk stops once the
// k-th key's D^2 is below that bound squared, or the bound exceeds the radius.
// The selected set is exact; weights are then summed in key order (nearest
// first), the order the FP64 definition uses.
#pragma once
#include "auv_internal.hpp"

#include <climits>
#include <cmath>

namespace auv {

namespace dense {

constexpr int kDT = 8;  // 8x8 nodes per wave

__device__ inline int xcd_tile(int bid, int ntiles)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int q = ntiles >> 3, rem = ntiles & 7;
    return xcd * q + min(xcd, rem) + local;
}

struct NodeL {
    int X, q;
};

__device__ inline NodeL node_lat(int j, double d)
{
#pragma clang fp contract(off)
    const double u = ((double)j + 0.5) * d;
    const double t = u * kLatticePerMetre;
    const double r = rint(t);
    NodeL o;
    o.X = (int)r;
    o.q = (int)rint((t - r) * 32768.0);
    return o;
}

__device__ inline float wfast(float d2, int pmode, float power, float inv_r2)
{
    d2 = fmaxf(d2, 0x1p-40f);
    if (pmode == 1)
        return __builtin_amdgcn_rsqf(d2);
    if (pmode == 2)
        return __builtin_amdgcn_rcpf(d2);
    if (pmode == 3) {
        const float r = __builtin_amdgcn_rsqf(d2);
        return r * r * r;
    }
    // general power on the radius-normalised distance (>= 1 inside the disk)
    return __builtin_amdgcn_exp2f(-0.5f * power * __builtin_amdgcn_logf(d2 * inv_r2));
}

// Exact value of node (row an, column b) by one lane (no wave-wide operations,
// so any subset of lanes may call it): ring search for the max_pts nearest
// keys (max_pts <= KMAX), then the weighted sum in key order.  Writes the
// node's outputs.
template <int kMode, int KMAX>
__device__ void dense_node(const auv_bin_view &bv, const IdwArgs &a, int b, int an, int pmode)
{
    constexpr bool kIdw = (kMode & 1) != 0;
    const NodeL nx_l = node_lat(b, a.dx), ny_l = node_lat(an, a.dy);
    const int Xn = nx_l.X, Yn = ny_l.X;
    const int s = bv.bin_log2;
    const int B = 1 << s;
    const int hB = bv.halo << s;
    const int R = a.R;
    const long long R2 = (long long)R * R;
    const int kb = bv.idx_bits;
    const int kcap = a.max_pts;  // 1 <= kcap <= KMAX
    const int bxn = (Xn + hB) >> s, byn = (Yn + hB) >> s;
    // distance from the node to the nearest edge of its bin
    const int ux = Xn + hB - (bxn << s), uy = Yn + hB - (byn << s);
    const int m0 = min(min(ux, B - ux), min(uy, B - uy));

    unsigned long long list[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        list[j] = ~0ull;
    int found = 0;

    auto consider = [&](int k) {
        const int dX = bv.X[k] - Xn, dY = bv.Y[k] - Yn;
        const long long D2 = (long long)dX * dX + (long long)dY * dY;
        if (D2 > R2)
            return;
        ++found;
        const unsigned long long key = ((unsigned long long)D2 << kb) | (unsigned)bv.idx[k];
        // insert into the ascending list, dropping its largest entry
        if (key < list[KMAX - 1]) {
#pragma unroll
            for (int j = KMAX - 1; j > 0; --j) {
                const unsigned long long lo = list[j - 1], cur = list[j];
                list[j] = key < lo ? lo : (key < cur ? key : cur);
            }
            list[0] = key < list[0] ? key : list[0];
        }
    };
    auto segment = [&](int row, int c0, int c1) {
        c0 = max(c0, 0);
        c1 = min(c1, bv.nbx - 1);
        if (row < 0 || row >= bv.nby || c0 > c1)
            return;
        const int id = row * bv.nbx;
        const int e = bv.cell_start[id + c1 + 1];
        for (int k = bv.cell_start[id + c0]; k < e; ++k)
            consider(k);
    };

    {
        for (int d = 0;; ++d) {
            segment(byn - d, bxn - d, bxn + d);
            if (d > 0) {
                segment(byn + d, bxn - d, bxn + d);
                for (int r = byn - d + 1; r <= byn + d - 1; ++r) {
                    segment(r, bxn - d, bxn - d);
                    segment(r, bxn + d, bxn + d);
                }
            }
            // every unvisited sounding is at least lb away
            const long long lb = (long long)d * B + m0;
            if (lb * lb > R2)
                break;
            if (found >= kcap && (long long)(list[kcap - 1] >> kb) < lb * lb)
                break;
        }
    }

    const int m = min(found, kcap);
    const int64_t o = (int64_t)an * a.nx + b;
    const unsigned long long imask = (1ull << kb) - 1ull;
    if (kMode & 2) {
        const int bi = m > 0 ? (int)(list[0] & imask) : -1;
        if (a.nn_idx_out)
            a.nn_idx_out[o] = bi;
        if (a.nn_z_out)
            a.nn_z_out[o] = m > 0 ? __int_as_float(bv.rec[bi].w) : NAN;
    }
    if constexpr (kIdw) {
        if (a.cnt_out)
            a.cnt_out[o] = m;
        float v;
        if (m == 0) {
            v = NAN;
        } else if ((list[0] >> kb) == 0ull) {
            // hits: the members with D^2 == 0, in ascending index
            double hs = 0.0;
            int nh = 0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < m && (list[j] >> kb) == 0ull) {
                    hs += (double)__int_as_float(bv.rec[(int)(list[j] & imask)].w);
                    ++nh;
                }
            }
            v = (float)(hs / (double)nh);
        } else if (m < a.min_pts) {
            v = NAN;
        } else {
            const float z0 = __int_as_float(bv.rec[(int)(list[0] & imask)].w);
            float num = 0.0f, den = 0.0f, zmin = z0, zmax = z0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < m) {
                    const int4 r = bv.rec[(int)(list[j] & imask)];
                    const float z = __int_as_float(r.w);
                    const int qx = (int)(int16_t)((uint32_t)r.z & 0xffffu);
                    const int qy = (int)(int16_t)((uint32_t)r.z >> 16);
                    const float fx = (float)(r.x - Xn) + (float)(qx - nx_l.q) * kResidualUnit;
                    const float fy = (float)(r.y - Yn) + (float)(qy - ny_l.q) * kResidualUnit;
                    const float w = wfast(fx * fx + fy * fy, pmode, a.power, a.inv_r2);
                    num += w * (z - z0);
                    den += w;
                    zmin = fminf(zmin, z);
                    zmax = fmaxf(zmax, z);
                }
            }
            double r = (double)z0 + (double)num / (double)den;
            r = fmin(fmax(r, (double)zmin), (double)zmax);
            v = (float)r;
        }
        a.z_out[o] = v;
    }
}

// Node tile of the dense form: tile_w columns (a power of two from 1 to 64,
// default 8) by 64 / tile_w rows.
__host__ __device__ inline int dense_tile_w(const IdwArgs &a)
{
    return a.tile_w >= 1 && a.tile_w <= 64 && (a.tile_w & (a.tile_w - 1)) == 0 ? a.tile_w : kDT;
}

// One 64-lane wave per node tile (8 x 8 by default), one node per lane.
template <int kMode, int KMAX>
__device__ void dense_tile(const auv_bin_view &bv, const IdwArgs &a, int tile, int ntx,
                           int pmode)
{
    const int lane = threadIdx.x & 63;
    const int TW = dense_tile_w(a), TH = 64 / TW;
    const int tx = tile % ntx, ty = tile / ntx;
    const int b = tx * TW + (lane & (TW - 1)), an = ty * TH + lane / TW;
    if (b < a.nx && an < a.ny)
        dense_node<kMode, KMAX>(bv, a, b, an, pmode);
}

template <int kMode, int KMAX>
__global__ __launch_bounds__(64) void k_idw_dense(auv_bin_view bv, IdwArgs a, int ntx,
                                                   int nty, int pmode)
{
    dense_tile<kMode, KMAX>(bv, a, xcd_tile(blockIdx.x, ntx * nty), ntx, pmode);
}

}  // namespace dense
}  // namespace auv
