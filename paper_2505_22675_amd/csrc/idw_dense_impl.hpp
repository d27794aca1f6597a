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

// FP64 minimum / maximum of two non-NaN values (the list entries below):
// one instruction each, without the NaN quieting the compiler adds to fmin /
// fmax of values it cannot prove canonical.
__device__ inline double dmin(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ inline double dmax(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Key held in an FP64 list entry (see dense_node).
__device__ inline unsigned long long key_of(double v)
{
    return (unsigned long long)__double_as_longlong(v) - (1ull << 52);
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
    // explicitly global pointers (descriptors read from memory would
    // otherwise give flat loads)
    const auto gX = gmem(bv.X), gY = gmem(bv.Y), gI = gmem(bv.idx);
    const auto gC = gmem(bv.cell_start);
    typedef int v4i __attribute__((ext_vector_type(4)));
    const auto gR = gmem(reinterpret_cast<const v4i *>(bv.rec));
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

    // The k smallest keys, ascending.  A key (below 2^62) is held as the
    // FP64 number whose bit pattern is key + 2^52: a normal positive double,
    // so FP64 order is key order and the sorted insert is a min/max network
    // (list'[j] = max(list[j-1], min(key, list[j]))), two full-rate FP64
    // operations per entry instead of compares and 64-bit selects.
    double list[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        list[j] = __builtin_huge_val();
    int found = 0;

    // One candidate (valid: it exists).  The insert is branch-free: a key not
    // below the list's last entry leaves the sorted list unchanged under the
    // min/max network, so candidates outside the disk enter as +infinity.
    // (A branch around the network costs more: some lane of the wave nearly
    // always inserts, and the two paths' list registers then need copies.)
    auto consider = [&](int Ik, int Xk, int Yk, bool valid) {
        const int dX = Xk - Xn, dY = Yk - Yn;
        const long long D2 = (long long)dX * dX + (long long)dY * dY;
        const bool in = valid & (D2 <= R2);
        found += in ? 1 : 0;
        const unsigned long long key = ((unsigned long long)D2 << kb) | (unsigned)Ik;
        const double kd =
            in ? __longlong_as_double((long long)(key + (1ull << 52))) : __builtin_huge_val();
#pragma unroll
        for (int j = KMAX - 1; j > 0; --j)
            list[j] = dmax(list[j - 1], dmin(kd, list[j]));
        list[0] = dmin(kd, list[0]);
    };
    // the soundings of one bin segment, four at a time (their coordinates and
    // indices are loaded together, so the loads overlap; a missing fourth
    // reloads the segment's last sounding and enters as invalid)
    auto segment = [&](int row, int c0, int c1) {
        c0 = max(c0, 0);
        c1 = min(c1, bv.nbx - 1);
        if (row < 0 || row >= bv.nby || c0 > c1)
            return;
        const int id = row * bv.nbx;
        const int e = gC[id + c1 + 1];
        for (int k = gC[id + c0]; k < e; k += 4) {
            int Xk[4], Yk[4], Ik[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kk = min(k + u, e - 1);
                Xk[u] = gX[kk];
                Yk[u] = gY[kk];
                Ik[u] = gI[kk];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                consider(Ik[u], Xk[u], Yk[u], k + u < e);
        }
    };

    {
        for (int d = 0;; ++d) {
            // ring d: its top and bottom rows, then the left and right bins of
            // the rows between (one loop, so the candidate code is inlined once)
            const int nseg = d == 0 ? 1 : 4 * d;
            for (int sg = 0; sg < nseg; ++sg) {
                int row, c0, c1;
                if (sg < 2) {
                    row = sg == 0 ? byn - d : byn + d;
                    c0 = bxn - d;
                    c1 = bxn + d;
                } else {
                    row = byn - d + 1 + ((sg - 2) >> 1);
                    c0 = c1 = (sg & 1) ? bxn + d : bxn - d;
                }
                segment(row, c0, c1);
            }
            // every unvisited sounding is at least lb away
            const long long lb = (long long)d * B + m0;
            if (lb * lb > R2)
                break;
            if (found >= kcap && (long long)(key_of(list[kcap - 1]) >> kb) < lb * lb)
                break;
        }
    }

    const int m = min(found, kcap);
    unsigned long long keys[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        keys[j] = key_of(list[j]);
    const int64_t o = (int64_t)an * a.nx + b;
    const unsigned long long imask = (1ull << kb) - 1ull;
    if (kMode & 2) {
        const int bi = m > 0 ? (int)(keys[0] & imask) : -1;
        if (a.nn_idx_out)
            gmem(a.nn_idx_out)[o] = bi;
        if (a.nn_z_out)
            gmem(a.nn_z_out)[o] = m > 0 ? __int_as_float(gR[bi].w) : NAN;
    }
    if constexpr (kIdw) {
        if (a.cnt_out)
            gmem(a.cnt_out)[o] = m;
        float v;
        if (m == 0) {
            v = NAN;
        } else if ((keys[0] >> kb) == 0ull) {
            // hits: the members with D^2 == 0, in ascending index
            double hs = 0.0;
            int nh = 0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < m && (keys[j] >> kb) == 0ull) {
                    hs += (double)__int_as_float(gR[(int)(keys[j] & imask)].w);
                    ++nh;
                }
            }
            v = (float)(hs / (double)nh);
        } else if (m < a.min_pts) {
            v = NAN;
        } else {
            const float z0 = __int_as_float(gR[(int)(keys[0] & imask)].w);
            float num = 0.0f, den = 0.0f, zmin = z0, zmax = z0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < m) {
                    const v4i r = gR[(int)(keys[j] & imask)];
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
        gmem(a.z_out)[o] = v;
    }
}

// Whether the dense form's keys fit: (R^2 << index bits) plus the largest
// index stays below 2^62 (the FP64 list entries hold key + 2^52).
__host__ __device__ inline bool dense_key_ok(int32_t R, int32_t idx_bits)
{
    const unsigned __int128 top = ((unsigned __int128)((unsigned long long)R * (unsigned long long)R)
                                   << idx_bits) +
                                  ((unsigned __int128)1 << idx_bits);
    return top < ((unsigned __int128)1 << 62);
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
