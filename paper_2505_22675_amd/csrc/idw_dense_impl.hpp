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

// Element k of a binned array through a 32-bit byte offset from its base
// (k < 2^30: the dense form needs at most 30 index bits), so that a uniform
// base takes the scalar-base form of the load instead of 64-bit addresses.
template <class T>
__device__ inline T ld_at(gptr<const T> base, uint32_t k)
{
    return *(gptr<const T>)((gptr<const char>)base + (k * (uint32_t)sizeof(T)));
}

// Compare-exchange: a takes the smaller, b the larger.
__device__ inline void cex(double &a, double &b)
{
    const double lo = dmin(a, b), hi = dmax(a, b);
    a = lo;
    b = hi;
}

// Merge four new entries into the ascending list of the K smallest (K a
// power of two, at least 8), keeping the K smallest of the union, ascending.
// The four are sorted (five compare-exchanges); the element-wise minimum of
// the list with them reversed and padded with +infinity at the front holds
// the K smallest and is bitonic (the lower half of a bitonic half-cleaner),
// and a bitonic merge sorts it.  In its first stage only the pairs that
// meet a changed entry can be out of order.  Four inserts one by one would
// take 4 (2K - 1) operations; this takes 4 + 10 + 2 (K/2 log2 K - K/2 + 4).
template <int K>
__device__ inline void merge4(double (&list)[K], double k0, double k1, double k2, double k3)
{
    static_assert(K >= 8 && (K & (K - 1)) == 0, "list length");
    cex(k0, k1);
    cex(k2, k3);
    cex(k0, k2);
    cex(k1, k3);
    cex(k1, k2);
    list[K - 4] = dmin(list[K - 4], k3);
    list[K - 3] = dmin(list[K - 3], k2);
    list[K - 2] = dmin(list[K - 2], k1);
    list[K - 1] = dmin(list[K - 1], k0);
#pragma unroll
    for (int i = K / 2 - 4; i < K / 2; ++i)
        cex(list[i], list[i + K / 2]);
#pragma unroll
    for (int d = K / 4; d >= 1; d >>= 1) {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((i & d) == 0)
                cex(list[i], list[i + d]);
    }
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
__device__ __forceinline__ void dense_node(const auv_bin_view &bv, const IdwArgs &a, int b, int an,
                                           int pmode)
{
    constexpr bool kIdw = (kMode & 1) != 0;
    // explicitly global pointers (descriptors read from memory would
    // otherwise give flat loads)
    const gptr<const int32_t> gX = gmem(bv.X), gY = gmem(bv.Y), gI = gmem(bv.idx);
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
    // so FP64 order is key order and the list is kept by min/max networks
    // (full-rate FP64 operations instead of compares and 64-bit selects).
    double list[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        list[j] = __builtin_huge_val();

    // The list entry of one candidate (valid: it exists); candidates outside
    // the disk enter as +infinity, which no merge keeps ahead of a key.  The
    // merge is branch-free (a branch around it costs more: some lane of the
    // wave nearly always inserts, and the two paths' list registers then need
    // copies).  The list's finite entries are the min(found, KMAX) nearest
    // members, so the number found is not kept: "at least j found" is
    // list[j - 1] < inf.
    auto entry = [&](int Ik, int Xk, int Yk, bool valid) {
        const int dX = Xk - Xn, dY = Yk - Yn;
        const long long D2 = (long long)dX * dX + (long long)dY * dY;
        const bool in = valid & (D2 <= R2);
        const unsigned long long key = ((unsigned long long)D2 << kb) | (unsigned)Ik;
        return in ? __longlong_as_double((long long)(key + (1ull << 52))) : __builtin_huge_val();
    };
    // the soundings of one bin segment, four at a time (their coordinates and
    // indices are loaded together, so the loads overlap; a missing fourth
    // reloads the segment's last sounding and enters as invalid)
    auto segment = [&](int row, int c0, int c1) {
        // an empty range for a segment outside the bin domain (no early
        // return: the list stays in the same registers on every path)
        c0 = max(c0, 0);
        c1 = min(c1, bv.nbx - 1);
        const bool ok = row >= 0 && row < bv.nby && c0 <= c1;
        const int id = ok ? row * bv.nbx : 0;
        int k = ok ? gC[id + c0] : 0;
        const int e = ok ? gC[id + c1 + 1] : 0;
        for (; k < e; k += 4) {
            int Xk[4], Yk[4], Ik[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t kk = (uint32_t)min(k + u, e - 1);
                Xk[u] = ld_at(gX, kk);
                Yk[u] = ld_at(gY, kk);
                Ik[u] = ld_at(gI, kk);
            }
            // the first candidate is always valid; without this the compiler
            // moves its index load into a branch that waits for it alone
            asm volatile("" : "+v"(Ik[0]));
            merge4(list, entry(Ik[0], Xk[0], Yk[0], true), entry(Ik[1], Xk[1], Yk[1], k + 1 < e),
                   entry(Ik[2], Xk[2], Yk[2], k + 2 < e), entry(Ik[3], Xk[3], Yk[3], k + 3 < e));
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
            // the cap-th key (a select chain over the list: an indexed read
            // would copy the list into consecutive registers every ring)
            double kth = list[0];
#pragma unroll
            for (int j = 1; j < KMAX; ++j)
                kth = j == kcap - 1 ? list[j] : kth;
            if (kth < __builtin_huge_val() && (long long)(key_of(kth) >> kb) < lb * lb)
                break;
        }
    }

    int m = 0;  // members taken: min(found, kcap)
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        m += (j < kcap && list[j] < __builtin_huge_val()) ? 1 : 0;
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
// index stays below 2^62 (the FP64 list entries hold key + 2^52), and the
// binned arrays are addressed by 32-bit byte offsets (at most 30 index bits).
__host__ __device__ inline bool dense_key_ok(int32_t R, int32_t idx_bits)
{
    if (idx_bits > 30)
        return false;
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
