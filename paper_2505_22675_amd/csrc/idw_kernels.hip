// Radius-limited IDW and nearest-neighbour gridding on gfx950.
//
// One 64-lane wavefront (one workgroup) owns an 8x8 tile of grid nodes, one
// node per lane.  The binned soundings of every bin row that meets the tile
// grown by the radius are contiguous in memory; the wave stages them into LDS
// in chunks and every lane tests each staged sounding against its node
// (broadcast LDS reads, no bank conflicts).
//
// Exactness: membership, ranking, hits and the nearest pick use the exact
// lattice D^2 (integers carried in FP64: |dX| < 2^26, so the products and the
// sum are exact).  Distances and weights run in FP32 from the lattice offset
// plus the stored sub-lattice residuals; the final num/den division is FP64.
//
// Cap: a node with more than max_pts members finds the rank-k key (D^2,
// index) by bisection over D^2 and then over the index among ties, re-sweeping
// the staged candidates; only waves that hold such a node pay for it.
#include "auv_internal.hpp"

#include <algorithm>
#include <climits>
#include <cmath>

namespace auv {

namespace {

constexpr int kTW = 8, kTH = 8;    // nodes per wave tile
constexpr int kCap = 512;          // staged soundings per chunk
constexpr int kMaxRows = 64;       // bin rows staged per pass

struct __align__(16) Cand {
    int X, Y;
    uint32_t res;
    float z;
};

// Map a linear block id to a tile so that each of the 8 XCDs (blocks are
// dealt round-robin to XCDs) works on one contiguous band of tiles, keeping
// the halo re-reads of neighbouring tiles in the same L2.
__device__ inline int xcd_tile(int bid, int ntiles)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int q = ntiles >> 3, rem = ntiles & 7;
    return xcd * q + min(xcd, rem) + local;
}

struct NodeLat {
    int X;      // lattice coordinate
    int q;      // residual in 2^-15 lattice units
};

// FP64 rebase of a node coordinate ((j + 1/2) d) onto the lattice.
__device__ inline NodeLat node_lattice(int j, double d)
{
#pragma clang fp contract(off)
    const double u = ((double)j + 0.5) * d;
    const double t = u * kLatticePerMetre;
    const double r = rint(t);
    NodeLat o;
    o.X = (int)r;
    o.q = (int)rint((t - r) * 32768.0);
    return o;
}

// Fast weights for p = 1, 2, 3 on the squared distance normalised by R^2
// (so that w >= 1 and the common scale cancels in num/den).  The floor only
// guards an exactly-zero offset; real offsets stay far above it.
__device__ inline float weight_fast(float d2n, int pmode)
{
    d2n = fmaxf(d2n, 0x1p-80f);
    if (pmode == 1)
        return __builtin_amdgcn_rsqf(d2n);
    if (pmode == 2)
        return __builtin_amdgcn_rcpf(d2n);
    const float r = __builtin_amdgcn_rsqf(d2n);
    return r * r * r;
}

// Per-lane accumulator over the selected set.
struct Acc {
    int cnt;
    double best_d2;
    int best_i;
    float best_z;
    int hits;
    double hit_sum;
    float z_first, num, den, zmin, zmax;
    float emax;  // running max exponent (general power only)

    __device__ void reset()
    {
        emax = -INFINITY;
        cnt = 0;
        best_d2 = 1e300;
        best_i = INT_MAX;
        best_z = 0.0f;
        hits = 0;
        hit_sum = 0.0;
        z_first = 0.0f;
        num = 0.0f;
        den = 0.0f;
        zmin = INFINITY;
        zmax = -INFINITY;
    }
};

struct Tile {
    int bx_lo, nbx_row;   // first bin column, bins per row segment
    int by_lo, nrows;     // first bin row, number of rows
};

// Stage the tile's candidates chunk by chunk and call f(cand, orig_idx) on
// every lane for every staged sounding.  Must be called by the whole wave.
template <class F>
__device__ inline void sweep(const auv_bin_view &bv, const Tile &t, Cand *s_c,
                             int *s_i, int *s_beg, int *s_off, F &&f)
{
    const int lane = threadIdx.x;
    for (int r0 = 0; r0 < t.nrows; r0 += kMaxRows) {
        const int nr = min(kMaxRows, t.nrows - r0);
        int beg = 0, len = 0;
        if (lane < nr) {
            const int id0 = (t.by_lo + r0 + lane) * bv.nbx + t.bx_lo;
            beg = bv.cell_start[id0];
            len = bv.cell_start[id0 + t.nbx_row] - beg;
        }
        // exclusive scan of the row lengths across the wave
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
            s_beg[lane] = beg;
            s_off[lane] = inc - len;
        }
        if (lane == 0)
            s_off[nr] = total;
        __syncthreads();
        for (int c0 = 0; c0 < total; c0 += kCap) {
            const int cn = min(kCap, total - c0);
            for (int e = lane; e < cn; e += 64) {
                const int g = c0 + e;
                // row of g: last r with s_off[r] <= g
                int lo = 0, hi = nr - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= g)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const int src = s_beg[lo] + (g - s_off[lo]);
                Cand c;
                c.X = bv.X[src];
                c.Y = bv.Y[src];
                c.res = bv.res[src];
                c.z = bv.z[src];
                s_c[e] = c;
                s_i[e] = bv.idx[src];
            }
            __syncthreads();
            for (int e = 0; e < cn; ++e)
                f(s_c[e], s_i[e]);
            __syncthreads();
        }
    }
}

template <int kMode>
__global__ __launch_bounds__(64) void k_idw_tile(auv_bin_view bv, IdwArgs a,
                                                  int ntx, int nty, int pmode)
{
    __shared__ Cand s_c[kCap];
    __shared__ int s_i[kCap];
    __shared__ int s_beg[kMaxRows];
    __shared__ int s_off[kMaxRows + 1];

    constexpr bool kIdw = (kMode & 1) != 0;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int tx = tile % ntx, ty = tile / ntx;
    const int lane = threadIdx.x;
    const int b = tx * kTW + (lane % kTW);
    const int arow = ty * kTH + (lane / kTW);
    const bool active = b < a.nx && arow < a.ny;

    const NodeLat nx_l = node_lattice(b, a.dx);
    const NodeLat ny_l = node_lattice(arow, a.dy);

    // tile extent on the lattice -> bin rows and columns to stage
    const int b0 = tx * kTW, b1 = min(b0 + kTW, a.nx) - 1;
    const int a0 = ty * kTH, a1 = min(a0 + kTH, a.ny) - 1;
    const int hB = bv.halo << bv.bin_log2;
    const int R = a.R;
    Tile t;
    t.bx_lo = (node_lattice(b0, a.dx).X - R + hB) >> bv.bin_log2;
    t.nbx_row = ((node_lattice(b1, a.dx).X + R + hB) >> bv.bin_log2) - t.bx_lo + 1;
    t.by_lo = (node_lattice(a0, a.dy).X - R + hB) >> bv.bin_log2;
    t.nrows = ((node_lattice(a1, a.dy).X + R + hB) >> bv.bin_log2) - t.by_lo + 1;

    const double R2 = (double)R * (double)R;
    const float invR2 = (float)(1.0 / R2);
    const int kcap = a.max_pts;
    const int nqx = nx_l.q, nqy = ny_l.q;

    Acc acc;
    acc.reset();
    // selection predicate on (D^2, index): everything, or key <= (T, J)
    bool capped = false;
    double selT = 0.0;
    int selJ = INT_MAX;

    auto consider = [&](const Cand &c, int ci) {
        const int dX = c.X - nx_l.X, dY = c.Y - ny_l.X;
        const double fx = (double)dX, fy = (double)dY;
        const double d2 = fx * fx + fy * fy;  // exact
        if (!(d2 <= R2))
            return;
        if (capped && !(d2 < selT || (d2 == selT && ci <= selJ)))
            return;
        acc.cnt += 1;
        if (d2 < acc.best_d2 || (d2 == acc.best_d2 && ci < acc.best_i)) {
            acc.best_d2 = d2;
            acc.best_i = ci;
            acc.best_z = c.z;
        }
        if constexpr (kIdw) {
            if (d2 == 0.0) {
                acc.hits += 1;
                acc.hit_sum += (double)c.z;
            }
            if (acc.cnt == 1)
                acc.z_first = c.z;
            const int cqx = (int)(int16_t)(c.res & 0xffffu);
            const int cqy = (int)(int16_t)(c.res >> 16);
            const float ox = (float)dX + (float)(cqx - nqx) * kResidualUnit;
            const float oy = (float)dY + (float)(cqy - nqy) * kResidualUnit;
            const float d2n = (ox * ox + oy * oy) * invR2;
            float w;
            if (pmode != 0) {
                w = weight_fast(d2n, pmode);
            } else {
                // w = d2n^(-p/2) carried as 2^(e - emax) with a running
                // maximum exponent, so that no power overflows
                const float e = -0.5f * a.power * __builtin_amdgcn_logf(fmaxf(d2n, 0x1p-120f));
                if (e > acc.emax) {
                    const float sc = __builtin_amdgcn_exp2f(acc.emax - e);
                    acc.num *= sc;
                    acc.den *= sc;
                    acc.emax = e;
                }
                w = __builtin_amdgcn_exp2f(e - acc.emax);
            }
            acc.num += w * (c.z - acc.z_first);
            acc.den += w;
            acc.zmin = fminf(acc.zmin, c.z);
            acc.zmax = fmaxf(acc.zmax, c.z);
        }
    };

    sweep(bv, t, s_c, s_i, s_beg, s_off, consider);

    // exact k-cap for nodes with more than max_pts members
    bool over = active && kcap > 0 && acc.cnt > kcap;
    if (__any(over)) {
        double lo = 0.0, hi = R2;
        while (__any(over && lo < hi)) {
            const double mid = floor((lo + hi) * 0.5);
            int c = 0;
            sweep(bv, t, s_c, s_i, s_beg, s_off, [&](const Cand &cd, int) {
                const double fx = (double)(cd.X - nx_l.X), fy = (double)(cd.Y - ny_l.X);
                c += (fx * fx + fy * fy <= mid) ? 1 : 0;
            });
            if (over && lo < hi) {
                if (c >= kcap)
                    hi = mid;
                else
                    lo = mid + 1.0;
            }
        }
        // lo = D^2 of the rank-k member; keep `need` of the ties at lo
        int clt = 0, ceq = 0;
        sweep(bv, t, s_c, s_i, s_beg, s_off, [&](const Cand &cd, int) {
            const double fx = (double)(cd.X - nx_l.X), fy = (double)(cd.Y - ny_l.X);
            const double d2 = fx * fx + fy * fy;
            clt += d2 < lo ? 1 : 0;
            ceq += d2 == lo ? 1 : 0;
        });
        const int need = kcap - clt;
        bool tie = over && ceq > need;
        long long jlo = 0, jhi = INT_MAX;
        while (__any(tie && jlo < jhi)) {
            const long long mid = (jlo + jhi) >> 1;
            int c = 0;
            sweep(bv, t, s_c, s_i, s_beg, s_off, [&](const Cand &cd, int ci) {
                const double fx = (double)(cd.X - nx_l.X), fy = (double)(cd.Y - ny_l.X);
                c += (fx * fx + fy * fy == lo && ci <= mid) ? 1 : 0;
            });
            if (tie && jlo < jhi) {
                if (c >= need)
                    jhi = mid;
                else
                    jlo = mid + 1;
            }
        }
        if (over) {
            capped = true;
            selT = lo;
            selJ = tie ? (int)jlo : INT_MAX;
            acc.reset();
        }
        // lanes that are not over keep their accumulator: consider() is
        // re-applied only where `capped` holds
        Acc keep = acc;
        sweep(bv, t, s_c, s_i, s_beg, s_off, [&](const Cand &cd, int ci) {
            if (capped)
                consider(cd, ci);
        });
        if (!capped)
            acc = keep;
    }

    if (!active)
        return;
    const int64_t o = (int64_t)arow * a.nx + b;
    const int m = acc.cnt;
    if (kMode & 2) {
        if (a.nn_idx_out)
            a.nn_idx_out[o] = m > 0 ? acc.best_i : -1;
        if (a.nn_z_out)
            a.nn_z_out[o] = m > 0 ? acc.best_z : NAN;
    }
    if constexpr (kIdw) {
        if (a.cnt_out)
            a.cnt_out[o] = m;
        float v;
        if (acc.hits > 0) {
            v = (float)(acc.hit_sum / (double)acc.hits);
        } else if (m == 0 || m < a.min_pts) {
            v = NAN;
        } else {
            double r = (double)acc.z_first + (double)acc.num / (double)acc.den;
            r = fmin(fmax(r, (double)acc.zmin), (double)acc.zmax);
            v = (float)r;
        }
        a.z_out[o] = v;
    }
}

}  // namespace

auv_status launch_idw(const auv_bin_view &bv, const IdwArgs &a_in, hipStream_t st)
{
    IdwArgs a = a_in;
    const int ntx = (a.nx + kTW - 1) / kTW, nty = (a.ny + kTH - 1) / kTH;
    const int64_t ntiles = (int64_t)ntx * nty;
    if (ntiles > INT_MAX)
        return fail(AUV_ERR_RANGE, "too many tiles");
    int pmode = 0;
    if (a.power == 1.0f)
        pmode = 1;
    else if (a.power == 2.0f)
        pmode = 2;
    else if (a.power == 3.0f)
        pmode = 3;
    a.pmode = pmode;
    if (a.dense)
        return launch_idw_dense(bv, a, pmode, st);
    WinGeom wg;
    if (window_geometry(a, &wg))
        return launch_idw_window(bv, a, wg, pmode, st);
    if (a.precision != AUV_P_FP32_REBASE)
        return fail(AUV_ERR_INVALID,
                    "precision variants need a node spacing that is a multiple of 2^-15 m "
                    "and a window of at most 256 nodes");
    const dim3 grid((unsigned)ntiles), block(64);
    switch (a.mode) {
    case 1: k_idw_tile<1><<<grid, block, 0, st>>>(bv, a, ntx, nty, pmode); break;
    case 2: k_idw_tile<2><<<grid, block, 0, st>>>(bv, a, ntx, nty, pmode); break;
    case 3: k_idw_tile<3><<<grid, block, 0, st>>>(bv, a, ntx, nty, pmode); break;
    default: return fail(AUV_ERR_INVALID, "bad IDW mode");
    }
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
