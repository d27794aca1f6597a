// Bilinear (Sec. III-A) and Catmull-Rom bicubic (Sec. III-B) resampling of
// one grid onto another.
//
// The source index coordinate of a node is computed in FP64 with the same
// operations, in the same order, as its definition (no contraction), so the
// corner choice is exact; the blend itself is FP32 in lerp form (top, bottom, then vertical),
// which keeps constants exact and lets a NaN corner propagate: a hole.
#include "resample_axis.hpp"

#include <algorithm>
#include <climits>
#include <cmath>

namespace auv {

namespace {


struct BilArgs {
    const float *src;
    float *dst;
    double sx0, sy0, sdx, sdy;
    double dx0, dy0, ddx, ddy;
    int snx, sny, dnx, dny;
    int groups;  // k_bilinear: row groups per block (1 .. kBilGroups)
};

constexpr int kBilThreads = 256;
constexpr int kBilCols = kBilThreads * 4;  // destination columns per block
constexpr int kBilRows = 8;                // destination rows per block
constexpr int kBilStage = 6144;            // source values staged in LDS

// Patch of a block in a 1-D launch of ncb x nrb patches (row-major: column
// band fastest).  Blocks are dealt round-robin to the 8 XCDs; each XCD takes
// a contiguous run of patches, so it writes whole destination rows instead of
// one column band of every row.
__device__ inline void patch_of(int ncb, int nrb, int *bx, int *by)
{
    const int total = ncb * nrb;
    const int b = (int)blockIdx.x;
    const int xcd = b & 7, q = total >> 3, rem = total & 7;
    const int t = xcd * q + min(xcd, rem) + (b >> 3);
    *bx = t % ncb;
    *by = t / ncb;
}

// One block owns a 1024-column band of p.groups row groups of 8 rows each:
// up to kBilGroups while the launch keeps at least 1024 blocks (at cfg2 2x, 2,
// 4, 8 and 16 groups gave 73, 70, 68 and 104 us), one when the rectangles
// are too large to stage (then there is nothing to prefetch).
// The FP64 axis maps of its columns are computed once into LDS, those of its
// rows likewise; each row group's source rectangle is staged into LDS when it
// fits (otherwise corners are gathered from global memory), and the next
// group's rectangle is loaded into registers while the current group is
// blended and stored, so the reads' latency hides behind the stores.  Every
// thread produces four consecutive nodes per row with one 16-byte streaming
// store.
constexpr int kBilGroups = 8;  // row groups per block, at most
constexpr int kBilPf = 12;     // prefetched values per thread (rectangles up to 3072 values)

__global__ __launch_bounds__(kBilThreads) void k_bilinear(BilArgs p)
{
    __shared__ int s_i0[kBilCols], s_i1[kBilCols];
    __shared__ float s_t[kBilCols];
    __shared__ int s_j0[kBilGroups * kBilRows], s_j1[kBilGroups * kBilRows];
    __shared__ float s_s[kBilGroups * kBilRows];
    __shared__ float s_src[kBilStage];
    const int ngroups = (p.dny + kBilRows - 1) / kBilRows;
    int pbx, pby;
    patch_of((p.dnx + kBilCols - 1) / kBilCols, (ngroups + p.groups - 1) / p.groups, &pbx,
             &pby);
    const int col0 = pbx * kBilCols;
    const int g0 = pby * p.groups;               // first row group of the block
    const int ng = min(p.groups, ngroups - g0);  // row groups of the block
    const int ncol = min(kBilCols, p.dnx - col0);
    for (int c = threadIdx.x; c < kBilCols; c += kBilThreads) {
        const Axis a = axis_of(p.dx0, p.ddx, min(col0 + c, p.dnx - 1), p.sx0, p.sdx, p.snx);
        s_i0[c] = a.i0;
        s_i1[c] = a.i1;
        s_t[c] = a.t;
    }
    if (threadIdx.x < p.groups * kBilRows) {
        const int row = min(g0 * kBilRows + (int)threadIdx.x, p.dny - 1);
        const Axis a = axis_of(p.dy0, p.ddy, row, p.sy0, p.sdy, p.sny);
        s_j0[threadIdx.x] = a.i0;
        s_j1[threadIdx.x] = a.i1;
        s_s[threadIdx.x] = a.t;
    }
    __syncthreads();
    // source columns read by the band (the maps are monotone)
    const int il = s_i0[0], ih = s_i1[ncol - 1];
    const int sw = ih - il + 1;
    // source rows (first, count) of row group g
    auto rows_of = [&](int g) {
        const int nrow = min(kBilRows, p.dny - (g0 + g) * kBilRows);
        const int jl = s_j0[g * kBilRows];
        return make_int2(jl, s_j1[g * kBilRows + nrow - 1] - jl + 1);
    };
    // this thread's share of a rectangle: element e = threadIdx.x + k
    // kBilThreads at (row e / sw, column e % sw), walked incrementally
    float pf[kBilPf];
    auto fetch = [&](int jl, int sh) {
        const int n = sw * sh;
        const int t = (int)threadIdx.x;
        if (t >= n)
            return;
        int r = t / sw, cc = t - r * sw;
        const int dr = kBilThreads / sw, dc = kBilThreads - dr * sw;
        const float *row = p.src + (int64_t)(jl + r) * p.snx + il;
#pragma unroll
        for (int k = 0; k < kBilPf; ++k) {
            if (t + k * kBilThreads < n)
                pf[k] = row[cc];
            cc += dc;
            int step = dr;
            if (cc >= sw) {
                cc -= sw;
                ++step;
            }
            row += (int64_t)step * p.snx;
        }
    };
    auto place = [&](int sh) {
        const int n = sw * sh;
#pragma unroll
        for (int k = 0; k < kBilPf; ++k) {
            const int e = (int)threadIdx.x + k * kBilThreads;
            if (e < n)
                s_src[e] = pf[k];
        }
    };
    const int c = threadIdx.x * 4;
    int i0[4], i1[4];
    float t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        i0[k] = s_i0[min(c + k, kBilCols - 1)];
        i1[k] = s_i1[min(c + k, kBilCols - 1)];
        t[k] = s_t[min(c + k, kBilCols - 1)];
    }
    const bool vec = c + 4 <= ncol && (p.dnx & 3) == 0 &&
                     (reinterpret_cast<uintptr_t>(p.dst) & 15) == 0;
    int2 rc = rows_of(0);
    bool staged = (long long)sw * rc.y <= kBilStage;
    if (staged)
        stage_rect(p.src, p.snx, rc.x, il, sw, rc.y, s_src, kBilThreads);
    __syncthreads();
    for (int g = 0; g < ng; ++g) {
        const int2 nx = g + 1 < ng ? rows_of(g + 1) : make_int2(0, 0);
        const bool nstaged = g + 1 < ng && (long long)sw * nx.y <= kBilStage;
        // small rectangles (2x upsampling: about 2600 values) are loaded into
        // registers now and land in LDS after this group's stores
        const bool pref = nstaged && sw * nx.y <= kBilThreads * kBilPf;
        if (pref)
            fetch(nx.x, nx.y);
        const int row0 = (g0 + g) * kBilRows;
        const int nrow = min(kBilRows, p.dny - row0);
        const int jl = rc.x;
        if (c < ncol) {
            for (int r = 0; r < nrow; ++r) {
                const int q = g * kBilRows + r;
                const float s = s_s[q];
                float v[4];
                if (staged) {
                    const float *r0 = s_src + (s_j0[q] - jl) * sw - il;
                    const float *r1 = s_src + (s_j1[q] - jl) * sw - il;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float q00 = r0[i0[k]], q10 = r0[i1[k]];
                        const float q01 = r1[i0[k]], q11 = r1[i1[k]];
                        const float top = q00 + t[k] * (q10 - q00);
                        const float bot = q01 + t[k] * (q11 - q01);
                        v[k] = top + s * (bot - top);
                    }
                } else {
                    const float *r0 = p.src + (int64_t)s_j0[q] * p.snx;
                    const float *r1 = p.src + (int64_t)s_j1[q] * p.snx;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float q00 = r0[i0[k]], q10 = r0[i1[k]];
                        const float q01 = r1[i0[k]], q11 = r1[i1[k]];
                        const float top = q00 + t[k] * (q10 - q00);
                        const float bot = q01 + t[k] * (q11 - q01);
                        v[k] = top + s * (bot - top);
                    }
                }
                float *out = p.dst + (int64_t)(row0 + r) * p.dnx + col0 + c;
                if (vec) {
                    // streaming store: the destination is not re-read by this kernel
                    typedef float f4v __attribute__((ext_vector_type(4)));
                    const f4v vv = {v[0], v[1], v[2], v[3]};
                    __builtin_nontemporal_store(vv, reinterpret_cast<f4v *>(out));
                } else {
                    for (int k = 0; k < 4 && c + k < ncol; ++k)
                        out[k] = v[k];
                }
            }
        }
        __syncthreads();  // every read of this group's rectangle is done
        if (pref)
            place(nx.y);
        else if (nstaged)
            stage_rect(p.src, p.snx, nx.x, il, sw, nx.y, s_src, kBilThreads);
        __syncthreads();
        rc = nx;
        staged = nstaged;
    }
}

// Catmull-Rom cubic (Sec. III-B) through p0..p3 at t in [0, 1] between p1
// and p2, in Horner form.
__device__ inline float catmull_rom(float p0, float p1, float p2, float p3, float t)
{
    const float a1 = p2 - p0;
    const float a2 = 2.0f * p0 - 5.0f * p1 + 4.0f * p2 - p3;
    const float a3 = 3.0f * (p1 - p2) + p3 - p0;
    return 0.5f * (((a3 * t + a2) * t + a1) * t + 2.0f * p1);
}

constexpr int kCubStage = 6144;  // source values staged in LDS (with a one-tap halo)

// The row walk of k_bicubic for one thread's four columns: taps from the
// staged rectangle (kStaged) or from the source grid in global memory.
template <bool kStaged>
__device__ __forceinline__ void bicubic_walk(const BilArgs &p, const float *s_src,
                                             const int *s_i0, const float *s_t,
                                             const int *s_j0, const float *s_s, int il, int jl,
                                             int sw, int c, int ncol, int nrow, int row0,
                                             int col0)
{
    auto src_row = [&](int jr) -> const float * {
        if constexpr (kStaged)
            return s_src + (jr - jl) * sw;
        else
            return p.src + (int64_t)jr * p.snx;
    };
    // tap columns (relative to the staged rectangle, or absolute) per node
    int tc[4][4];
    float t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i0 = s_i0[min(c + k, ncol - 1)];
        t[k] = s_t[min(c + k, ncol - 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            tc[k][q] = min(max(i0 - 1 + q, 0), p.snx - 1) - (kStaged ? il : 0);
    }
    // horizontal cubics of source row jr at this thread's 4 columns
    auto hrow = [&](int jr) {
        const float *row = src_row(jr);
        float4 h;
        h.x = catmull_rom(row[tc[0][0]], row[tc[0][1]], row[tc[0][2]], row[tc[0][3]], t[0]);
        h.y = catmull_rom(row[tc[1][0]], row[tc[1][1]], row[tc[1][2]], row[tc[1][3]], t[1]);
        h.z = catmull_rom(row[tc[2][0]], row[tc[2][1]], row[tc[2][2]], row[tc[2][3]], t[2]);
        h.w = catmull_rom(row[tc[3][0]], row[tc[3][1]], row[tc[3][2]], row[tc[3][3]], t[3]);
        return h;
    };
    auto clampr = [&](int j) { return min(max(j, 0), p.sny - 1); };
    float4 h0 = make_float4(0.f, 0.f, 0.f, 0.f), h1 = h0, h2 = h0, h3 = h0;
    int cur = INT_MIN;  // j0 of the rows held in h0..h3 (block-uniform)
    const bool vec = c + 4 <= ncol && (p.dnx & 3) == 0 &&
                     (reinterpret_cast<uintptr_t>(p.dst) & 15) == 0;
    for (int r = 0; r < nrow; ++r) {
        const float s = s_s[r];
        const int j0 = s_j0[r];
        if (j0 != cur) {
            if (j0 == cur + 1) {
                h0 = h1;
                h1 = h2;
                h2 = h3;
                h3 = hrow(clampr(j0 + 2));
            } else {
                h0 = hrow(clampr(j0 - 1));
                h1 = hrow(clampr(j0));
                h2 = hrow(clampr(j0 + 1));
                h3 = hrow(clampr(j0 + 2));
            }
            cur = j0;
        }
        float v[4];
        v[0] = catmull_rom(h0.x, h1.x, h2.x, h3.x, s);
        v[1] = catmull_rom(h0.y, h1.y, h2.y, h3.y, s);
        v[2] = catmull_rom(h0.z, h1.z, h2.z, h3.z, s);
        v[3] = catmull_rom(h0.w, h1.w, h2.w, h3.w, s);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!isfinite(v[k])) {
                // bilinear on the inner taps (the corners of the node's cell)
                const float *r1 = src_row(clampr(j0));
                const float *r2 = src_row(clampr(j0 + 1));
                const float q00 = r1[tc[k][1]], q10 = r1[tc[k][2]];
                const float q01 = r2[tc[k][1]], q11 = r2[tc[k][2]];
                const float top = q00 + t[k] * (q10 - q00);
                const float bot = q01 + t[k] * (q11 - q01);
                v[k] = top + s * (bot - top);
            }
        }
        float *outp = p.dst + (int64_t)(row0 + r) * p.dnx + col0 + c;
        if (vec) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            const f4v vv = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(vv, reinterpret_cast<f4v *>(outp));
        } else {
            for (int k = 0; k < 4 && c + k < ncol; ++k)
                outp[k] = v[k];
        }
    }
}

// Catmull-Rom resample, the same patch layout as k_bilinear.  Taps are the
// source indices i0 - 1 .. i0 + 2 (clamped to the grid) around each node's
// cell; the cubic runs along x on the 4 tap rows, then along y.  The cubic is
// separable: walking down its patch, each thread keeps the horizontal cubics
// of the 4 current tap rows at its 4 columns in registers and computes a tap
// row's horizontal cubics only when the row enters the window, so each node
// costs one vertical cubic.  A node with a non-finite tap (NaN propagates
// through the cubic, so its result is not finite) takes the bilinear value of
// its 4 inner taps, NaN when one of them is NaN: a hole.
__global__ __launch_bounds__(kBilThreads) void k_bicubic(BilArgs p)
{
    __shared__ int s_i0[kBilCols];
    __shared__ float s_t[kBilCols];
    __shared__ int s_j0[kBilRows];
    __shared__ float s_s[kBilRows];
    __shared__ float s_src[kCubStage];
    int pbx, pby;
    patch_of((p.dnx + kBilCols - 1) / kBilCols, (p.dny + kBilRows - 1) / kBilRows, &pbx, &pby);
    const int col0 = pbx * kBilCols;
    const int row0 = pby * kBilRows;
    const int ncol = min(kBilCols, p.dnx - col0);
    const int nrow = min(kBilRows, p.dny - row0);
    for (int c = threadIdx.x; c < kBilCols; c += kBilThreads) {
        const Axis a = axis_of(p.dx0, p.ddx, min(col0 + c, p.dnx - 1), p.sx0, p.sdx, p.snx);
        s_i0[c] = a.i0;
        s_t[c] = a.t;
    }
    if (threadIdx.x < kBilRows) {
        const Axis a = axis_of(p.dy0, p.ddy, min(row0 + (int)threadIdx.x, p.dny - 1), p.sy0,
                               p.sdy, p.sny);
        s_j0[threadIdx.x] = a.i0;
        s_s[threadIdx.x] = a.t;
    }
    __syncthreads();
    // source rectangle of every tap of the patch, clamped to the grid (the
    // maps are monotone)
    const int il = max(s_i0[0] - 1, 0), ih = min(s_i0[ncol - 1] + 2, p.snx - 1);
    const int jl = max(s_j0[0] - 1, 0), jh = min(s_j0[nrow - 1] + 2, p.sny - 1);
    const int sw = ih - il + 1, sh = jh - jl + 1;
    const bool staged = (long long)sw * sh <= kCubStage;
    if (staged) {
        stage_rect(p.src, p.snx, jl, il, sw, sh, s_src, kBilThreads);
        __syncthreads();
    }
    const int c = threadIdx.x * 4;
    if (c >= ncol)
        return;
    // separate instantiations keep LDS and global reads apart (a pointer that
    // may be either would make every tap a flat load)
    if (staged)
        bicubic_walk<true>(p, s_src, s_i0, s_t, s_j0, s_s, il, jl, sw, c, ncol, nrow, row0, col0);
    else
        bicubic_walk<false>(p, s_src, s_i0, s_t, s_j0, s_s, il, jl, sw, c, ncol, nrow, row0, col0);
}

}  // namespace

auv_status launch_bicubic(const float *src, const auv_grid_desc &s, float *dst,
                          const auv_grid_desc &d, hipStream_t st)
{
    BilArgs p;
    p.src = src;
    p.dst = dst;
    p.sx0 = s.x0;
    p.sy0 = s.y0;
    p.sdx = s.dx;
    p.sdy = s.dy;
    p.dx0 = d.x0;
    p.dy0 = d.y0;
    p.ddx = d.dx;
    p.ddy = d.dy;
    p.snx = s.nx;
    p.sny = s.ny;
    p.dnx = d.nx;
    p.dny = d.ny;
    p.groups = 1;
    const unsigned grid = (unsigned)(((d.nx + kBilCols - 1) / kBilCols) *
                                     ((d.ny + kBilRows - 1) / kBilRows));
    k_bicubic<<<grid, kBilThreads, 0, st>>>(p);
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

auv_status launch_bilinear(const float *src, const auv_grid_desc &s, float *dst,
                           const auv_grid_desc &d, hipStream_t st)
{
    BilArgs p;
    p.src = src;
    p.dst = dst;
    p.sx0 = s.x0;
    p.sy0 = s.y0;
    p.sdx = s.dx;
    p.sdy = s.dy;
    p.dx0 = d.x0;
    p.dy0 = d.y0;
    p.ddx = d.dx;
    p.ddy = d.dy;
    p.snx = s.nx;
    p.sny = s.ny;
    p.dnx = d.nx;
    p.dny = d.ny;
    const int ngroups = (d.ny + kBilRows - 1) / kBilRows;
    const int64_t ncb = (d.nx + kBilCols - 1) / kBilCols;
    // a row group's source rectangle, roughly: several groups per block only
    // pay when it is staged (the next one is prefetched meanwhile)
    const double rect = (kBilCols * d.dx / s.dx + 2.0) * (kBilRows * d.dy / s.dy + 2.0);
    p.groups = rect > kBilStage
                   ? 1
                   : (int)std::max<int64_t>(1, std::min<int64_t>(kBilGroups,
                                                                 ncb * ngroups / 1024));
    const unsigned grid = (unsigned)(ncb * ((ngroups + p.groups - 1) / p.groups));
    k_bilinear<<<grid, kBilThreads, 0, st>>>(p);
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
