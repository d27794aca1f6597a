// Ordinary kriging resample of one grid onto another (Sec. III-C).
//
// A destination node maps to the source index coordinate u (as in the
// bilinear resample); its neighbourhood is the 5 x 5 source nodes centred on
// the node nearest to u, moved inward at the grid edges.  The weights solve
// the ordinary-kriging system
//     [ G  1 ] [ lambda ]   [ g ]
//     [ 1' 0 ] [   mu   ] = [ 1 ]
// with G the variogram between the 25 nodes, g the variogram between each node
// and the destination point and gamma(h) = 1 - exp(-h / a) (the sill cancels
// from the weights).  K = [G 1; 1' 0] depends only on the node spacing and the
// range, not on where the window sits, so it is inverted once on the host
// (FP64, Gauss-Jordan with partial pivoting) and, written as
//     z = z_c + sum_j g_j w_j,   w = K^-1 (z - z_c, 0)
// (z_c: the window centre; K is symmetric), w depends only on the window: a
// thread walking down a column computes it once per window and each node adds
// one 26-term product.
//
// K commutes with the mirror images of the window in x and in y, so in the
// basis of sums and differences of mirrored nodes (per axis: a0+a4, a1+a3,
// a2 | a0-a4, a1-a3) its inverse is block diagonal, with blocks for the four
// parity classes (even/odd in y, even/odd in x) of 10 (with the unbiasedness
// row), 6, 6 and 4 rows: w costs 178 multiply-adds and two 40-add transforms
// instead of 650 multiply-adds.  A window with a non-finite value falls back to
// bilinear.
#include "resample_axis.hpp"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <type_traits>

namespace auv {

namespace {

constexpr int kKrigCols = 256;    // destination columns per block (one per thread)
constexpr int kKrigRows = 32;     // destination rows per block, at most
constexpr int kKrigStage = 6144;  // source values staged in LDS
constexpr int kBlockFloats = 10 * 9 + 6 * 6 + 6 * 6 + 4 * 4;
constexpr double kMaxRangeSpacings = 1e4;  // the FP64 inverse stays well conditioned

struct KrigArgs {
    const float *src;
    float *dst;
    double sx0, sy0, sdx, sdy;
    double dx0, dy0, ddx, ddy;
    int snx, sny, dnx, dny;
    float fdx, fdy;  // source spacing
    float c2;        // (log2(e) / range)^2, or (1 / range)^2 for the series form
    int rows;        // destination rows per block (8 .. kKrigRows)
    // the diagonal blocks of K^-1 in the mirror basis, row-major: even-even
    // 10 x 9 (rows: 9 nodes and the unbiasedness entry; its column is never
    // used since the data vector has a zero there), even-odd 6 x 6, odd-even
    // 6 x 6, odd-odd 4 x 4
    float mb[kBlockFloats];
};

using cfloat = const __attribute__((address_space(4))) float;

// First index of the 5-node window centred on the node nearest to u.
__device__ inline int window_start(double u, int n)
{
    const int c = (int)floor(u + 0.5);
    return min(max(c - 2, 0), n - 5);
}

// The inverse of the kriging matrix K = [G 1; 1' 0] splits as [A b; b' c]
// with 1'A = 0 and 1'b = 1 (the weights A g + b sum to one for any g).  For
// w = K^-1 (z - z_c, 0), sum_q w_q = 0, so with g_q = 1 - e_q,
// e_q = exp(-h_q / range):
//     z = z_c + sum_q g_q w_q + w_25 = z_c + w_25 - sum_q e_q w_q.
// The entries of A grow with range / spacing while g shrinks, so the FP32
// rounding of e_q (about 6e-8 near 1) times w_q grows with the range: the
// exp form is kept to ranges under 16 hypot(dx, dy) (22.6 spacings on a
// square grid; relative depth error of a few 1e-6).  A window node lies at
// most 4 spacings per axis from the destination point (2.5 inside the grid,
// 4 where the window is moved in at an edge), so from there on every t =
// h / range is at most 1/4 and kSeries evaluates g_q = 1 - exp(-t) by its
// Taylor series to t^7 (truncation under 2e-9 relative), whose rounding is
// relative to g_q itself, and sums z = z_c + w_25 + sum_q g_q w_q.
template <bool kSeries>
__global__ __launch_bounds__(kKrigCols) void k_kriging(const KrigArgs p)
{
    __shared__ int s_wx[kKrigCols], s_i0[kKrigCols], s_i1[kKrigCols];
    __shared__ float s_du[kKrigCols], s_t[kKrigCols];
    __shared__ int s_wy[kKrigRows], s_j0[kKrigRows], s_j1[kKrigRows];
    __shared__ float s_dv[kKrigRows], s_s[kKrigRows];
    __shared__ float s_src[kKrigStage];
    const int col0 = blockIdx.x * kKrigCols;
    const int row0 = blockIdx.y * p.rows;
    const int ncol = min(kKrigCols, p.dnx - col0);
    const int nrow = min(p.rows, p.dny - row0);
    {
        const int c = threadIdx.x;
        const Axis a = axis_of(p.dx0, p.ddx, min(col0 + c, p.dnx - 1), p.sx0, p.sdx, p.snx);
        const int wx = window_start(a.u, p.snx);
        s_wx[c] = wx;
        s_du[c] = (float)(a.u - wx);
        s_i0[c] = a.i0;
        s_i1[c] = a.i1;
        s_t[c] = a.t;
    }
    if (threadIdx.x < p.rows) {
        const int r = threadIdx.x;
        const Axis a = axis_of(p.dy0, p.ddy, min(row0 + r, p.dny - 1), p.sy0, p.sdy, p.sny);
        const int wy = window_start(a.u, p.sny);
        s_wy[r] = wy;
        s_dv[r] = (float)(a.u - wy);
        s_j0[r] = a.i0;
        s_j1[r] = a.i1;
        s_s[r] = a.t;
    }
    __syncthreads();
    // source rectangle of every window of the patch (window starts are
    // monotone); the bilinear corners of a node lie inside its window
    const int il = s_wx[0], ih = s_wx[ncol - 1] + 4;
    const int jl = s_wy[0], jh = s_wy[nrow - 1] + 4;
    const int sw = ih - il + 1, sh = jh - jl + 1;
    const bool staged = (long long)sw * sh <= kKrigStage;
    if (staged) {
        stage_rect(p.src, p.snx, jl, il, sw, sh, s_src, kKrigCols);
        __syncthreads();
    }
    const int c = threadIdx.x;
    if (c >= ncol)
        return;
    // separate instantiations keep LDS and global reads apart (a value that
    // may come from either would make every read a flat load)
    auto walk = [&](auto staged_t) {
        constexpr bool kStaged = decltype(staged_t)::value;
        auto at = [&](int j, int i) {  // source value at row j, column i
            if constexpr (kStaged)
                return s_src[(j - jl) * sw + (i - il)];
            else
                return p.src[(int64_t)j * p.snx + i];
        };
        const int wx = s_wx[c];
        // squared x offsets to the window columns, scaled by (log2(e) / range)^2
        float ex2[5];
        {
            const float du = s_du[c];
    #pragma unroll
            for (int i = 0; i < 5; ++i) {
                const float e = ((float)i - du) * p.fdx;
                ex2[i] = e * e * p.c2;
            }
        }
        // the node's 25 covariance terms depend only on its offsets in the
        // window: x is fixed for the thread's column and rows cycle through a
        // few y offsets (two at a 2x resample), so the terms of the last two
        // offsets are kept and reused when a row's offset recurs
        float ca[25], cb[25];
        float dva = NAN, dvb = NAN;
        bool fill_a = true;
        auto terms = [&](float (&e)[25], float dv) {
    #pragma unroll
            for (int k = 0; k < 5; ++k) {
                const float ey = ((float)k - dv) * p.fdy;
                const float ey2 = ey * ey * p.c2;
    #pragma unroll
                for (int i = 0; i < 5; ++i) {
                    const float t = __builtin_amdgcn_sqrtf(ex2[i] + ey2);
                    if constexpr (kSeries) {
                        // 1 - exp(-t) = t (1 - t/2 (1 - t/3 (... (1 - t/7))))
                        float g = fmaf(-t, 1.0f / 7.0f, 1.0f);
                        g = fmaf(-t * (1.0f / 6.0f), g, 1.0f);
                        g = fmaf(-t * (1.0f / 5.0f), g, 1.0f);
                        g = fmaf(-t * (1.0f / 4.0f), g, 1.0f);
                        g = fmaf(-t * (1.0f / 3.0f), g, 1.0f);
                        g = fmaf(-t * 0.5f, g, 1.0f);
                        e[k * 5 + i] = t * g;
                    } else {
                        e[k * 5 + i] = __builtin_amdgcn_exp2f(-t);
                    }
                }
            }
        };
        float w[26];
        auto dot = [&](const float (&e)[25]) {
            float acc = 0.0f;
    #pragma unroll
            for (int q = 0; q < 25; ++q)
                acc = fmaf(e[q], w[q], acc);
            return acc;
        };
        float zc = 0.0f;
        bool bad = false;
        int cur = -1;  // window row start of w (the same for every thread of the block)
        for (int r = 0; r < nrow; ++r) {
            const int wy = s_wy[r];
            if (wy != cur) {
                float dz[25];
                zc = at(wy + 2, wx + 2);
                bad = false;
    #pragma unroll
                for (int q = 0; q < 25; ++q) {
                    const float z = at(wy + q / 5, wx + q % 5);
                    bad |= !isfinite(z);
                    dz[q] = z - zc;
                }
                // mirror transform per row (x), then per column (y):
                // component order per axis: sums 0+4, 1+3, 2 | differences 0-4, 1-3
                float t[25];
    #pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const float *d = &dz[k * 5];
                    t[k * 5 + 0] = d[0] + d[4];
                    t[k * 5 + 1] = d[1] + d[3];
                    t[k * 5 + 2] = d[2];
                    t[k * 5 + 3] = d[0] - d[4];
                    t[k * 5 + 4] = d[1] - d[3];
                }
                float sv[25];
    #pragma unroll
                for (int i = 0; i < 5; ++i) {
                    sv[0 * 5 + i] = t[0 * 5 + i] + t[4 * 5 + i];
                    sv[1 * 5 + i] = t[1 * 5 + i] + t[3 * 5 + i];
                    sv[2 * 5 + i] = t[2 * 5 + i];
                    sv[3 * 5 + i] = t[0 * 5 + i] - t[4 * 5 + i];
                    sv[4 * 5 + i] = t[1 * 5 + i] - t[3 * 5 + i];
                }
                // the blocks are read from the argument segment through scalar
                // loads here, once per window: an opaque pointer keeps the 178
                // values from being held in registers across the row loop
                cfloat *mb = (cfloat *)((const __attribute__((address_space(4))) char *)
                                            __builtin_amdgcn_kernarg_segment_ptr() +
                                        offsetof(KrigArgs, mb));
                asm volatile("" : "+s"(mb));
                float uv[25];
                float u25;
                // even-even: y components 0..2, x components 0..2, then the
                // unbiasedness row
    #pragma unroll
                for (int r = 0; r < 10; ++r) {
                    float acc = 0.0f;
    #pragma unroll
                    for (int c = 0; c < 9; ++c)
                        acc = fmaf(mb[r * 9 + c], sv[(c / 3) * 5 + c % 3], acc);
                    if (r < 9)
                        uv[(r / 3) * 5 + r % 3] = acc;
                    else
                        u25 = acc;
                }
                // even-odd: y 0..2, x 3..4
    #pragma unroll
                for (int r = 0; r < 6; ++r) {
                    float acc = 0.0f;
    #pragma unroll
                    for (int c = 0; c < 6; ++c)
                        acc = fmaf(mb[90 + r * 6 + c], sv[(c / 2) * 5 + 3 + c % 2], acc);
                    uv[(r / 2) * 5 + 3 + r % 2] = acc;
                }
                // odd-even: y 3..4, x 0..2
    #pragma unroll
                for (int r = 0; r < 6; ++r) {
                    float acc = 0.0f;
    #pragma unroll
                    for (int c = 0; c < 6; ++c)
                        acc = fmaf(mb[126 + r * 6 + c], sv[(3 + c / 3) * 5 + c % 3], acc);
                    uv[(3 + r / 3) * 5 + r % 3] = acc;
                }
                // odd-odd: y 3..4, x 3..4
    #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float acc = 0.0f;
    #pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc = fmaf(mb[162 + r * 4 + c], sv[(3 + c / 2) * 5 + 3 + c % 2], acc);
                    uv[(3 + r / 2) * 5 + 3 + r % 2] = acc;
                }
                // back to nodes: transpose of the mirror transform, y then x
    #pragma unroll
                for (int i = 0; i < 5; ++i) {
                    t[0 * 5 + i] = uv[0 * 5 + i] + uv[3 * 5 + i];
                    t[4 * 5 + i] = uv[0 * 5 + i] - uv[3 * 5 + i];
                    t[1 * 5 + i] = uv[1 * 5 + i] + uv[4 * 5 + i];
                    t[3 * 5 + i] = uv[1 * 5 + i] - uv[4 * 5 + i];
                    t[2 * 5 + i] = uv[2 * 5 + i];
                }
    #pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const float *y = &t[k * 5];
                    w[k * 5 + 0] = y[0] + y[3];
                    w[k * 5 + 4] = y[0] - y[3];
                    w[k * 5 + 1] = y[1] + y[4];
                    w[k * 5 + 3] = y[1] - y[4];
                    w[k * 5 + 2] = y[2];
                }
                w[25] = u25;
                cur = wy;
            }
            float v;
            if (bad) {
                // a non-finite neighbour: bilinear on the node's cell corners
                const int i0 = s_i0[c], i1 = s_i1[c], j0 = s_j0[r], j1 = s_j1[r];
                const float t = s_t[c], s = s_s[r];
                const float q00 = at(j0, i0), q10 = at(j0, i1);
                const float q01 = at(j1, i0), q11 = at(j1, i1);
                const float top = q00 + t * (q10 - q00);
                const float bot = q01 + t * (q11 - q01);
                v = top + s * (bot - top);
            } else {
                const float dv = s_dv[r];
                float acc;
                if (dv == dva) {
                    acc = dot(ca);
                } else if (dv == dvb) {
                    acc = dot(cb);
                } else if (fill_a) {
                    terms(ca, dv);
                    dva = dv;
                    fill_a = false;
                    acc = dot(ca);
                } else {
                    terms(cb, dv);
                    dvb = dv;
                    fill_a = true;
                    acc = dot(cb);
                }
                v = kSeries ? zc + (w[25] + acc) : zc + (w[25] - acc);
            }
            p.dst[(int64_t)(row0 + r) * p.dnx + col0 + c] = v;
        }
    };
    if (staged)
        walk(std::true_type{});
    else
        walk(std::false_type{});
}

// Inverse of the 26 x 26 kriging matrix for node spacing (dx, dy) and range a,
// by Gauss-Jordan elimination with partial pivoting in FP64.
bool kriging_inverse(double dx, double dy, double range, double *out)
{
    constexpr int n = 26;
    double A[n][2 * n];
    for (int pi = 0; pi < 25; ++pi) {
        for (int qi = 0; qi < 25; ++qi) {
            const double h = std::hypot((pi % 5 - qi % 5) * dx, (pi / 5 - qi / 5) * dy);
            A[pi][qi] = -std::expm1(-h / range);
        }
        A[pi][25] = 1.0;
        A[25][pi] = 1.0;
    }
    A[25][25] = 0.0;
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < n; ++k)
            A[r][n + k] = r == k ? 1.0 : 0.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col]))
                piv = r;
        if (!(std::fabs(A[piv][col]) > 0.0))
            return false;
        if (piv != col)
            for (int k = 0; k < 2 * n; ++k)
                std::swap(A[piv][k], A[col][k]);
        const double d = A[col][col];
        for (int k = 0; k < 2 * n; ++k)
            A[col][k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col || A[r][col] == 0.0)
                continue;
            const double f = A[r][col];
            for (int k = 0; k < 2 * n; ++k)
                A[r][k] -= f * A[col][k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < n; ++k)
            out[r * n + k] = A[r][n + k];
    return true;
}

// M = D^-1 T K^-1 T' D^-1 for the mirror transform T (per axis: rows
// a0+a4, a1+a3, a2, a0-a4, a1-a3; the unbiasedness entry kept) and D = T T',
// so that K^-1 = T' M T.  M is block diagonal over the parity classes; its
// blocks are packed as the kernel reads them.  Fails if an entry outside the
// blocks is not negligible (it is zero in exact arithmetic).
bool mirror_blocks(const double *kinv, float *out)
{
    static const double ax[5][5] = {{1, 0, 0, 0, 1},
                                    {0, 1, 0, 1, 0},
                                    {0, 0, 1, 0, 0},
                                    {1, 0, 0, 0, -1},
                                    {0, 1, 0, -1, 0}};
    static const double dax[5] = {2, 2, 1, 2, 2};
    double T[26][26] = {}, Dinv[26];
    for (int ky = 0; ky < 5; ++ky)
        for (int kx = 0; kx < 5; ++kx) {
            for (int k = 0; k < 5; ++k)
                for (int i = 0; i < 5; ++i)
                    T[ky * 5 + kx][k * 5 + i] = ax[ky][k] * ax[kx][i];
            Dinv[ky * 5 + kx] = 1.0 / (dax[ky] * dax[kx]);
        }
    T[25][25] = 1.0;
    Dinv[25] = 1.0;
    double A[26][26], M[26][26];  // A = K^-1 T'
    for (int r = 0; r < 26; ++r)
        for (int c = 0; c < 26; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 26; ++k)
                acc += kinv[r * 26 + k] * T[c][k];
            A[r][c] = acc;
        }
    double big = 0.0;
    for (int r = 0; r < 26; ++r)
        for (int c = 0; c < 26; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 26; ++k)
                acc += T[r][k] * A[k][c];
            M[r][c] = Dinv[r] * acc * Dinv[c];
            big = std::max(big, std::fabs(M[r][c]));
        }
    // parity class of a mirror-basis index: 0 even-even, 1 even-odd,
    // 2 odd-even, 3 odd-odd (the unbiasedness entry is even-even)
    auto cls = [](int q) { return q == 25 ? 0 : 2 * (q / 5 >= 3) + (q % 5 >= 3); };
    for (int r = 0; r < 26; ++r)
        for (int c = 0; c < 26; ++c)
            if (cls(r) != cls(c) && !(std::fabs(M[r][c]) <= 1e-9 * big))
                return false;
    // members of each class in the kernel's order
    int ee[10], eo[6], oe[6], oo[4];
    for (int r = 0; r < 9; ++r)
        ee[r] = (r / 3) * 5 + r % 3;
    ee[9] = 25;
    for (int r = 0; r < 6; ++r) {
        eo[r] = (r / 2) * 5 + 3 + r % 2;
        oe[r] = (3 + r / 3) * 5 + r % 3;
    }
    for (int r = 0; r < 4; ++r)
        oo[r] = (3 + r / 2) * 5 + 3 + r % 2;
    int o = 0;
    for (int r = 0; r < 10; ++r)
        for (int c = 0; c < 9; ++c)
            out[o++] = (float)M[ee[r]][ee[c]];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c)
            out[o++] = (float)M[eo[r]][eo[c]];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c)
            out[o++] = (float)M[oe[r]][oe[c]];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            out[o++] = (float)M[oo[r]][oo[c]];
    return o == kBlockFloats;
}

// The last few inverses, keyed by (dx, dy, range): a resample loop over
// tiles of one survey pays the elimination once.
struct KrigCache {
    std::mutex mu;
    struct Entry {
        double dx, dy, range;
        double kinv[26 * 26];
    } e[8];
    int used = 0, next = 0;
};

bool cached_inverse(double dx, double dy, double range, double *out)
{
    static KrigCache cache;
    {
        std::lock_guard<std::mutex> lk(cache.mu);
        for (int i = 0; i < cache.used; ++i) {
            const KrigCache::Entry &e = cache.e[i];
            if (e.dx == dx && e.dy == dy && e.range == range) {
                std::memcpy(out, e.kinv, sizeof(e.kinv));
                return true;
            }
        }
    }
    if (!kriging_inverse(dx, dy, range, out))
        return false;
    std::lock_guard<std::mutex> lk(cache.mu);
    KrigCache::Entry &e = cache.e[cache.next];
    e.dx = dx;
    e.dy = dy;
    e.range = range;
    std::memcpy(e.kinv, out, sizeof(e.kinv));
    cache.next = (cache.next + 1) % 8;
    cache.used = std::min(cache.used + 1, 8);
    return true;
}

}  // namespace

auv_status launch_kriging(const float *src, const auv_grid_desc &s, float *dst,
                          const auv_grid_desc &d, double range, hipStream_t st)
{
    if (!(range > 0.0) || !std::isfinite(range))
        return fail(AUV_ERR_INVALID, "range must be positive and finite");
    if (s.nx < 5 || s.ny < 5)  // no 5 x 5 neighbourhood: every node is bilinear
        return launch_bilinear(src, s, dst, d, st);
    KrigArgs p;
    std::memset(&p, 0, sizeof(p));
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
    p.fdx = (float)s.dx;
    p.fdy = (float)s.dy;
    // a window node lies at most 4 spacings per axis from the destination
    // point (the point is clamped into the grid, the window moved in at edges)
    const double hmax = 4.0 * std::hypot(s.dx, s.dy);
    const bool series = hmax / range <= 0.25;
    if (range > kMaxRangeSpacings * std::max(s.dx, s.dy))
        return fail(AUV_ERR_RANGE, "kriging range above 1e4 source spacings");
    const double l = (series ? 1.0 : 1.4426950408889634) / range;
    p.c2 = (float)(l * l);
    double kinv[26 * 26];
    if (!cached_inverse(s.dx, s.dy, range, kinv))
        return fail(AUV_ERR_INVALID, "singular kriging system for this spacing and range");
    if (!mirror_blocks(kinv, p.mb))
        return fail(AUV_ERR_INVALID, "kriging inverse lost its mirror symmetry (range far outside the node spacing)");
    // more rows per block reuse more covariance terms, but a small grid needs
    // the blocks: halve from kKrigRows (down to 8) while under 1024 blocks
    const int64_t ncb = (d.nx + kKrigCols - 1) / kKrigCols;
    p.rows = kKrigRows;
    while (p.rows > 8 && ncb * ((d.ny + p.rows - 1) / p.rows) < 1024)
        p.rows /= 2;
    const dim3 grid((unsigned)ncb, (unsigned)((d.ny + p.rows - 1) / p.rows));
    if (series)
        k_kriging<true><<<grid, kKrigCols, 0, st>>>(p);
    else
        k_kriging<false><<<grid, kKrigCols, 0, st>>>(p);
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
