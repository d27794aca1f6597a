// Bilinear resample of one grid onto another (Sec. III-A of the paper).
//
// Each thread produces four consecutive destination nodes of one row and
// writes them with one 16-byte store when the row allows it.  The source
// index coordinate of a node is computed in FP64 with the same operations, in
// the same order, as its definition (no contraction), so the corner choice is
// exact; the blend itself is FP32 in lerp form (top, bottom, then vertical),
// which keeps constants exact and lets a NaN corner propagate: a hole.
#include "auv_internal.hpp"

#include <algorithm>
#include <cmath>

namespace auv {

namespace {

struct Axis {
    int i0, i1;
    float t;
};

__device__ inline Axis axis_of(double x0d, double dd, int j, double x0s, double ds,
                               int ns)
{
#pragma clang fp contract(off)
    const double xd = x0d + ((double)j + 0.5) * dd;
    double u = (xd - x0s) / ds - 0.5;
    u = u < 0.0 ? 0.0 : u;
    u = u > (double)(ns - 1) ? (double)(ns - 1) : u;
    const double f = floor(u);
    Axis a;
    a.i0 = (int)f;
    a.i1 = a.i0 + 1 < ns ? a.i0 + 1 : ns - 1;
    a.t = (float)(u - f);
    return a;
}

struct BilArgs {
    const float *src;
    float *dst;
    double sx0, sy0, sdx, sdy;
    double dx0, dy0, ddx, ddy;
    int snx, sny, dnx, dny;
    int groups;  // 4-node groups per destination row
};

__global__ __launch_bounds__(256) void k_bilinear(BilArgs p)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)p.groups * p.dny;
    if (g >= total)
        return;
    const int row = (int)(g / p.groups);
    const int c0 = (int)(g - (int64_t)row * p.groups) * 4;
    const Axis ay = axis_of(p.dy0, p.ddy, row, p.sy0, p.sdy, p.sny);
    const float *r0 = p.src + (int64_t)ay.i0 * p.snx;
    const float *r1 = p.src + (int64_t)ay.i1 * p.snx;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = min(c0 + k, p.dnx - 1);
        const Axis ax = axis_of(p.dx0, p.ddx, c, p.sx0, p.sdx, p.snx);
        const float q00 = r0[ax.i0], q10 = r0[ax.i1];
        const float q01 = r1[ax.i0], q11 = r1[ax.i1];
        const float top = q00 + ax.t * (q10 - q00);
        const float bot = q01 + ax.t * (q11 - q01);
        v[k] = top + ay.t * (bot - top);
    }
    float *out = p.dst + (int64_t)row * p.dnx + c0;
    if (c0 + 4 <= p.dnx && ((reinterpret_cast<uintptr_t>(out) & 15) == 0)) {
        *reinterpret_cast<float4 *>(out) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        for (int k = 0; k < 4 && c0 + k < p.dnx; ++k)
            out[k] = v[k];
    }
}

}  // namespace

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
    p.groups = (d.nx + 3) / 4;
    const int64_t total = (int64_t)p.groups * d.ny;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > INT32_MAX)
        return fail(AUV_ERR_RANGE, "destination grid too large");
    k_bilinear<<<(unsigned)blocks, 256, 0, st>>>(p);
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
