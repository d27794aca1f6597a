// Destination-node to source-index mapping shared by the grid resamplers.
#pragma once
#include "auv_internal.hpp"

#include <cmath>

namespace auv {

// A destination node at x = x0d + (j + 1/2) dd maps to the source index
// coordinate u = (x - x0s) / ds - 1/2, clamped to [0, ns - 1]: i0 = floor(u),
// i1 = min(i0 + 1, ns - 1), t = u - i0.  Computed in FP64 in the order of its
// definition (no contraction), so the corner choice is exact.
struct Axis {
    int i0, i1;
    float t;
    double u;
};

__device__ inline Axis axis_of(double x0d, double dd, int j, double x0s, double ds, int ns)
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
    a.u = u;
    return a;
}

// Copy the source rectangle [jl, jl + sh) x [il, il + sw) into s_dst
// (row-major, pitch sw) with nthreads threads: element e = t + k nthreads
// walks (row, column) incrementally, one division per thread in all.
__device__ inline void stage_rect(const float *__restrict__ src, int snx, int jl, int il,
                                  int sw, int sh, float *s_dst, int nthreads)
{
    const int t = (int)threadIdx.x;
    const int n = sw * sh;
    if (t >= n)
        return;
    int r = t / sw, c = t - r * sw;
    const int dr = nthreads / sw, dc = nthreads - dr * sw;
    const float *row = src + (int64_t)(jl + r) * snx + il;
    for (int e = t; e < n; e += nthreads) {
        s_dst[e] = row[c];
        c += dc;
        int step = dr;
        if (c >= sw) {
            c -= sw;
            ++step;
        }
        r += step;
        row += (int64_t)step * snx;
    }
}

}  // namespace auv
