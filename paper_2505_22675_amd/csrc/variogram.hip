// Empirical semivariogram of a grid along its axes, and the exponential
// variogram fit that gives kriging (Sec. III-C) its range.
//
//   k_vario_partial  one block per (axis, lag, band of rows): FP64 sum of the
//                    squared differences of the pairs at that lag with both
//                    values finite, and their count
//   k_vario_final    one block per (axis, lag): the bands' partials summed in
//                    band order
// Every sum runs in a fixed order (no atomics), so the result does not depend
// on timing.  The fit is host arithmetic on a few dozen points.
#include "auv_internal.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace auv {
namespace {

constexpr int kVThreads = 256;
constexpr int kMaxBands = 128;
constexpr int kMaxLags = 1024;

struct VPart {
    double sum;
    long long cnt;
};

__device__ inline void block_sum(double &s, long long &c, VPart *lds)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s += __shfl_xor(s, d, 64);
        c += __shfl_xor(c, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        lds[w] = VPart{s, c};
    __syncthreads();
    if (threadIdx.x == 0) {
        s = 0.0;
        c = 0;
        for (int i = 0; i < kVThreads / 64; ++i) {
            s += lds[i].sum;
            c += lds[i].cnt;
        }
    }
}

// grid: (bands, nlags, 2 axes).  Band b takes rows [b * ny / bands, (b+1) * ny / bands).
__global__ __launch_bounds__(kVThreads) void k_vario_partial(const float *__restrict__ src,
                                                             int nx, int ny, int nlags,
                                                             VPart *__restrict__ part)
{
    __shared__ VPart lds[kVThreads / 64];
    const int bands = gridDim.x, band = blockIdx.x, k = blockIdx.y + 1, axis = blockIdx.z;
    const int r0 = (int)((long long)band * ny / bands);
    const int r1 = (int)((long long)(band + 1) * ny / bands);
    double s = 0.0;
    long long c = 0;
    for (int a = r0; a < r1; ++a) {
        const float *row = src + (size_t)a * nx;
        if (axis == 0) {
            for (int b = threadIdx.x; b + k < nx; b += kVThreads) {
                const float z1 = row[b], z2 = row[b + k];
                if (isfinite(z1) && isfinite(z2)) {
                    const double d = (double)z1 - (double)z2;
                    s += d * d;
                    c += 1;
                }
            }
        } else if (a + k < ny) {
            const float *row2 = row + (size_t)k * nx;
            for (int b = threadIdx.x; b < nx; b += kVThreads) {
                const float z1 = row[b], z2 = row2[b];
                if (isfinite(z1) && isfinite(z2)) {
                    const double d = (double)z1 - (double)z2;
                    s += d * d;
                    c += 1;
                }
            }
        }
    }
    block_sum(s, c, lds);
    if (threadIdx.x == 0)
        part[((size_t)axis * nlags + (k - 1)) * bands + band] = VPart{s, c};
}

// grid: (nlags * 2): out[axis * nlags + lag] = sum over bands, in band order
// within each thread and in thread order across the block.
__global__ __launch_bounds__(kVThreads) void k_vario_final(const VPart *__restrict__ part,
                                                           int bands, VPart *__restrict__ out)
{
    __shared__ VPart lds[kVThreads / 64];
    const VPart *p = part + (size_t)blockIdx.x * bands;
    double s = 0.0;
    long long c = 0;
    for (int i = threadIdx.x; i < bands; i += kVThreads) {
        s += p[i].sum;
        c += p[i].cnt;
    }
    block_sum(s, c, lds);
    if (threadIdx.x == 0)
        out[blockIdx.x] = VPart{s, c};
}

int bands_for(int ny) { return std::max(1, std::min(ny, kMaxBands)); }

size_t vario_ws_bytes(int ny, int nlags)
{
    const size_t parts = (size_t)2 * nlags * bands_for(ny) * sizeof(VPart);
    return ((parts + 255) & ~size_t(255)) + (size_t)2 * nlags * sizeof(VPart);
}

auv_status check_vario_args(const auv_grid_desc *s, int32_t nlags)
{
    if (!s || s->nx < 1 || s->ny < 1)
        return fail(AUV_ERR_INVALID, "bad grid descriptor");
    if (!(s->dx > 0.0) || !(s->dy > 0.0) || !std::isfinite(s->dx) || !std::isfinite(s->dy))
        return fail(AUV_ERR_INVALID, "grid spacing must be finite and positive");
    if (nlags < 1 || nlags > kMaxLags)
        return fail(AUV_ERR_INVALID, "nlags must be in [1, 1024]");
    return AUV_OK;
}

// Weighted residual of the exponential model at range a, the sill at its
// least-squares value for that range.
double exp_residual(const double *h, const double *g, const double *w, int n, double a,
                    double *sill)
{
    double sgf = 0.0, sff = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!(w[j] > 0.0) || !std::isfinite(g[j]) || !(h[j] > 0.0))
            continue;
        const double f = -std::expm1(-h[j] / a);
        sgf += w[j] * g[j] * f;
        sff += w[j] * f * f;
    }
    const double c = sff > 0.0 ? sgf / sff : 0.0;
    if (sill)
        *sill = c;
    // the residual summed term by term (the expanded form cancels near a
    // perfect fit and would blur the minimum)
    double r = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!(w[j] > 0.0) || !std::isfinite(g[j]) || !(h[j] > 0.0))
            continue;
        const double e = g[j] + c * std::expm1(-h[j] / a);
        r += w[j] * e * e;
    }
    return r;
}

}  // namespace
}  // namespace auv

using namespace auv;

extern "C" {

auv_status auv_variogram_workspace_size(const auv_grid_desc *s, int32_t nlags, size_t *bytes)
{
    if (!bytes)
        return fail(AUV_ERR_INVALID, "bytes is null");
    const auv_status st = check_vario_args(s, nlags);
    if (st != AUV_OK)
        return st;
    *bytes = vario_ws_bytes(s->ny, nlags);
    return AUV_OK;
}

auv_status auv_variogram(const float *src, const auv_grid_desc *s, int32_t nlags, void *ws,
                         size_t ws_bytes, double *gamma_x, double *gamma_y, int64_t *pairs_x,
                         int64_t *pairs_y, auv_stream stream)
{
    auv_status st = check_vario_args(s, nlags);
    if (st != AUV_OK)
        return st;
    if (!src || !ws || !gamma_x || !gamma_y)
        return fail(AUV_ERR_INVALID, "null argument");
    if (ws_bytes < vario_ws_bytes(s->ny, nlags))
        return fail(AUV_ERR_BUDGET, "workspace smaller than auv_variogram_workspace_size");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(AUV_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int bands = bands_for(s->ny);
    VPart *part = static_cast<VPart *>(ws);
    const size_t parts = (size_t)2 * nlags * bands * sizeof(VPart);
    VPart *out = reinterpret_cast<VPart *>(static_cast<char *>(ws) + ((parts + 255) & ~size_t(255)));
    k_vario_partial<<<dim3((unsigned)bands, (unsigned)nlags, 2), kVThreads, 0, hs>>>(
        src, s->nx, s->ny, nlags, part);
    k_vario_final<<<(unsigned)(2 * nlags), kVThreads, 0, hs>>>(part, bands, out);
    AUV_HIP(hipGetLastError());
    std::vector<VPart> host(2 * (size_t)nlags);
    AUV_HIP(hipMemcpyAsync(host.data(), out, sizeof(VPart) * host.size(), hipMemcpyDeviceToHost,
                           hs));
    AUV_HIP(hipStreamSynchronize(hs));
    for (int k = 0; k < nlags; ++k) {
        const VPart px = host[k], py = host[nlags + k];
        gamma_x[k] = px.cnt > 0 ? px.sum / (2.0 * (double)px.cnt) : NAN;
        gamma_y[k] = py.cnt > 0 ? py.sum / (2.0 * (double)py.cnt) : NAN;
        if (pairs_x)
            pairs_x[k] = px.cnt;
        if (pairs_y)
            pairs_y[k] = py.cnt;
    }
    return AUV_OK;
}

auv_status auv_fit_exponential(const double *h, const double *gamma, const double *w, int32_t n,
                               double *range, double *sill)
{
    if (!h || !gamma || !w || !range || n < 1)
        return fail(AUV_ERR_INVALID, "null argument or no point");
    double hmin = INFINITY, hmax = 0.0;
    int used = 0;
    for (int j = 0; j < n; ++j) {
        if (!(w[j] > 0.0) || !std::isfinite(gamma[j]) || !(h[j] > 0.0))
            continue;
        hmin = std::min(hmin, h[j]);
        hmax = std::max(hmax, h[j]);
        ++used;
    }
    if (used < 2)
        return fail(AUV_ERR_INVALID, "fewer than two usable points");
    // log-spaced scan of the range, then golden-section search between the
    // neighbours of the best scanned value
    const int m = 4001;
    const double l0 = std::log(hmin / 100.0), l1 = std::log(1000.0 * hmax);
    auto at = [&](int i) { return l0 + (l1 - l0) * (double)i / (double)(m - 1); };
    int best = 0;
    double best_r = INFINITY;
    for (int i = 0; i < m; ++i) {
        const double r = exp_residual(h, gamma, w, n, std::exp(at(i)), nullptr);
        if (r < best_r) {
            best_r = r;
            best = i;
        }
    }
    double c = 0.0;
    if (best == 0 || best == m - 1) {
        *range = std::exp(at(best));
        exp_residual(h, gamma, w, n, *range, &c);
        if (sill)
            *sill = c;
        return fail(AUV_ERR_RANGE, "no sill inside [min lag / 100, 1000 max lag]");
    }
    const double phi = 0.5 * (std::sqrt(5.0) - 1.0);
    double lo = at(best - 1), hi = at(best + 1);
    double p = hi - phi * (hi - lo), q = lo + phi * (hi - lo);
    double rp = exp_residual(h, gamma, w, n, std::exp(p), nullptr);
    double rq = exp_residual(h, gamma, w, n, std::exp(q), nullptr);
    for (int it = 0; it < 120; ++it) {
        if (rp <= rq) {
            hi = q;
            q = p;
            rq = rp;
            p = hi - phi * (hi - lo);
            rp = exp_residual(h, gamma, w, n, std::exp(p), nullptr);
        } else {
            lo = p;
            p = q;
            rp = rq;
            q = lo + phi * (hi - lo);
            rq = exp_residual(h, gamma, w, n, std::exp(q), nullptr);
        }
    }
    *range = std::exp(0.5 * (lo + hi));
    exp_residual(h, gamma, w, n, *range, &c);
    if (sill)
        *sill = c;
    return AUV_OK;
}

}  // extern "C"
