// C ABI of libauvgrid: argument validation, handles, workspace carve-up and
// kernel launches.  Every entry point validates synchronously and only
// enqueues device work on the caller's stream.
#include "auv_internal.hpp"
#include "idw_dense_impl.hpp"

#include <cmath>
#include <cstring>
#include <new>
#include <string>

namespace auv {

namespace {
thread_local std::string g_last_error;
}

auv_status fail(auv_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

auv_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return AUV_ERR_HIP;
}

namespace {

// Reject pointers the device cannot dereference (pageable host memory, null,
// wild values) before any kernel reads them.
auv_status check_device_ptr(const void *p, const char *name)
{
    if (!p)
        return fail(AUV_ERR_INVALID, std::string(name) + " is null");
    hipPointerAttribute_t attr;
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky error of the query
        return fail(AUV_ERR_INVALID, std::string(name) + " is not device memory");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged &&
        attr.type != hipMemoryTypeHost)
        return fail(AUV_ERR_INVALID, std::string(name) + " is not device-accessible");
    return AUV_OK;
}

#define AUV_TRY(expr)                                                          \
    do {                                                                       \
        auv_status s_ = (expr);                                                \
        if (s_ != AUV_OK)                                                      \
            return s_;                                                         \
    } while (0)

auv_status check_desc(const auv_grid_desc *d)
{
    if (!d)
        return fail(AUV_ERR_INVALID, "grid descriptor is null");
    if (d->nx < 1 || d->ny < 1)
        return fail(AUV_ERR_INVALID, "grid needs nx, ny >= 1");
    if (!(d->dx > 0.0) || !(d->dy > 0.0) || !std::isfinite(d->dx) ||
        !std::isfinite(d->dy) || !std::isfinite(d->x0) || !std::isfinite(d->y0))
        return fail(AUV_ERR_INVALID, "grid origin/spacing must be finite, spacing > 0");
    if ((double)d->nx * d->dx >= 16384.0 || (double)d->ny * d->dy >= 16384.0)
        return fail(AUV_ERR_RANGE, "grid extent must stay below 16384 m per axis");
    return AUV_OK;
}

int32_t node_lattice_host(int32_t j, double d)
{
    const double u = ((double)j + 0.5) * d;
    return (int32_t)std::nearbyint(u * kLatticePerMetre);
}

}  // namespace

auv_status bin_into(const auv_grid *grid, const double *x, const double *y, const double *z,
                    int64_t n, double radius, int32_t bin_log2, void *ws, size_t ws_bytes,
                    hipStream_t stream, auv_bins *b)
{
    if (!grid)
        return fail(AUV_ERR_INVALID, "grid is null");
    if (n < 0 || n >= INT32_MAX)
        return fail(AUV_ERR_INVALID, "n must be in [0, 2^31-1)");
    BinGeom geom;
    AUV_TRY(bin_geometry(grid, radius, bin_log2, &geom));
    BinWorkspace w;
    const size_t need = bin_workspace_layout(n, geom, static_cast<char *>(ws), &w);
    if (ws_bytes < need)
        return fail(AUV_ERR_BUDGET, "workspace smaller than auv_bin_workspace_size");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(AUV_ERR_INVALID, "workspace must be 256-byte aligned");
    AUV_TRY(check_device_ptr(ws, "workspace"));
    if (n > 0) {
        AUV_TRY(check_device_ptr(x, "x"));
        AUV_TRY(check_device_ptr(y, "y"));
        AUV_TRY(check_device_ptr(z, "z"));
    }
    AUV_TRY(launch_binning(grid, geom, x, y, z, n, w, stream));
    b->v.cell_start = w.cell_start;
    b->v.X = w.X;
    b->v.Y = w.Y;
    b->v.res = w.res;
    b->v.z = w.z;
    b->v.idx = w.idx;
    b->v.rec = w.rec;
    {
        int bits = 1;
        while (bits < 31 && (int64_t(1) << bits) < n)
            ++bits;
        b->v.idx_bits = bits;
    }
    b->v.nbx = geom.nbx;
    b->v.nby = geom.nby;
    b->v.halo = geom.halo;
    b->v.bin_log2 = geom.s;
    b->v.R = geom.R;
    b->grid = grid;
    b->radius = radius;
    b->n = n;
    b->stats = w.stats;
    b->ws = ws;
    b->ws_bytes = ws_bytes;
    return AUV_OK;
}

}  // namespace auv

using namespace auv;

extern "C" {

const char *auv_version(void) { return "auvgrid 0.1 (gfx950)"; }

const char *auv_last_error(void) { return g_last_error.c_str(); }

auv_status auv_grid_create(const auv_grid_desc *desc, auv_grid **out)
{
    if (!out)
        return fail(AUV_ERR_INVALID, "out is null");
    *out = nullptr;
    AUV_TRY(check_desc(desc));
    auv_grid *g = new (std::nothrow) auv_grid;
    if (!g)
        return fail(AUV_ERR_INVALID, "out of host memory");
    g->d = *desc;
    g->x_last = node_lattice_host(desc->nx - 1, desc->dx);
    g->y_last = node_lattice_host(desc->ny - 1, desc->dy);
    *out = g;
    return AUV_OK;
}

void auv_grid_destroy(auv_grid *grid) { delete grid; }

auv_status auv_bin_workspace_size(const auv_grid *grid, int64_t n, double radius,
                                  int32_t bin_log2, size_t *bytes)
{
    if (!grid || !bytes)
        return fail(AUV_ERR_INVALID, "null argument");
    if (n < 0 || n >= INT32_MAX)
        return fail(AUV_ERR_INVALID, "n must be in [0, 2^31-1)");
    BinGeom geom;
    AUV_TRY(bin_geometry(grid, radius, bin_log2, &geom));
    *bytes = bin_workspace_layout(n, geom, nullptr, nullptr);
    return AUV_OK;
}

auv_status auv_bin_points(const auv_grid *grid, const double *x, const double *y,
                          const double *z, int64_t n, double radius,
                          int32_t bin_log2, void *ws, size_t ws_bytes,
                          auv_stream stream, auv_bins **out)
{
    if (!out)
        return fail(AUV_ERR_INVALID, "out is null");
    *out = nullptr;
    auv_bins *b = new (std::nothrow) auv_bins;
    if (!b)
        return fail(AUV_ERR_INVALID, "out of host memory");
    const auv_status st = bin_into(grid, x, y, z, n, radius, bin_log2, ws, ws_bytes,
                                   static_cast<hipStream_t>(stream), b);
    if (st != AUV_OK) {
        delete b;
        return st;
    }
    *out = b;
    return AUV_OK;
}

auv_status auv_bins_info(const auv_bins *bins, int32_t *nbx, int32_t *nby,
                         int32_t *halo, int32_t *bin_log2)
{
    if (!bins)
        return fail(AUV_ERR_INVALID, "bins is null");
    if (nbx)
        *nbx = bins->v.nbx;
    if (nby)
        *nby = bins->v.nby;
    if (halo)
        *halo = bins->v.halo;
    if (bin_log2)
        *bin_log2 = bins->v.bin_log2;
    return AUV_OK;
}

auv_status auv_bins_export(const auv_bins *bins, int32_t *cell_start, int32_t *perm,
                           int64_t *counts, auv_stream stream)
{
    if (!bins)
        return fail(AUV_ERR_INVALID, "bins is null");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t c[4] = {0, 0, 0, 0};
    AUV_HIP(hipMemcpyAsync(c, bins->stats, sizeof(c), hipMemcpyDeviceToHost, st));
    AUV_HIP(hipStreamSynchronize(st));
    const int64_t nb = (int64_t)bins->v.nbx * bins->v.nby;
    if (cell_start) {
        AUV_TRY(check_device_ptr(cell_start, "cell_start"));
        AUV_HIP(hipMemcpyAsync(cell_start, bins->v.cell_start, sizeof(int32_t) * (nb + 1),
                               hipMemcpyDeviceToDevice, st));
    }
    if (perm && c[0] > 0) {
        AUV_TRY(check_device_ptr(perm, "perm"));
        AUV_HIP(hipMemcpyAsync(perm, bins->v.idx, sizeof(int32_t) * c[0],
                               hipMemcpyDeviceToDevice, st));
    }
    if (counts) {
        counts[0] = c[0];
        counts[1] = c[1];
        counts[2] = c[2];
    }
    AUV_HIP(hipStreamSynchronize(st));
    return AUV_OK;
}

void auv_bins_destroy(auv_bins *bins) { delete bins; }

static auv_status idw_common(const auv_grid *grid, const auv_bins *bins,
                             double radius, IdwArgs *a)
{
    if (!grid || !bins)
        return fail(AUV_ERR_INVALID, "grid or bins is null");
    if (bins->grid != grid)
        return fail(AUV_ERR_INVALID, "bins were built for another grid");
    if (!(radius > 0.0) || !(radius <= 256.0))
        return fail(AUV_ERR_INVALID, "radius must be in (0, 256] metres");
    const double Rd = std::rint(radius * kLatticePerMetre);
    if (Rd < 1.0 || Rd > (double)bins->v.R)
        return fail(AUV_ERR_INVALID, "radius exceeds the radius the bins were built for");
    std::memset(a, 0, sizeof(*a));
    a->dx = grid->d.dx;
    a->dy = grid->d.dy;
    a->nx = grid->d.nx;
    a->ny = grid->d.ny;
    a->R = (int32_t)Rd;
    a->R_stage = (int32_t)Rd;
    a->inv_r2 = (float)(1.0 / (Rd * Rd));
    a->r2f = (float)(radius * radius);
    a->x0 = grid->d.x0;
    a->y0 = grid->d.y0;
    return AUV_OK;
}

auv_status auv_interp_idw(const auv_grid *grid, const auv_bins *bins,
                          const auv_idw_params *params, float *z_out,
                          int32_t *cnt_out, int32_t *nn_idx_out, float *nn_z_out,
                          auv_stream stream)
{
    if (!params)
        return fail(AUV_ERR_INVALID, "params is null");
    if (!(params->power > 0.0) || !(params->power <= 64.0))
        return fail(AUV_ERR_INVALID, "power must be in (0, 64]");
    if (params->min_pts < 0 || params->max_pts < 0)
        return fail(AUV_ERR_INVALID, "min_pts/max_pts must be >= 0");
    if (params->algo < AUV_ALGO_AUTO || params->algo > AUV_ALGO_SPAN)
        return fail(AUV_ERR_INVALID, "unknown algo");
    if (params->precision < AUV_P_FP32_REBASE || params->precision > AUV_P_FP32_ABSOLUTE)
        return fail(AUV_ERR_INVALID, "unknown precision variant");
    IdwArgs a;
    AUV_TRY(idw_common(grid, bins, params->radius, &a));
    if (params->precision != AUV_P_FP32_REBASE) {
        // the variants' rounded distances may admit soundings slightly beyond
        // the radius: search one metre further (clamped to the bin domain)
        a.R_stage = a.R + (int32_t)kLatticePerMetre;
    }
    AUV_TRY(check_device_ptr(z_out, "z_out"));
    if (cnt_out)
        AUV_TRY(check_device_ptr(cnt_out, "cnt_out"));
    if (nn_idx_out)
        AUV_TRY(check_device_ptr(nn_idx_out, "nn_idx_out"));
    if (nn_z_out)
        AUV_TRY(check_device_ptr(nn_z_out, "nn_z_out"));
    a.power = (float)params->power;
    a.min_pts = params->min_pts;
    a.max_pts = params->max_pts;
    a.precision = params->precision;
    a.mode = (nn_idx_out || nn_z_out) ? 3 : 1;
    {
        // expected soundings per disk, from the input count over the grid
        // grown by the radius
        const double r = params->radius;
        const double area = (grid->d.nx * grid->d.dx + 2 * r) * (grid->d.ny * grid->d.dy + 2 * r);
        const double lambda = (double)bins->n / area * 3.141592653589793 * r * r;
        const bool dense_ok = params->max_pts >= 1 && params->max_pts <= 32 &&
                              params->precision == AUV_P_FP32_REBASE &&
                              dense::dense_key_ok(a.R, bins->v.idx_bits);
        if (params->algo == AUV_ALGO_DENSE && !dense_ok)
            return fail(AUV_ERR_INVALID,
                        "the dense form needs 1 <= max_pts <= 32, AUV_P_FP32_REBASE and "
                        "(R^2 << index bits) below 2^62");
        a.dense = params->algo == AUV_ALGO_DENSE ||
                  (params->algo == AUV_ALGO_AUTO && dense_ok && lambda >= 0.5 * params->max_pts);
        a.span = params->algo == AUV_ALGO_SPAN;
    }
    a.z_out = z_out;
    a.cnt_out = cnt_out;
    a.nn_idx_out = nn_idx_out;
    a.nn_z_out = nn_z_out;
    return launch_idw(bins->v, a, static_cast<hipStream_t>(stream));
}

auv_status auv_interp_nearest(const auv_grid *grid, const auv_bins *bins,
                              double radius, int32_t *idx_out, float *z_out,
                              auv_stream stream)
{
    IdwArgs a;
    AUV_TRY(idw_common(grid, bins, radius, &a));
    AUV_TRY(check_device_ptr(idx_out, "idx_out"));
    if (z_out)
        AUV_TRY(check_device_ptr(z_out, "z_out"));
    a.power = 2.0f;
    a.mode = 2;
    a.nn_idx_out = idx_out;
    a.nn_z_out = z_out;
    return launch_idw(bins->v, a, static_cast<hipStream_t>(stream));
}

auv_status auv_resample_bilinear(const float *src, const auv_grid_desc *s, float *dst,
                                 const auv_grid_desc *d, auv_stream stream)
{
    AUV_TRY(check_desc(s));
    AUV_TRY(check_desc(d));
    AUV_TRY(check_device_ptr(src, "src"));
    AUV_TRY(check_device_ptr(dst, "dst"));
    return launch_bilinear(src, *s, dst, *d, static_cast<hipStream_t>(stream));
}

auv_status auv_resample_bicubic(const float *src, const auv_grid_desc *s, float *dst,
                                const auv_grid_desc *d, auv_stream stream)
{
    AUV_TRY(check_desc(s));
    AUV_TRY(check_desc(d));
    AUV_TRY(check_device_ptr(src, "src"));
    AUV_TRY(check_device_ptr(dst, "dst"));
    return launch_bicubic(src, *s, dst, *d, static_cast<hipStream_t>(stream));
}

auv_status auv_resample_kriging(const float *src, const auv_grid_desc *s, float *dst,
                                const auv_grid_desc *d, double range, auv_stream stream)
{
    AUV_TRY(check_desc(s));
    AUV_TRY(check_desc(d));
    AUV_TRY(check_device_ptr(src, "src"));
    AUV_TRY(check_device_ptr(dst, "dst"));
    return launch_kriging(src, *s, dst, *d, range, static_cast<hipStream_t>(stream));
}

}  // extern "C"
