// Internal declarations shared by the HIP translation units of libauvgrid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "auvgrid.h"

namespace auv {

// Lattice: 2^16 units per metre, relative to the grid's lower-left corner.
constexpr double kLatticePerMetre = 65536.0;
constexpr int kLatticeLog2 = 16;
// Residual (sounding position minus its lattice point) is stored as a signed
// 16-bit fixed-point number of 2^-15 lattice units.
constexpr float kResidualUnit = 1.0f / 32768.0f;

// Thread-local error message behind auv_last_error().
auv_status fail(auv_status st, const std::string &msg);
auv_status hip_fail(hipError_t e, const char *what);

#define AUV_TRY_S(expr)                                                        \
    do {                                                                       \
        auv_status s_ = (expr);                                                \
        if (s_ != AUV_OK)                                                      \
            return s_;                                                         \
    } while (0)

#define AUV_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::auv::hip_fail(e_, #call);                                 \
    } while (0)

}  // namespace auv

// Validated grid plus the lattice coordinates of its extreme nodes.
struct auv_grid {
    auv_grid_desc d;
    int32_t x_last;  // lattice X of node column nx-1
    int32_t y_last;  // lattice Y of node row ny-1
};

// Device view of binned soundings.  Binned position k (0 <= k < n_binned)
// holds the k-th sounding in (bin id, original index) order.
struct auv_bin_view {
    const int32_t *cell_start;  // [nbx*nby + 1]
    const int32_t *X;           // lattice x
    const int32_t *Y;           // lattice y
    const uint32_t *res;        // packed residuals: low 16 bits x, high 16 bits y
    const float *z;             // depth rounded to float
    const int32_t *idx;         // original index (perm)
    const int4 *rec;            // per original index: X, Y, residuals, depth bits
    int32_t nbx, nby, halo, bin_log2;
    int32_t idx_bits;           // bits of the largest original index
    int32_t R;                  // lattice radius the bins were built for
};

struct auv_bins {
    auv_bin_view v;
    const auv_grid *grid;
    double radius;
    int64_t n;                  // soundings given
    int64_t *stats;             // device [4]: binned, invalid, outside, big bins
    void *ws;
    size_t ws_bytes;
};

namespace auv {

// Bin geometry shared by the workspace query and the binning itself.
struct BinGeom {
    int32_t R;      // lattice radius
    int32_t s;      // bin_log2
    int32_t halo;   // bins added on each side
    int32_t nbx, nby;
};
auv_status bin_geometry(const auv_grid *g, double radius, int32_t bin_log2,
                        BinGeom *out);
int32_t default_bin_log2(int32_t R);

// Workspace carve-up of auv_bin_points.
struct BinWorkspace {
    int32_t *counts;      // [nb]
    int32_t *cell_start;  // [nb + 1]
    int32_t *partials;    // scan partials
    int32_t *key;         // [n] bin id per input sounding (or -1)
    int32_t *slot;        // [n] arrival order inside the bin (atomics)
    int4 *rec;            // [n] rebased record in input order: X, Y, res, z
    int32_t *perm_tmp;    // [n] unordered perm after the scatter
    int32_t *X, *Y;       // [n] binned SoA
    uint32_t *res;
    float *z;
    int32_t *idx;
    int64_t *stats;       // [4]
    int32_t *big_list;    // [nb] bins too long for one thread
    int32_t *row_count;   // [nby] soundings per bin row (row path)
    int32_t *row_start;   // [nby + 1]
    int32_t *rowid;       // [n] bin row per input sounding (or -1)
    unsigned long long *keys;  // [n] (bin column << 32 | original index)
    unsigned long long *keys2; // [n] scratch for the per-row sort
    int32_t *drops;            // per-block dropped-sounding counters
    size_t bytes;
};
size_t bin_workspace_layout(int64_t n, const BinGeom &g, char *base,
                            BinWorkspace *w);

// Binned structure-of-arrays outputs.
struct SoA {
    int32_t *X, *Y;
    uint32_t *res;
    float *z;
    int32_t *idx;
};

// Everything one item needs for the row-wise counting sort.
struct RowItem {
    const double *x, *y, *z;
    int64_t n;
    double x0, y0, lo, hix, hiy;
    int32_t s, hB, nbx, nby;
    int32_t nblk;  // k_row_hist blocks of this item (drop partials)
    // optional (serving): lattice box X min, Y min, X max, Y max of the
    // binned soundings, widened atomically from a caller-seeded empty box
    int32_t *bbox;
    int32_t *row_count, *row_start, *rowid, *pos, *colkey, *drops, *cell_start;
    int4 *rec;
    unsigned long long *keys, *keys2, *stats;
    SoA o;
};

// Pointers that reach a kernel inside a descriptor in memory cannot be told
// from LDS pointers by the compiler, which then emits flat accesses; an
// explicitly global-typed copy gives global loads and stores (32-bit offsets,
// no LDS counter waits).
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> gmem(T *p)
{
    return (gptr<T>)p;
}

// Batched launches: block b belongs to the item i with off[i] <= b < off[i+1]
// (off ascending, count items; empty items have off[i] == off[i+1]).
__device__ inline int item_of(const int32_t *off, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

bool row_path_ok(const BinGeom &geom);
RowItem make_row_item(const auv_grid *g, const BinGeom &geom, const double *x,
                      const double *y, const double *z, int64_t n, const BinWorkspace &w);
int32_t row_hist_blocks(int64_t n);
int32_t row_scatter_blocks(int64_t n);
// max_nbx / max_nby: the largest bin domain among the items (sizes the LDS);
// keys_per_row: the largest mean of input soundings per bin row among the
// items (picks the sort's LDS key area; longer rows stay correct, on slower
// paths).
auv_status launch_binning_batch(const RowItem *d_items, const int32_t *d_hist_off,
                                const int32_t *d_scatter_off, const int32_t *d_sort_off,
                                int32_t count, int32_t hist_blocks, int32_t scatter_blocks,
                                int32_t sort_blocks, int32_t max_nbx, int32_t max_nby,
                                double keys_per_row, hipStream_t st);

// The work of auv_bin_points into a caller-provided handle (no allocation).
auv_status bin_into(const auv_grid *grid, const double *x, const double *y, const double *z,
                    int64_t n, double radius, int32_t bin_log2, void *ws, size_t ws_bytes,
                    hipStream_t stream, auv_bins *b);

auv_status launch_binning(const auv_grid *g, const BinGeom &geom,
                          const double *x, const double *y, const double *z,
                          int64_t n, const BinWorkspace &w, hipStream_t st);

// IDW / nearest kernels.
struct IdwArgs {
    double x_first, y_first;  // unused placeholder for alignment
    double dx, dy;            // grid spacing (metres)
    int32_t nx, ny;
    int32_t R;                // lattice search radius
    float power;
    int32_t min_pts, max_pts;
    int32_t precision;
    int32_t mode;             // bit 0: IDW value, bit 1: nearest outputs,
                              // bit 2: accumulate into acc_* (serving)
    float inv_r2;             // 1 / R^2 (lattice units)
    int32_t R_stage;          // lattice reach of the candidate search (>= R)
    float r2f;                // radius^2 in m^2, FP32 (precision variants)
    double x0, y0;            // grid origin (precision variants)
    bool dense;               // use the dense (ring search, top-k) form
    bool span;                // sparse: the span form where it applies
    int32_t pmode;            // 1, 2, 3: integer power (fast weights), 0: general
    int32_t tile_w, tile_h;   // nodes per wave tile (0: the form's default): window
                              // form 16 x 16 or 16 x 8; dense form any power-of-two
                              // shape of 64 nodes (8 x 8, 16 x 4, 4 x 16, ...)
    float *z_out;
    int32_t *cnt_out;
    int32_t *nn_idx_out;
    float *nn_z_out;
    // accumulate mode: resident sums over all requests so far, depths
    // relative to zref_acc
    float *acc_num, *acc_den;
    int32_t *acc_cnt;
    float *acc_lo, *acc_hi;   // smallest / largest member depth (valid where acc_cnt > 0)
    double zref_acc;
};
auv_status launch_idw(const auv_bin_view &bins, const IdwArgs &a, hipStream_t st);

// Window form of the IDW kernel (linear node lattice, window <= 256 cells).
struct WinGeom {
    int DXl, DYl;   // node spacing in lattice units
    int X0, Y0;     // lattice coordinate of node column 0 / row 0
    int Wx, Wy;     // nodes per axis a sounding can reach
    int ncells, nchunks;
};
bool window_geometry(const IdwArgs &a, WinGeom *g);
auv_status launch_idw_window(const auv_bin_view &bins, const IdwArgs &a, const WinGeom &g,
                             int pmode, hipStream_t st);
auv_status launch_idw_dense(const auv_bin_view &bins, const IdwArgs &a, int pmode,
                            hipStream_t st);
auv_status launch_idw_window_prec(const auv_bin_view &bins, const IdwArgs &a,
                                  const WinGeom &g, int pmode, hipStream_t st);

auv_status launch_bilinear(const float *src, const auv_grid_desc &s, float *dst,
                           const auv_grid_desc &d, hipStream_t st);
auv_status launch_bicubic(const float *src, const auv_grid_desc &s, float *dst,
                          const auv_grid_desc &d, hipStream_t st);
auv_status launch_kriging(const float *src, const auv_grid_desc &s, float *dst,
                          const auv_grid_desc &d, double range, hipStream_t st);

}  // namespace auv
