/*
 * FP64 CPU oracle for scattered-sounding gridding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source, header, table or helper with
 * the HIP library: every definition below is written out here on its own.
 *
 * Definitions followed (the paper, "Towards Real-Time Interpolation for
 * Enhanced AUV Deep Sea Mapping", has no IDW; the IDW/NN readings are stated
 * where each function is defined, in auv_oracle.c):
 *   - bilinear: Sec. III-A, the four-corner weighted average;
 *   - NaN samples are invalid candidates: Sec. III-B and III-D;
 *   - holes (no fallback for bilinear): Sec. III-D and V-D (Kerguelen);
 *   - "nearest n valid candidate neighbours" helper: Sec. III-D, item 1,
 *     generalised to a radius-limited, optionally capped neighbour set.
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py
 * (closed forms, invariants, scipy cKDTree, torch interpolate, brute force
 * against binned search).  No function is "parity unpinned".
 */
#ifndef AUV_ORACLE_H
#define AUV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Regular grid: node (row a, column b) sits at (x0 + (b+1/2)dx, y0 + (a+1/2)dy);
 * values are stored row-major, index a*nx + b. */
typedef struct {
    double x0, y0, dx, dy;
    int32_t nx, ny;
} orc_grid;

/* return codes */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ENOMEM (-3)

/* Bin domain for a grid, radius and bin size 2^bin_log2 lattice units
 * (lattice quantum 2^-16 m).  Writes the bin counts per axis and the halo h. */
int orc_bin_dims(const orc_grid *g, double radius, int32_t bin_log2,
                 int32_t *nbx, int32_t *nby, int32_t *halo);

/* O4: stable counting sort of the valid, in-domain soundings into bins.
 * cell_start has nbx*nby+1 entries; perm receives original indices ordered by
 * (bin id, original index); n_invalid counts non-finite soundings, n_outside
 * valid soundings outside the bin domain. */
int orc_bin(const orc_grid *g, const double *x, const double *y, const double *z,
            int64_t n, double radius, int32_t bin_log2,
            int32_t *cell_start, int32_t *perm, int64_t *n_binned,
            int64_t *n_invalid, int64_t *n_outside);

/* O1: radius-limited, optionally capped inverse-distance weighting.
 * bin_log2 < 0 selects the brute-force search over every sounding, otherwise
 * candidates come from the bins of orc_bin.  nodes == NULL evaluates every
 * node; otherwise n_nodes flat node indices (a*nx+b) and the outputs are
 * indexed like the list.  max_pts == 0 means no cap.  Outputs: z_out (NaN for
 * no value), cnt_out = size of the selected set, nn_out = index of the first
 * selected sounding (-1 if none).  cnt_out / nn_out may be NULL. */
int orc_idw(const orc_grid *g, const double *x, const double *y, const double *z,
            int64_t n, double radius, double power, int32_t min_pts,
            int32_t max_pts, int32_t bin_log2, const int64_t *nodes,
            int64_t n_nodes, double *z_out, int32_t *cnt_out, int32_t *nn_out,
            int32_t nthreads);

/* Bounds of O1's selected set S(n): smallest and largest depth over it (NaN
 * when S(n) is empty).  Same search and node list conventions as orc_idw. */
int orc_idw_bounds(const orc_grid *g, const double *x, const double *y, const double *z,
                   int64_t n, double radius, int32_t max_pts, int32_t bin_log2,
                   const int64_t *nodes, int64_t n_nodes, double *lo_out, double *hi_out,
                   int32_t nthreads);

/* O2: nearest sounding within the radius by the key (D^2, original index).
 * idx_out = -1 and z_out = NaN where no sounding is within the radius. */
int orc_nearest(const orc_grid *g, const double *x, const double *y,
                const double *z, int64_t n, double radius, int32_t bin_log2,
                const int64_t *nodes, int64_t n_nodes, int32_t *idx_out,
                double *z_out, int32_t nthreads);

/* O3: bilinear resample of a source grid onto the nodes of a destination grid
 * (Sec. III-A formula; source index coordinate clamped to the grid; any NaN
 * corner gives NaN). */
int orc_bilinear(const orc_grid *src_g, const double *src, const orc_grid *dst_g,
                 double *dst, int32_t nthreads);

/* O5: Catmull-Rom bicubic resample (Sec. III-B): the same source index
 * coordinate as O3, 4 x 4 taps from index i0 - 1 .. i0 + 2 (clamped to the
 * grid), the cubic along x on each tap row, then along y; when any tap is
 * not finite (NaN marks an invalid value) the node falls back to O3's
 * bilinear value (reading the fallback sentence of Sec. III-B as "not enough
 * valid neighbours"), which may itself be a hole. */
int orc_bicubic(const orc_grid *src_g, const double *src, const orc_grid *dst_g,
                double *dst, int32_t nthreads);

/* O6: ordinary kriging resample (Sec. III-C): the 5 x 5 source nodes centred
 * on the node nearest to the destination point (same index coordinate as O3;
 * the window moves inward at the grid edges), the exponential variogram
 * gamma(h) = 1 - exp(-h / range) (h in metres; the sill cancels from the
 * weights), the 26 x 26 system with the unbiasedness row solved by Gaussian
 * elimination with partial pivoting, and z = sum of weights x depths.  Any
 * non-finite window value (or a grid under 5 x 5) falls back to O3's
 * bilinear value, as the cubic does. */
int orc_kriging(const orc_grid *src_g, const double *src, const orc_grid *dst_g,
                double range, double *dst, int32_t nthreads);

/* O7: empirical semivariogram along the grid axes (classical estimator):
 * gamma_x[k-1] over the pairs (a, b), (a, b + k) with both values finite,
 * gamma_y[k-1] over (a, b), (a + k, b), each sum of squared differences over
 * twice the pair count (NaN without pairs), k = 1..nlags; pair counts to
 * pairs_x / pairs_y when non-null.  The variogram whose parameters Sec. III-C
 * leaves unstated is fitted to these. */
int orc_variogram(const orc_grid *g, const double *src, int32_t nlags, double *gamma_x,
                  double *gamma_y, int64_t *pairs_x, int64_t *pairs_y);

/* O8: weighted least-squares fit of the exponential variogram
 * gamma(h) = C0 (1 - exp(-h / a)) (Sec. III-C's model) to n points (h_j > 0,
 * gamma_j, w_j >= 0; zero-weight or non-finite points ignored): a by a log-grid
 * scan and ternary refinement of the residual with C0 at its least-squares
 * value.  ORC_ERANGE when the best range is an end of the scanned interval
 * [min h / 100, 1000 max h] (no sill). */
int orc_fit_exponential(const double *h, const double *gam, const double *w, int32_t n,
                        double *range, double *sill);

#ifdef __cplusplus
}
#endif
#endif
