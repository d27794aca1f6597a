/*
 * auvgrid — gridding scattered multibeam soundings on one MI355X (gfx950).
 *
 * C ABI of libauvgrid.so.  Plain pointers and sizes only.  Pointers marked
 * "device" must be device memory of the current HIP device (any allocator);
 * pointers marked "host" are ordinary host memory.  The caller owns every
 * buffer; the library owns only the opaque handles it returns and frees them
 * in the matching *_destroy call.
 *
 * Streams: `auv_stream` is a hipStream_t (NULL = the legacy default stream).
 * Argument validation is synchronous and returns a status; kernels are only
 * enqueued on the given stream.  A device fault surfaces as AUV_ERR_HIP from a
 * later call.  No call synchronises the stream unless its comment says so.
 *
 * Errors: every call returns an auv_status; on failure auv_last_error()
 * returns a message for the calling thread.  No exception crosses the ABI.
 *
 * Source of the method: "Towards Real-Time Interpolation for Enhanced AUV
 * Deep Sea Mapping" (Saxena).  The paper defines bilinear interpolation
 * (Sec. III-A), NaN samples as invalid candidates (Sec. III-B, III-D), holes
 * where bilinear has no value (Sec. III-D, V-D), a "nearest n valid candidate
 * neighbours" helper (Sec. III-D) and GPU-resident real-time interpolation
 * with the host only in control (Sec. IV).  The radius-limited IDW and the
 * nearest-neighbour gridding below generalise that helper; their exact
 * definitions are given at each entry point.
 *
 * Geometry.  A grid is pixel-centred: node (row a, column b) sits at
 * (x0 + (b + 1/2) dx, y0 + (a + 1/2) dy) in projected metres (Sec. III, Fig. 1:
 * the interpolated value sits at the centre of its cell).  Every grid array is
 * row-major [ny][nx], element a*nx + b.
 *
 * Lattice.  Every discrete decision (bin, radius membership, ranking, hit,
 * nearest pick) is taken exactly on a lattice of 2^-16 m relative to the
 * grid's lower-left corner: X = rne((x - x0) 2^16) for a sounding,
 * X_b = rne(((b + 1/2) dx) 2^16) for a node, R = rne(r 2^16) for a radius,
 * D^2 = dX^2 + dY^2, member iff D^2 <= R^2 (closed disk).  The key (D^2,
 * original index) ranks candidates.
 */
#ifndef AUVGRID_H
#define AUVGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *auv_stream; /* hipStream_t */

typedef enum {
    AUV_OK = 0,
    AUV_ERR_INVALID = -1, /* a bad argument (null pointer, bad size, ...)     */
    AUV_ERR_RANGE = -2,   /* grid/radius/bin too large for the int32 lattice  */
    AUV_ERR_BUDGET = -3,  /* workspace or arena too small                     */
    AUV_ERR_HIP = -4,     /* a HIP runtime call failed                        */
    AUV_ERR_STATE = -5    /* call not valid in the object's current state     */
} auv_status;

/* Grid descriptor.  Limits: nx, ny >= 1; dx, dy > 0; nx*dx and ny*dy below
 * 16384 m (the lattice must fit in 31 bits with its halo). */
typedef struct {
    double x0, y0; /* lower-left corner of the grid, projected metres */
    double dx, dy; /* node spacing (metres)                            */
    int32_t nx, ny;
} auv_grid_desc;

typedef struct auv_grid auv_grid; /* immutable validated grid */
typedef struct auv_bins auv_bins; /* soundings binned for one grid and radius */

/* Precision variants of the IDW distance and weight arithmetic. */
enum {
    AUV_P_FP32_REBASE = 0,   /* FP64 rebase to the grid lattice, FP32 weights */
    AUV_P_FP16_OFFSETS = 1,  /* FP16 offsets from the tile centre, FP32 sums  */
    AUV_P_FP32_ABSOLUTE = 2  /* FP32 absolute coordinates, no rebase          */
};

typedef struct {
    double power;    /* p > 0: weight d^-p                                  */
    double radius;   /* r > 0 metres; must not exceed the bins' radius       */
    int32_t min_pts; /* fewer selected soundings than this -> NaN (0 or 1 = none) */
    int32_t max_pts; /* cap k on the selected set, 0 = no cap                */
    int32_t precision; /* AUV_P_*; only AUV_P_FP32_REBASE meets the exact
                          lattice contract, the others are measured variants */
    int32_t algo;      /* AUV_ALGO_*: kernel form; every form computes the same
                          result, they differ only in speed */
} auv_idw_params;

/* Kernel forms of auv_interp_idw. */
enum {
    AUV_ALGO_AUTO = 0,   /* dense form when the expected disk population is at
                            least max_pts / 2 (and 1 <= max_pts <= 32): many
                            nodes would exceed the cap; else sparse */
    AUV_ALGO_SPARSE = 1, /* node windows scattered from each sounding */
    AUV_ALGO_DENSE = 2,  /* per-node ring search with a register top-k list;
                            needs 1 <= max_pts <= 32 and AUV_P_FP32_REBASE */
    AUV_ALGO_SPAN = 3    /* sparse, span form: (sounding, node) pairs packed 64
                            per instruction, LDS atomics; integer powers
                            1..3 with AUV_P_FP32_REBASE, else the window
                            form runs */
};

/* Library version string (static storage). */
const char *auv_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *auv_last_error(void);

/* Validate a grid descriptor and return an immutable handle.
 * Errors: AUV_ERR_INVALID for null pointers or non-positive sizes/spacings,
 * AUV_ERR_RANGE when the extent exceeds the lattice limit. */
auv_status auv_grid_create(const auv_grid_desc *desc, auv_grid **out);
void auv_grid_destroy(auv_grid *grid);

/* Size in bytes of the device workspace auv_bin_points needs for n soundings,
 * a search radius (metres) and a bin size of 2^bin_log2 lattice units
 * (bin_log2 in [12, 26]; 0 picks the default: the smallest power of two not
 * below the radius, clamped to that range). */
auv_status auv_bin_workspace_size(const auv_grid *grid, int64_t n, double radius,
                                  int32_t bin_log2, size_t *bytes);

/* Bin soundings for one grid (stable counting sort, "cell hash").
 *   x, y, z  device, float64, n elements each (projected metres; z is the
 *            signed elevation, negative down).  Read only during the kernels
 *            enqueued by this call.
 *   n        0 <= n < 2^31.
 *   radius   the largest search radius (metres) that will be used with the
 *            bins; the bin domain is the grid grown by this radius.
 *   ws       device workspace of at least auv_bin_workspace_size bytes, 256-B
 *            aligned; it holds the bins and must outlive the returned handle.
 * A sounding with a non-finite x, y or z is invalid and dropped (NaN samples
 * are invalid candidates, Sec. III-B / III-D).  A valid sounding outside the
 * grid grown by the radius cannot reach any node and is dropped too.  Within a
 * bin, soundings keep ascending original index, so the result is
 * deterministic.  Enqueues work on `stream`; returns at once. */
auv_status auv_bin_points(const auv_grid *grid, const double *x, const double *y,
                          const double *z, int64_t n, double radius,
                          int32_t bin_log2, void *ws, size_t ws_bytes,
                          auv_stream stream, auv_bins **out);

/* Geometry of the bins: bins per axis, halo (bins added on each side),
 * bin_log2 actually used.  Host call, no device work. */
auv_status auv_bins_info(const auv_bins *bins, int32_t *nbx, int32_t *nby,
                         int32_t *halo, int32_t *bin_log2);

/* Copy the bins out for inspection.
 *   cell_start  device, nbx*nby+1 int32: first binned position of each bin
 *               (exclusive prefix of the counts), nullable;
 *   perm        device, capacity n int32: original index of each binned
 *               position, ordered by (bin id, original index), nullable;
 *   counts      host, 3 int64: binned, invalid, outside.  Synchronises
 *               `stream` when non-null. */
auv_status auv_bins_export(const auv_bins *bins, int32_t *cell_start,
                           int32_t *perm, int64_t *counts, auv_stream stream);
void auv_bins_destroy(auv_bins *bins);

/* Radius-limited inverse-distance weighting on every node of `grid`.
 * For node n: C(n) = valid soundings with D^2 <= R^2; S(n) = the first
 * min(|C|, max_pts) of C ranked by (D^2, original index);
 *   - if some member of S has D^2 == 0 (a hit) the value is the mean depth of
 *     those members;
 *   - else if |S| < min_pts (or S is empty) the value is NaN (a hole);
 *   - else z = sum w_i z_i / sum w_i over S with w_i = d_i^-p, d_i the
 *     distance from the node computed from the sounding's double
 *     coordinates, clamped to [min, max] of the depths in S.
 * Distances and weights run in FP32 (with the FP64 rebase), the final
 * num/den division and the clamp in FP64, rounded once to FP32; the clamp
 * bounds are the depths rounded to FP32, so every returned value lies within
 * [min, max] of the FP32-rounded depths of S exactly.  Tolerance against the
 * FP64 definition: 1e-5 relative per node; S, the NaN mask, counts and the
 * nearest pick are exact.
 *   z_out      device float [ny][nx];
 *   cnt_out    device int32 [ny][nx] |S|, nullable;
 *   nn_idx_out device int32 [ny][nx] first member of S (the nearest sounding,
 *              -1 if none), nullable;
 *   nn_z_out   device float [ny][nx] its depth (NaN if none), nullable.
 * `bins` must come from this grid with a radius >= params->radius.
 * Errors: AUV_ERR_INVALID for bad params or a radius above the bins'. */
auv_status auv_interp_idw(const auv_grid *grid, const auv_bins *bins,
                          const auv_idw_params *params, float *z_out,
                          int32_t *cnt_out, int32_t *nn_idx_out, float *nn_z_out,
                          auv_stream stream);

/* Nearest-neighbour gridding: for every node, the valid sounding within the
 * radius that minimises (D^2, original index) — ties go to the lowest
 * original index.  idx_out (device int32 [ny][nx]) gets its original index or
 * -1; z_out (device float [ny][nx], nullable) its depth rounded to float, or
 * NaN.  radius must not exceed the bins' radius. */
auv_status auv_interp_nearest(const auv_grid *grid, const auv_bins *bins,
                              double radius, int32_t *idx_out, float *z_out,
                              auv_stream stream);

/* Bilinear resample (Sec. III-A) of a source grid onto the nodes of a
 * destination grid.  Each destination node maps to the source index
 * coordinate u = (x - x0_src)/dx_src - 1/2 (likewise v), clamped to
 * [0, n-1]; the value is the bilinear blend of the four surrounding source
 * nodes, and NaN when any of them is NaN (no fallback: a hole, Sec. III-D).
 *   src  device float [s.ny][s.nx];  dst  device float [d.ny][d.nx]. */
auv_status auv_resample_bilinear(const float *src, const auv_grid_desc *s,
                                 float *dst, const auv_grid_desc *d,
                                 auv_stream stream);

/* Catmull-Rom bicubic resample (Sec. III-B) with the same node mapping as
 * auv_resample_bilinear: the cubic through the source nodes at index
 * i0 - 1 .. i0 + 2 (clamped to the grid) runs along x on four rows, then
 * along y over the four results.  A node with a non-finite value (NaN: an
 * invalid sample) among its 16 taps falls back to the bilinear value (the
 * "not enough valid neighbours" fallback of Sec. III-B), which is itself NaN
 * when one of its four corners is (a hole).
 * Same arguments, layout and errors as auv_resample_bilinear. */
auv_status auv_resample_bicubic(const float *src, const auv_grid_desc *s,
                                float *dst, const auv_grid_desc *d,
                                auv_stream stream);

/* Ordinary-kriging resample (Sec. III-C) with the node mapping of
 * auv_resample_bilinear.  Neighbourhood: the 5 x 5 source nodes centred on
 * the source node nearest to the destination point, moved inward at the grid
 * edges.  Variogram: exponential, gamma(h) = C0 (1 - exp(-h / range)) with h
 * in metres (the sill C0 cancels from the weights, so only `range` is
 * given).  The weights solve the 26 x 26 ordinary-kriging system (unbiasedness
 * row included); z = sum of weights x depths.  A neighbourhood with a
 * non-finite value, or a source grid under 5 x 5, falls back to the bilinear
 * value (a hole when one of its corners is NaN).  FP32 arithmetic on depths
 * relative to the window centre; from a range of 16 hypot(dx, dy) on,
 * 1 - exp(-h / range) is taken from its Taylor series (every h / range is then
 * at most 1/4), which keeps the FP32 result to about 1e-6 relative however
 * long the range.  Errors as auv_resample_bilinear, plus AUV_ERR_INVALID for
 * a non-positive or non-finite range and AUV_ERR_RANGE for a range above 1e4
 * source spacings. */
auv_status auv_resample_kriging(const float *src, const auv_grid_desc *s,
                                float *dst, const auv_grid_desc *d, double range,
                                auv_stream stream);

/* Empirical semivariogram of a grid along its axes, the data the kriging
 * variogram's range is fitted to (Sec. III-C gives the exponential model but
 * not its parameters).  For lag k = 1..nlags: gamma_x[k-1] = the sum of
 * (z1 - z2)^2 over the pairs (row a, column b), (a, b + k) with both values
 * finite, over twice their count pairs_x[k-1] (lag k * dx metres); gamma_y
 * likewise over (a, b), (a + k, b) (lag k * dy); NaN where a lag has no pair.
 *   src    device float [s.ny][s.nx];
 *   ws     device workspace of auv_variogram_workspace_size bytes, 256-B aligned;
 *   gamma_x, gamma_y  host double [nlags];  pairs_x, pairs_y  host int64 [nlags],
 *          nullable.
 * Sums run in FP64 in a fixed order (deterministic).  Synchronises `stream`.
 * Errors: AUV_ERR_INVALID for nlags outside [1, 1024] or a bad descriptor,
 * AUV_ERR_BUDGET for a short workspace. */
auv_status auv_variogram_workspace_size(const auv_grid_desc *s, int32_t nlags, size_t *bytes);
auv_status auv_variogram(const float *src, const auv_grid_desc *s, int32_t nlags, void *ws,
                         size_t ws_bytes, double *gamma_x, double *gamma_y, int64_t *pairs_x,
                         int64_t *pairs_y, auv_stream stream);

/* Weighted least-squares fit of the exponential variogram of Sec. III-C,
 * gamma(h) = sill (1 - exp(-h / range)), to n host points (h_j > 0 metres,
 * gamma_j, weights w_j >= 0, e.g. pair counts; points with zero weight or a
 * non-finite gamma are ignored): the sill at its least-squares value for each
 * range, the range searched on a log scale over [min h / 100, 1000 max h] and
 * refined by golden section.  Host arithmetic only.  Errors: AUV_ERR_INVALID
 * for fewer than two usable points; AUV_ERR_RANGE when the best range is an
 * end of that interval (no sill: *range and *sill still hold the end). */
auv_status auv_fit_exponential(const double *h, const double *gamma, const double *w, int32_t n,
                               double *range, double *sill);

/* ------------------------------------------------- no device allocation --
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * auv_grid_idw_noalloc computes what auv_bin_points(grid, x, y, z, n,
 * params->radius, bin_log2, ...) followed by auv_interp_idw(grid, bins,
 * params, z_out, cnt_out, nn_idx_out, nn_z_out, ...) compute (same
 * definition, tolerance, exact counts and nearest picks), but the bins and
 * the binning scratch live in a static device array of
 * AUV_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  It calls no hipMalloc, hipFree or other
 * allocating routine; the caller still passes inputs (device float64 x, y, z,
 * n each) and outputs (device [ny][nx]; cnt_out, nn_idx_out, nn_z_out
 * nullable).  Work is enqueued on `stream` (of the current device).
 * Every call on one GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (different streams, or threads, without ordering between
 * them) race.  Serialise them on one stream or with events.
 * Errors: as auv_bin_points and auv_interp_idw, plus AUV_ERR_BUDGET when
 * auv_bin_workspace_size(grid, n, params->radius, bin_log2) exceeds
 * AUV_NOALLOC_SCRATCH_BYTES (the 2M-sounding swath on a 4096^2 grid at 2 m
 * with a 6 m radius needs about 149 MB). */
#define AUV_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
auv_status auv_grid_idw_noalloc(const auv_grid *grid, const double *x, const double *y,
                                const double *z, int64_t n, int32_t bin_log2,
                                const auv_idw_params *params, float *z_out, int32_t *cnt_out,
                                int32_t *nn_idx_out, float *nn_z_out, auv_stream stream);

/* ------------------------------------------------------------ batches --
 * Many independent, uneven gridding problems ("items") run as one unit: one
 * set of batched binning launches and one persistent IDW launch per kernel
 * form (sparse window, dense top-k; on two concurrent graph branches) whose
 * waves pull (item, tile) work from per-XCD queues, captured once into a HIP
 * graph and replayed on later launches.  Bin sizes and the kernel form per item come
 * from an autotune table (auv_batch_autotune) or from defaults.  Each item's
 * result is the auv_interp_idw result for that item (same definition and
 * tolerance); the batch only changes how the work is scheduled. */
typedef struct {
    auv_grid_desc grid;
    const double *x, *y, *z; /* device float64 [n] */
    int64_t n;
    auv_idw_params params;   /* precision must be AUV_P_FP32_REBASE */
    float *z_out;            /* device float [ny][nx] */
    int32_t *cnt_out;        /* device int32 [ny][nx], nullable */
    int32_t *nn_idx_out;     /* device int32 [ny][nx], nullable */
    float *nn_z_out;         /* device float [ny][nx], nullable */
} auv_batch_item;

typedef struct auv_batch auv_batch;

/* Validate `count` items (host array, copied) and plan the batch.  tune_path
 * (nullable) names a table written by auv_batch_autotune; items of a class it
 * does not list get the defaults (bin = smallest power of two >= radius,
 * kernel form chosen as by AUV_ALGO_AUTO).  Errors: AUV_ERR_INVALID for a bad
 * item (its index is in the message). */
auv_status auv_batch_plan(const auv_batch_item *items, int32_t count,
                          const char *tune_path, auv_batch **out);

/* Device workspace (bytes) that auv_batch_launch and auv_batch_launch_plain
 * need for this batch. */
auv_status auv_batch_workspace_size(const auv_batch *batch, size_t *bytes);

/* Run the batch.  The first call with a given workspace uploads the item
 * tables into it, captures the work into a HIP graph and launches it; later
 * calls with the same workspace replay the graph.  The inputs and outputs of
 * the items must stay at the same addresses between calls.  Asynchronous on
 * `stream` (which must not be in capture). */
auv_status auv_batch_launch(auv_batch *batch, void *ws, size_t ws_bytes,
                            auv_stream stream);

/* The plain form of the same batch, for comparison: for each item in turn,
 * auv_bin_points with the default bin size and auv_interp_idw with
 * AUV_ALGO_AUTO, launched one after another on `stream` (no graph). */
auv_status auv_batch_launch_plain(auv_batch *batch, void *ws, size_t ws_bytes,
                                  auv_stream stream);

/* Autotuner: group the items into classes (expected soundings per disk and
 * grid side, both bucketed by powers of two), time the candidate (bin size,
 * kernel form) pairs at the form's default node tile on one representative
 * item per class, then the winner with the form's other node tiles (window
 * form 16 x 16 or 16 x 8 nodes per wave; dense form 8 x 8, 16 x 4 or 4 x 16),
 * and write the fastest per class to tune_path (a small text table:
 * "class <dens> <side> bin_log2 <s> algo <a> tile <w> <h> ms <t>"; tables
 * without the tile fields stand for the default tiles).  Synchronises
 * `stream`; uses `ws` (at least auv_batch_workspace_size of a batch planned
 * from the same items) as scratch, and overwrites the items' outputs. */
auv_status auv_batch_autotune(const auv_batch_item *items, int32_t count, void *ws,
                              size_t ws_bytes, auv_stream stream, const char *tune_path);

/* Per-item plan actually used (for reports): bin_log2, kernel form and node
 * tile per wave (columns, rows).  Every pointer is nullable. */
auv_status auv_batch_item_plan(const auv_batch *batch, int32_t item, int32_t *bin_log2,
                               int32_t *algo, int32_t *tile_w, int32_t *tile_h);

void auv_batch_destroy(auv_batch *batch);

/* ------------------------------------------------------------ serving --
 * Real-time gridding of many vehicles' sounding streams with the grids kept
 * on the device; the host only controls (the real-time mode of Sec. IV).
 * Each vehicle owns a grid and resident per-node sums of the radius-limited
 * IDW (no k-cap, so the sums are additive): weighted depth, weight, count;
 * a coincident sounding adds a dominant weight, so the read-out of a node
 * with hits is the mean of its hits.  A request (a block of soundings from one
 * vehicle) is rebased, binned and gathered into the sums of the nodes within
 * the radius; reading a grid finalizes z = z_ref + sum(w dz) / sum(w) (NaN
 * where count < min_pts and no hit).  After any set of requests the read-out
 * equals auv_interp_idw (max_pts 0) on the union of that vehicle's soundings,
 * within the same tolerance.  A vehicle's requests are applied in submission
 * order, one per launch, so its grid does not depend on the other vehicles'
 * traffic or on the batching (bit for bit).
 *
 * A worker thread owned by the session drains the queue on its own stream:
 * AUV_SERVE_FIFO runs one request at a time and waits for it;
 * AUV_SERVE_BATCHED (continuous batching) launches every queued request it
 * can (at most one per vehicle and max_batch per launch) as one batched
 * launch, keeps two launches in flight and forms the next batch while the
 * GPU works. */
enum { AUV_SERVE_FIFO = 0, AUV_SERVE_BATCHED = 1 };
enum { AUV_T_QUEUED = 0, AUV_T_RUNNING = 1, AUV_T_DONE = 2, AUV_T_FAILED = 3 };

typedef struct {
    int32_t n_vehicles;
    const auv_grid_desc *grids; /* host [n_vehicles] */
    const double *z_ref;        /* host [n_vehicles] reference depth per vehicle, nullable (0) */
    auv_idw_params params;      /* power 1, 2 or 3; max_pts 0; precision AUV_P_FP32_REBASE;
                                   the node spacing times 2^16 must be an even integer and
                                   (2 r / dx + 1)(2 r / dy + 1) <= 256 */
    int32_t max_request;        /* soundings per request, 1 .. 2^24 */
    int32_t slots;              /* requests held at once (queued or running), 1 .. 4096 */
    int32_t mode;               /* AUV_SERVE_FIFO or AUV_SERVE_BATCHED */
    int32_t max_batch;          /* requests per batched launch, 1 .. 64 (0: 64) */
} auv_session_desc;

typedef struct {
    int32_t state;              /* AUV_T_* */
    int32_t vehicle;
    int64_t n;
    double t_arrival;           /* as given to auv_session_submit */
    double t_launch;            /* session clock when its launch was enqueued */
    double t_done;              /* session clock when its completion was observed */
} auv_ticket_info;

typedef struct auv_session auv_session;

/* Device bytes a session needs: `fixed` for the request slots' staging and
 * binning space and the launch tables, plus `per_vehicle` (20 bytes per node
 * of the largest grid) for each admitted vehicle.  Host only. */
auv_status auv_session_budget(const auv_session_desc *desc, size_t *fixed,
                              size_t *per_vehicle);

/* Create a session on the current device.  `arena` (device, 256-byte aligned,
 * caller-owned, at least `fixed` bytes) is the session's whole HBM budget:
 * slots, tables and every admitted vehicle's sums are carved from it.
 * Allocates pinned host staging (slots x max_request soundings).  Errors:
 * AUV_ERR_INVALID for a bad descriptor, AUV_ERR_BUDGET when the arena cannot
 * hold the fixed part. */
auv_status auv_session_create(const auv_session_desc *desc, void *arena, size_t arena_bytes,
                              auv_session **out);

/* Queue one request of n soundings (host float64 arrays, copied before the
 * call returns) for `vehicle`.  A vehicle is admitted at its first request:
 * its sums are carved from the arena and cleared; when the arena cannot hold
 * them the call fails with AUV_ERR_BUDGET and queues nothing.  Blocks while
 * every slot is taken.  t_arrival is the request's arrival on the session
 * clock (auv_session_now), kept for latency reports.  Thread-safe. */
auv_status auv_session_submit(auv_session *s, int32_t vehicle, const double *x,
                              const double *y, const double *z, int64_t n, double t_arrival,
                              uint64_t *ticket);

/* State and times of a ticket.  Thread-safe. */
auv_status auv_session_poll(auv_session *s, uint64_t ticket, auv_ticket_info *info);

/* Block until every request submitted so far has finished.  Returns
 * AUV_ERR_HIP if any of them failed. */
auv_status auv_session_drain(auv_session *s);

/* Wait for the vehicle's submitted requests, then enqueue the read-out of its
 * grid on `stream`: z_out device float [ny][nx] (NaN: no value; clamped to
 * the depth range of the node's soundings like auv_interp_idw), cnt_out
 * device int32 [ny][nx] (nullable; soundings within the radius so far).
 * The read-out covers exactly the requests submitted before the call: the
 * session's later launches wait for it on the device (an event recorded on
 * `stream`), so a submit right after it cannot change what it reads. */
auv_status auv_session_read_grid(auv_session *s, int32_t vehicle, float *z_out,
                                 int32_t *cnt_out, auv_stream stream);

/* Wait for the vehicle's requests and release its sums back to the arena
 * (its grid is lost; a later request admits it again, empty).  Work the
 * caller enqueued on other streams that reads the vehicle must be finished. */
auv_status auv_session_retire(auv_session *s, int32_t vehicle);

/* Seconds since the session was created (steady clock). */
double auv_session_now(const auv_session *s);

/* Drain, stop the worker and free host-side resources (not the arena). */
void auv_session_destroy(auv_session *s);

#ifdef __cplusplus
}
#endif
#endif /* AUVGRID_H */
