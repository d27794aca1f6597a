/*
 * FP64 CPU oracle for scattered-sounding gridding — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It is a plain, slow, obviously-correct statement of what
 * the GPU path computes: every per-node result is the definition written out,
 * all arithmetic in IEEE double (built with -ffp-contract=off, no fast-math).
 * OpenMP only splits the list of output nodes among threads; the arithmetic for
 * one node is sequential and in the order stated below.
 *
 * The lattice.  Every discrete decision (bin membership, radius membership,
 * ranking, hits, nearest pick) is taken on an exact integer lattice of 2^-16 m
 * relative to the grid's lower-left corner:
 *     X_i = rne((x_i - x0) * 2^16),  node X_b = rne(((b + 1/2) dx) * 2^16),
 *     R   = rne(r * 2^16),           D^2 = (X_i - X_b)^2 + (Y_i - Y_a)^2.
 * Values (weights, depths) are computed from the original double coordinates.
 *
 * Parity: pinned by tests/test_oracle_*.py; no function is unpinned.
 */
#include "auv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_Q 65536.0              /* lattice units per metre */
#define ORC_BIG 4503599627370496.0 /* 2^52: beyond this an offset is "far" */

/* ---------------------------------------------------------------- lattice -- */

/* Lattice coordinate of an offset in metres; 0 when it is non-finite or so far
 * away that it cannot be within any admissible radius of any node. */
static int orc_lattice(double off_m, int64_t *out)
{
    double t = off_m * ORC_Q;
    if (!(fabs(t) < ORC_BIG))
        return 0;
    *out = (int64_t)nearbyint(t); /* default rounding mode: nearest-even */
    return 1;
}

static int64_t orc_node_lattice(int32_t b, double d)
{
    double u = ((double)b + 0.5) * d;
    return (int64_t)nearbyint(u * ORC_Q);
}

static int orc_grid_ok(const orc_grid *g)
{
    if (!g || g->nx <= 0 || g->ny <= 0)
        return 0;
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !isfinite(g->dx) || !isfinite(g->dy))
        return 0;
    if (!isfinite(g->x0) || !isfinite(g->y0))
        return 0;
    /* node lattice must fit comfortably in 31 bits */
    if (((double)g->nx * g->dx) * ORC_Q >= 2147483648.0 * 0.5)
        return 0;
    if (((double)g->ny * g->dy) * ORC_Q >= 2147483648.0 * 0.5)
        return 0;
    return 1;
}

static int orc_radius_lattice(double radius, int64_t *R)
{
    if (!(radius > 0.0) || !(radius * ORC_Q < 1073741824.0))
        return 0;
    *R = (int64_t)nearbyint(radius * ORC_Q);
    return *R >= 1;
}

/* ------------------------------------------------------------------- bins -- */

int orc_bin_dims(const orc_grid *g, double radius, int32_t bin_log2,
                 int32_t *nbx, int32_t *nby, int32_t *halo)
{
    int64_t R;
    if (!orc_grid_ok(g) || !orc_radius_lattice(radius, &R))
        return ORC_EINVAL;
    if (bin_log2 < 4 || bin_log2 > 28)
        return ORC_EINVAL;
    int64_t B = (int64_t)1 << bin_log2;
    int64_t h = (R + B - 1) / B; /* ceil(R / B) */
    /* the last node plus R must fall in the last bin */
    int64_t xl = orc_node_lattice(g->nx - 1, g->dx) + R + h * B;
    int64_t yl = orc_node_lattice(g->ny - 1, g->dy) + R + h * B;
    int64_t bx = xl / B + 1, by = yl / B + 1;
    if (bx * B >= 2147483648LL || by * B >= 2147483648LL)
        return ORC_ERANGE;
    if (bx * by >= 2147483647LL)
        return ORC_ERANGE;
    *nbx = (int32_t)bx;
    *nby = (int32_t)by;
    *halo = (int32_t)h;
    return ORC_OK;
}

/* Bin id of a sounding, or -1 (non-finite) / -2 (outside the bin domain). */
static int64_t orc_bin_of(const orc_grid *g, double xi, double yi, double zi,
                          int32_t s, int64_t h, int64_t nbx, int64_t nby)
{
    if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi))
        return -1;
    int64_t X, Y;
    if (!orc_lattice(xi - g->x0, &X) || !orc_lattice(yi - g->y0, &Y))
        return -2;
    int64_t B = (int64_t)1 << s;
    int64_t ux = X + h * B, uy = Y + h * B;
    if (ux < 0 || uy < 0)
        return -2;
    int64_t bx = ux / B, by = uy / B;
    if (bx >= nbx || by >= nby)
        return -2;
    return by * nbx + bx;
}

int orc_bin(const orc_grid *g, const double *x, const double *y, const double *z,
            int64_t n, double radius, int32_t bin_log2, int32_t *cell_start,
            int32_t *perm, int64_t *n_binned, int64_t *n_invalid,
            int64_t *n_outside)
{
    int32_t nbx, nby, h;
    int rc = orc_bin_dims(g, radius, bin_log2, &nbx, &nby, &h);
    if (rc != ORC_OK)
        return rc;
    if (n < 0 || n >= 2147483647LL)
        return ORC_EINVAL;
    int64_t nb = (int64_t)nbx * nby;
    int64_t *id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!id)
        return ORC_ENOMEM;
    memset(cell_start, 0, sizeof(int32_t) * (size_t)(nb + 1));
    int64_t bad = 0, out = 0;
    /* pass 1: bin of every sounding and the count per bin */
    for (int64_t i = 0; i < n; ++i) {
        id[i] = orc_bin_of(g, x[i], y[i], z[i], bin_log2, h, nbx, nby);
        if (id[i] == -1)
            ++bad;
        else if (id[i] == -2)
            ++out;
        else
            cell_start[id[i] + 1] += 1;
    }
    /* exclusive prefix: cell_start[b] = number of soundings in bins < b */
    for (int64_t b = 0; b < nb; ++b)
        cell_start[b + 1] += cell_start[b];
    /* pass 2: place soundings in ascending original index -> stable */
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    if (!fill) {
        free(id);
        return ORC_ENOMEM;
    }
    memcpy(fill, cell_start, sizeof(int32_t) * (size_t)nb);
    for (int64_t i = 0; i < n; ++i)
        if (id[i] >= 0)
            perm[fill[id[i]]++] = (int32_t)i;
    free(fill);
    free(id);
    *n_binned = cell_start[nb];
    *n_invalid = bad;
    *n_outside = out;
    return ORC_OK;
}

/* ------------------------------------------------------- neighbour search -- */

typedef struct {
    int64_t d2; /* exact lattice squared distance */
    int64_t i;  /* original sounding index */
} orc_cand;

static int orc_cand_cmp(const void *pa, const void *pb)
{
    const orc_cand *a = (const orc_cand *)pa, *b = (const orc_cand *)pb;
    if (a->d2 != b->d2)
        return a->d2 < b->d2 ? -1 : 1;
    if (a->i != b->i)
        return a->i < b->i ? -1 : 1;
    return 0;
}

typedef struct {
    orc_cand *v;
    int64_t n, cap;
} orc_cbuf;

static int orc_push(orc_cbuf *c, int64_t d2, int64_t i)
{
    if (c->n == c->cap) {
        int64_t nc = c->cap ? 2 * c->cap : 64;
        orc_cand *nv = (orc_cand *)realloc(c->v, sizeof(orc_cand) * (size_t)nc);
        if (!nv)
            return 0;
        c->v = nv;
        c->cap = nc;
    }
    c->v[c->n].d2 = d2;
    c->v[c->n].i = i;
    c->n += 1;
    return 1;
}

/* Everything one search needs: soundings, their lattice coordinates, and the
 * bins when the binned search is used. */
typedef struct {
    const orc_grid *g;
    const double *x, *y, *z;
    int64_t n;
    int64_t R, R2;
    int64_t *X, *Y;  /* lattice coordinates */
    uint8_t *valid;  /* finite and representable */
    int32_t use_bins, s, h, nbx, nby;
    int32_t *cell_start, *perm;
} orc_search;

static void orc_search_free(orc_search *S)
{
    free(S->X);
    free(S->Y);
    free(S->valid);
    free(S->cell_start);
    free(S->perm);
}

static int orc_search_init(orc_search *S, const orc_grid *g, const double *x,
                           const double *y, const double *z, int64_t n,
                           double radius, int32_t bin_log2)
{
    memset(S, 0, sizeof(*S));
    if (!orc_grid_ok(g) || n < 0 || !orc_radius_lattice(radius, &S->R))
        return ORC_EINVAL;
    S->g = g;
    S->x = x;
    S->y = y;
    S->z = z;
    S->n = n;
    S->R2 = S->R * S->R;
    size_t m = (size_t)(n > 0 ? n : 1);
    S->X = (int64_t *)malloc(sizeof(int64_t) * m);
    S->Y = (int64_t *)malloc(sizeof(int64_t) * m);
    S->valid = (uint8_t *)malloc(m);
    if (!S->X || !S->Y || !S->valid) {
        orc_search_free(S);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        /* NaN / infinite soundings are invalid candidates */
        int ok = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]);
        ok = ok && orc_lattice(x[i] - g->x0, &S->X[i]);
        ok = ok && orc_lattice(y[i] - g->y0, &S->Y[i]);
        S->valid[i] = (uint8_t)ok;
    }
    if (bin_log2 >= 0) {
        int rc = orc_bin_dims(g, radius, bin_log2, &S->nbx, &S->nby, &S->h);
        if (rc != ORC_OK) {
            orc_search_free(S);
            return rc;
        }
        int64_t nb = (int64_t)S->nbx * S->nby;
        S->cell_start = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb + 1));
        S->perm = (int32_t *)malloc(sizeof(int32_t) * m);
        if (!S->cell_start || !S->perm) {
            orc_search_free(S);
            return ORC_ENOMEM;
        }
        int64_t nbin, nbad, nout;
        rc = orc_bin(g, x, y, z, n, radius, bin_log2, S->cell_start, S->perm,
                     &nbin, &nbad, &nout);
        if (rc != ORC_OK) {
            orc_search_free(S);
            return rc;
        }
        S->use_bins = 1;
        S->s = bin_log2;
    }
    return ORC_OK;
}

/* Membership test of sounding i against node lattice (Xn, Yn). */
static int orc_member(const orc_search *S, int64_t i, int64_t Xn, int64_t Yn,
                      int64_t *d2)
{
    if (!S->valid[i])
        return 0;
    int64_t ddx = S->X[i] - Xn, ddy = S->Y[i] - Yn;
    if (ddx > S->R || ddx < -S->R || ddy > S->R || ddy < -S->R)
        return 0;
    int64_t v = ddx * ddx + ddy * ddy;
    if (v > S->R2)
        return 0; /* the disk is closed: D^2 == R^2 is a member */
    *d2 = v;
    return 1;
}

/* C(n): every member of the node's disk, in no particular order. */
static int orc_collect(const orc_search *S, int64_t Xn, int64_t Yn, orc_cbuf *c)
{
    c->n = 0;
    int64_t d2;
    if (!S->use_bins) {
        for (int64_t i = 0; i < S->n; ++i)
            if (orc_member(S, i, Xn, Yn, &d2) && !orc_push(c, d2, i))
                return 0;
        return 1;
    }
    int64_t B = (int64_t)1 << S->s, hb = (int64_t)S->h * B;
    /* the bins that intersect [Xn - R, Xn + R] x [Yn - R, Yn + R] */
    int64_t bx0 = (Xn - S->R + hb) / B, bx1 = (Xn + S->R + hb) / B;
    int64_t by0 = (Yn - S->R + hb) / B, by1 = (Yn + S->R + hb) / B;
    for (int64_t by = by0; by <= by1; ++by)
        for (int64_t bx = bx0; bx <= bx1; ++bx) {
            int64_t id = by * S->nbx + bx;
            for (int32_t k = S->cell_start[id]; k < S->cell_start[id + 1]; ++k) {
                int64_t i = S->perm[k];
                if (orc_member(S, i, Xn, Yn, &d2) && !orc_push(c, d2, i))
                    return 0;
            }
        }
    return 1;
}

/* ------------------------------------------------------------------- IDW -- */

/* One node of O1, steps in order:
 *   1. C(n) = members of the closed lattice disk;
 *   2. S(n) = the first min(|C|, k) of C sorted by (D^2, original index);
 *   3. hits: members of S with D^2 == 0 -> their mean depth (ascending index),
 *      which takes precedence over min_pts;
 *   4. |S| < min_pts -> NaN;
 *   5. w_i = d_i^-p with d_i = hypot of the double offsets to the node;
 *   6. z = z0 + sum w_i (z_i - z0) / sum w_i, z0 the first of S, sums in S
 *      order, then clamped to [min, max] of the depths in S. */
static void orc_idw_node(const orc_search *S, double power, int32_t min_pts,
                         int32_t max_pts, int64_t a, int64_t b, orc_cbuf *c,
                         double *zo, int32_t *cnto, int32_t *nno, int *err)
{
    const orc_grid *g = S->g;
    int64_t Xn = orc_node_lattice((int32_t)b, g->dx);
    int64_t Yn = orc_node_lattice((int32_t)a, g->dy);
    double xn = g->x0 + ((double)b + 0.5) * g->dx;
    double yn = g->y0 + ((double)a + 0.5) * g->dy;
    if (!orc_collect(S, Xn, Yn, c)) {
        *err = 1;
        return;
    }
    qsort(c->v, (size_t)c->n, sizeof(orc_cand), orc_cand_cmp);
    int64_t m = c->n;
    if (max_pts > 0 && m > max_pts)
        m = max_pts;
    *cnto = (int32_t)m;
    *nno = m > 0 ? (int32_t)c->v[0].i : -1;

    int64_t hits = 0;
    double hsum = 0.0;
    while (hits < m && c->v[hits].d2 == 0) {
        hsum += S->z[c->v[hits].i];
        ++hits;
    }
    if (hits > 0) {
        *zo = hsum / (double)hits;
        return;
    }
    if (m < min_pts || m == 0) {
        *zo = NAN;
        return;
    }
    double z0 = S->z[c->v[0].i];
    double num = 0.0, den = 0.0, zmin = z0, zmax = z0;
    for (int64_t j = 0; j < m; ++j) {
        int64_t i = c->v[j].i;
        double d = hypot(S->x[i] - xn, S->y[i] - yn);
        double w = pow(d, -power);
        num += w * (S->z[i] - z0);
        den += w;
        if (S->z[i] < zmin)
            zmin = S->z[i];
        if (S->z[i] > zmax)
            zmax = S->z[i];
    }
    double v = z0 + num / den;
    if (v < zmin)
        v = zmin;
    if (v > zmax)
        v = zmax;
    *zo = v;
}

static int orc_nodes_ok(const orc_grid *g, const int64_t *nodes, int64_t n_nodes)
{
    if (!nodes)
        return 1;
    int64_t total = (int64_t)g->nx * g->ny;
    for (int64_t k = 0; k < n_nodes; ++k)
        if (nodes[k] < 0 || nodes[k] >= total)
            return 0;
    return 1;
}

int orc_idw(const orc_grid *g, const double *x, const double *y, const double *z,
            int64_t n, double radius, double power, int32_t min_pts,
            int32_t max_pts, int32_t bin_log2, const int64_t *nodes,
            int64_t n_nodes, double *z_out, int32_t *cnt_out, int32_t *nn_out,
            int32_t nthreads)
{
    if (!(power > 0.0) || !isfinite(power) || max_pts < 0 || min_pts < 0)
        return ORC_EINVAL;
    orc_search S;
    int rc = orc_search_init(&S, g, x, y, z, n, radius, bin_log2);
    if (rc != ORC_OK)
        return rc;
    if (!orc_nodes_ok(g, nodes, n_nodes)) {
        orc_search_free(&S);
        return ORC_EINVAL;
    }
    int64_t total = nodes ? n_nodes : (int64_t)g->nx * g->ny;
    int err = 0;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
    {
        orc_cbuf c = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < total; ++k) {
            int64_t f = nodes ? nodes[k] : k;
            int32_t cnt = 0, nn = -1;
            orc_idw_node(&S, power, min_pts, max_pts, f / g->nx, f % g->nx, &c,
                         &z_out[k], &cnt, &nn, &err);
            if (cnt_out)
                cnt_out[k] = cnt;
            if (nn_out)
                nn_out[k] = nn;
        }
        free(c.v);
    }
    orc_search_free(&S);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* Bounds of O1's selected set: the smallest and largest depth over S(n)
 * (steps 1-2 of O1: the closed lattice disk, ranked by (D^2, original index)
 * and cut to the first max_pts).  Every O1 value lies within them (step 6
 * clamps to them); NaN for both when S(n) is empty. */
int orc_idw_bounds(const orc_grid *g, const double *x, const double *y, const double *z,
                   int64_t n, double radius, int32_t max_pts, int32_t bin_log2,
                   const int64_t *nodes, int64_t n_nodes, double *lo_out, double *hi_out,
                   int32_t nthreads)
{
    if (max_pts < 0)
        return ORC_EINVAL;
    orc_search S;
    int rc = orc_search_init(&S, g, x, y, z, n, radius, bin_log2);
    if (rc != ORC_OK)
        return rc;
    if (!orc_nodes_ok(g, nodes, n_nodes)) {
        orc_search_free(&S);
        return ORC_EINVAL;
    }
    int64_t total = nodes ? n_nodes : (int64_t)g->nx * g->ny;
    int err = 0;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
    {
        orc_cbuf c = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < total; ++k) {
            int64_t f = nodes ? nodes[k] : k;
            int64_t Xn = orc_node_lattice((int32_t)(f % g->nx), g->dx);
            int64_t Yn = orc_node_lattice((int32_t)(f / g->nx), g->dy);
            if (!orc_collect(&S, Xn, Yn, &c)) {
                err = 1;
                continue;
            }
            qsort(c.v, (size_t)c.n, sizeof(orc_cand), orc_cand_cmp);
            int64_t m = c.n;
            if (max_pts > 0 && m > max_pts)
                m = max_pts;
            double lo = NAN, hi = NAN;
            for (int64_t j = 0; j < m; ++j) {
                double v = z[c.v[j].i];
                if (j == 0 || v < lo)
                    lo = v;
                if (j == 0 || v > hi)
                    hi = v;
            }
            lo_out[k] = lo;
            hi_out[k] = hi;
        }
        free(c.v);
    }
    orc_search_free(&S);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* -------------------------------------------------------------------- NN -- */

/* O2: argmin of (D^2, original index) over the disk, computed directly (no
 * sort) so that it checks the ranking used by O1. */
int orc_nearest(const orc_grid *g, const double *x, const double *y,
                const double *z, int64_t n, double radius, int32_t bin_log2,
                const int64_t *nodes, int64_t n_nodes, int32_t *idx_out,
                double *z_out, int32_t nthreads)
{
    orc_search S;
    int rc = orc_search_init(&S, g, x, y, z, n, radius, bin_log2);
    if (rc != ORC_OK)
        return rc;
    if (!orc_nodes_ok(g, nodes, n_nodes)) {
        orc_search_free(&S);
        return ORC_EINVAL;
    }
    int64_t total = nodes ? n_nodes : (int64_t)g->nx * g->ny;
    int err = 0;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
    {
        orc_cbuf c = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < total; ++k) {
            int64_t f = nodes ? nodes[k] : k;
            int64_t Xn = orc_node_lattice((int32_t)(f % g->nx), g->dx);
            int64_t Yn = orc_node_lattice((int32_t)(f / g->nx), g->dy);
            if (!orc_collect(&S, Xn, Yn, &c)) {
                err = 1;
                continue;
            }
            int64_t best = -1, bd2 = 0;
            for (int64_t j = 0; j < c.n; ++j) {
                int64_t d2 = c.v[j].d2, i = c.v[j].i;
                if (best < 0 || d2 < bd2 || (d2 == bd2 && i < best)) {
                    best = i;
                    bd2 = d2;
                }
            }
            idx_out[k] = (int32_t)best;
            z_out[k] = best >= 0 ? z[best] : NAN;
        }
        free(c.v);
    }
    orc_search_free(&S);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* -------------------------------------------------------------- bilinear -- */

/* Source index coordinate of a destination node along one axis, clamped to
 * [0, n-1], split into the lower corner index, the upper corner index and the
 * fractional position t in [0, 1). */
static void orc_axis(double x0d, double dd, int32_t j, double x0s, double ds,
                     int32_t ns, int32_t *i0, int32_t *i1, double *t)
{
    double xd = x0d + ((double)j + 0.5) * dd;
    double u = (xd - x0s) / ds - 0.5;
    if (u < 0.0)
        u = 0.0;
    if (u > (double)(ns - 1))
        u = (double)(ns - 1);
    double f = floor(u);
    *i0 = (int32_t)f;
    *i1 = *i0 + 1 < ns ? *i0 + 1 : ns - 1;
    *t = u - f;
}

/* Sec. III-A in index units at one destination node: x1 = i0, x2 = i0 + 1,
 * y1 = j0, y2 = j0 + 1, so (x2 - x1)(y2 - y1) = 1.  NaN when a corner is. */
static double orc_bilinear_at(const orc_grid *sg, const double *src, int32_t i0, int32_t i1,
                              double t, int32_t j0, int32_t j1, double s)
{
    double q11 = src[(int64_t)j0 * sg->nx + i0];
    double q21 = src[(int64_t)j0 * sg->nx + i1];
    double q12 = src[(int64_t)j1 * sg->nx + i0];
    double q22 = src[(int64_t)j1 * sg->nx + i1];
    double x2mx = 1.0 - t, xmx1 = t, y2my = 1.0 - s, ymy1 = s;
    double v = x2mx * y2my * q11 + xmx1 * y2my * q21 + x2mx * ymy1 * q12 + xmx1 * ymy1 * q22;
    if (isnan(q11) || isnan(q21) || isnan(q12) || isnan(q22))
        v = NAN; /* no fallback: a hole */
    return v;
}

int orc_bilinear(const orc_grid *sg, const double *src, const orc_grid *dg,
                 double *dst, int32_t nthreads)
{
    if (!orc_grid_ok(sg) || !orc_grid_ok(dg))
        return ORC_EINVAL;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t a = 0; a < dg->ny; ++a) {
        int32_t j0, j1;
        double s;
        orc_axis(dg->y0, dg->dy, (int32_t)a, sg->y0, sg->dy, sg->ny, &j0, &j1, &s);
        for (int32_t b = 0; b < dg->nx; ++b) {
            int32_t i0, i1;
            double t;
            orc_axis(dg->x0, dg->dx, b, sg->x0, sg->dx, sg->nx, &i0, &i1, &t);
            dst[a * dg->nx + b] = orc_bilinear_at(sg, src, i0, i1, t, j0, j1, s);
        }
    }
    return ORC_OK;
}

/* Catmull-Rom cubic through four equally spaced samples, at parameter t in
 * [0, 1] between P1 and P2 (Sec. III-B). */
static double orc_catmull_rom(double p0, double p1, double p2, double p3, double t)
{
    return 0.5 * (2.0 * p1 + (-p0 + p2) * t + (2.0 * p0 - 5.0 * p1 + 4.0 * p2 - p3) * t * t +
                  (-p0 + 3.0 * p1 - 3.0 * p2 + p3) * t * t * t);
}

static int32_t orc_clamp_index(int32_t v, int32_t n)
{
    return v < 0 ? 0 : (v > n - 1 ? n - 1 : v);
}

int orc_bicubic(const orc_grid *sg, const double *src, const orc_grid *dg,
                double *dst, int32_t nthreads)
{
    if (!orc_grid_ok(sg) || !orc_grid_ok(dg))
        return ORC_EINVAL;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t a = 0; a < dg->ny; ++a) {
        int32_t j0, j1;
        double s;
        orc_axis(dg->y0, dg->dy, (int32_t)a, sg->y0, sg->dy, sg->ny, &j0, &j1, &s);
        for (int32_t b = 0; b < dg->nx; ++b) {
            int32_t i0, i1;
            double t;
            orc_axis(dg->x0, dg->dx, b, sg->x0, sg->dx, sg->nx, &i0, &i1, &t);
            /* 4 x 4 taps around the cell (index clamped at the edges): first
             * along x on each of the 4 rows, then along y over the 4 results */
            double col[4];
            int any_nan = 0;
            for (int r = 0; r < 4; ++r) {
                const double *row = src + (int64_t)orc_clamp_index(j0 - 1 + r, sg->ny) * sg->nx;
                double p[4];
                for (int c = 0; c < 4; ++c) {
                    p[c] = row[orc_clamp_index(i0 - 1 + c, sg->nx)];
                    any_nan |= !isfinite(p[c]);
                }
                col[r] = orc_catmull_rom(p[0], p[1], p[2], p[3], t);
            }
            double v = orc_catmull_rom(col[0], col[1], col[2], col[3], s);
            if (any_nan) /* an invalid neighbour: bilinear (may be a hole) */
                v = orc_bilinear_at(sg, src, i0, i1, t, j0, j1, s);
            dst[a * dg->nx + b] = v;
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- kriging -- */

/* Exponential variogram (Sec. III-C) with unit sill: the sill scales the
 * whole system and cancels from the weights. */
static double orc_gamma(double h, double a) { return 1.0 - exp(-h / a); }

/* Solve A x = b (n x n, row-major, overwritten) by Gaussian elimination with
 * partial pivoting.  Returns 0 when a pivot vanishes. */
static int orc_gauss_solve(double *A, double *b, int n)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[p * n + c]))
                p = r;
        if (A[p * n + c] == 0.0)
            return 0;
        if (p != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k];
                A[c * n + k] = A[p * n + k];
                A[p * n + k] = t;
            }
            double t = b[c];
            b[c] = b[p];
            b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k)
                A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double v = b[r];
        for (int k = r + 1; k < n; ++k)
            v -= A[r * n + k] * b[k];
        b[r] = v / A[r * n + r];
    }
    return 1;
}

/* First index of the 5-node window centred on the node nearest to index
 * coordinate u (already clamped to [0, n-1]), moved inward at the edges. */
static int32_t orc_window_start(double u, int32_t n)
{
    int32_t c = (int32_t)floor(u + 0.5);
    int32_t s = c - 2;
    if (s > n - 5)
        s = n - 5;
    if (s < 0)
        s = 0;
    return s;
}

int orc_kriging(const orc_grid *sg, const double *src, const orc_grid *dg, double range,
                double *dst, int32_t nthreads)
{
    if (!orc_grid_ok(sg) || !orc_grid_ok(dg) || !(range > 0.0) || !isfinite(range))
        return ORC_EINVAL;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
    const int small = sg->nx < 5 || sg->ny < 5;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t a = 0; a < dg->ny; ++a) {
        int32_t j0, j1;
        double s;
        orc_axis(dg->y0, dg->dy, (int32_t)a, sg->y0, sg->dy, sg->ny, &j0, &j1, &s);
        for (int32_t b = 0; b < dg->nx; ++b) {
            int32_t i0, i1;
            double t;
            orc_axis(dg->x0, dg->dx, b, sg->x0, sg->dx, sg->nx, &i0, &i1, &t);
            double v;
            int ok = !small;
            int32_t wx = 0, wy = 0;
            if (ok) {
                /* the destination point in source index units (as bilinear) */
                double u = i0 + t, w = j0 + s;
                wx = orc_window_start(u, sg->nx);
                wy = orc_window_start(w, sg->ny);
                for (int k = 0; k < 25 && ok; ++k)
                    ok = isfinite(src[(int64_t)(wy + k / 5) * sg->nx + wx + k % 5]);
            }
            if (ok) {
                /* ordinary kriging system: variogram between the 25 window
                 * nodes, the unbiasedness row and column, and the variogram
                 * between each node and the destination point */
                double A[26 * 26], rhs[26];
                double u = i0 + t, w = j0 + s;
                for (int p = 0; p < 25; ++p) {
                    double xp = (wx + p % 5) * sg->dx, yp = (wy + p / 5) * sg->dy;
                    for (int q = 0; q < 25; ++q) {
                        double xq = (wx + q % 5) * sg->dx, yq = (wy + q / 5) * sg->dy;
                        A[p * 26 + q] = orc_gamma(hypot(xp - xq, yp - yq), range);
                    }
                    A[p * 26 + 25] = 1.0;
                    A[25 * 26 + p] = 1.0;
                    rhs[p] = orc_gamma(hypot(xp - u * sg->dx, yp - w * sg->dy), range);
                }
                A[25 * 26 + 25] = 0.0;
                rhs[25] = 1.0;
                if (orc_gauss_solve(A, rhs, 26)) {
                    v = 0.0;
                    for (int p = 0; p < 25; ++p)
                        v += rhs[p] * src[(int64_t)(wy + p / 5) * sg->nx + wx + p % 5];
                } else {
                    v = orc_bilinear_at(sg, src, i0, i1, t, j0, j1, s);
                }
            } else {
                /* an invalid neighbour (or a grid under 5 x 5): bilinear */
                v = orc_bilinear_at(sg, src, i0, i1, t, j0, j1, s);
            }
            dst[a * dg->nx + b] = v;
        }
    }
    return ORC_OK;
}

/* -------------------------------------------------------------- variogram -- */

/* O7: empirical semivariogram along the grid axes (the classical method-of-
 * moments estimator): for lag k = 1..nlags, the pairs (row a, column b) and
 * (a, b + k) with both values finite give
 *     gamma_x[k-1] = sum (z1 - z2)^2 / (2 * pairs_x[k-1])   (lag k * dx),
 * the pairs (a, b) and (a + k, b) likewise gamma_y (lag k * dy); NaN where a
 * lag has no pair.  The paper leaves the variogram's parameters unstated
 * (Sec. III-C); this is the data the fit below reads. */
int orc_variogram(const orc_grid *g, const double *src, int32_t nlags, double *gamma_x,
                  double *gamma_y, int64_t *pairs_x, int64_t *pairs_y)
{
    if (!orc_grid_ok(g) || nlags < 1)
        return ORC_EINVAL;
    for (int32_t k = 1; k <= nlags; ++k) {
        double sx = 0.0, sy = 0.0;
        int64_t cx = 0, cy = 0;
        for (int64_t a = 0; a < g->ny; ++a) {
            for (int64_t b = 0; b < g->nx; ++b) {
                const double z1 = src[a * g->nx + b];
                if (!isfinite(z1))
                    continue;
                if (b + k < g->nx) {
                    const double z2 = src[a * g->nx + b + k];
                    if (isfinite(z2)) {
                        sx += (z1 - z2) * (z1 - z2);
                        cx += 1;
                    }
                }
                if (a + k < g->ny) {
                    const double z2 = src[(a + k) * g->nx + b];
                    if (isfinite(z2)) {
                        sy += (z1 - z2) * (z1 - z2);
                        cy += 1;
                    }
                }
            }
        }
        gamma_x[k - 1] = cx > 0 ? sx / (2.0 * (double)cx) : NAN;
        gamma_y[k - 1] = cy > 0 ? sy / (2.0 * (double)cy) : NAN;
        if (pairs_x)
            pairs_x[k - 1] = cx;
        if (pairs_y)
            pairs_y[k - 1] = cy;
    }
    return ORC_OK;
}

/* Weighted residual of the exponential model at range a, with the sill at its
 * least-squares value for that range (the model is linear in the sill). */
static double orc_exp_residual(const double *h, const double *gam, const double *w, int32_t n,
                               double a, double *sill)
{
    double sgf = 0.0, sff = 0.0, sgg = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        if (!(w[j] > 0.0) || !isfinite(gam[j]))
            continue;
        const double f = 1.0 - exp(-h[j] / a);
        sgf += w[j] * gam[j] * f;
        sff += w[j] * f * f;
        sgg += w[j] * gam[j] * gam[j];
    }
    const double c = sff > 0.0 ? sgf / sff : 0.0;
    if (sill)
        *sill = c;
    return sgg - 2.0 * c * sgf + c * c * sff;
}

/* O8: weighted least-squares fit of gamma(h) = C0 (1 - exp(-h / a)) to n
 * points (h_j > 0 in metres, gamma_j, weights w_j >= 0; points with zero
 * weight or a non-finite gamma are ignored): the range a minimises the
 * residual with C0 at its least-squares value for that a.  a is searched on a
 * log grid of 20001 values from min(h) / 100 to 1000 max(h), then refined by
 * ternary search between the grid neighbours of the best value.  Returns
 * ORC_EINVAL for no usable point, ORC_ERANGE when the best range is an end of
 * the grid (no sill within it). */
int orc_fit_exponential(const double *h, const double *gam, const double *w, int32_t n,
                        double *range, double *sill)
{
    double hmin = INFINITY, hmax = 0.0;
    int32_t used = 0;
    for (int32_t j = 0; j < n; ++j) {
        if (!(w[j] > 0.0) || !isfinite(gam[j]) || !(h[j] > 0.0))
            continue;
        hmin = fmin(hmin, h[j]);
        hmax = fmax(hmax, h[j]);
        ++used;
    }
    if (used < 2)
        return ORC_EINVAL;
    const int32_t m = 20001;
    const double l0 = log(hmin / 100.0), l1 = log(1000.0 * hmax);
    int32_t best = 0;
    double best_r = INFINITY;
    for (int32_t i = 0; i < m; ++i) {
        const double a = exp(l0 + (l1 - l0) * (double)i / (double)(m - 1));
        const double r = orc_exp_residual(h, gam, w, n, a, NULL);
        if (r < best_r) {
            best_r = r;
            best = i;
        }
    }
    if (best == 0 || best == m - 1) {
        *range = exp(best == 0 ? l0 : l1);
        orc_exp_residual(h, gam, w, n, *range, sill);
        return ORC_ERANGE;
    }
    double lo = l0 + (l1 - l0) * (double)(best - 1) / (double)(m - 1);
    double hi = l0 + (l1 - l0) * (double)(best + 1) / (double)(m - 1);
    for (int it = 0; it < 200; ++it) {
        const double p = lo + (hi - lo) / 3.0, q = hi - (hi - lo) / 3.0;
        if (orc_exp_residual(h, gam, w, n, exp(p), NULL) <=
            orc_exp_residual(h, gam, w, n, exp(q), NULL))
            hi = q;
        else
            lo = p;
    }
    *range = exp(0.5 * (lo + hi));
    orc_exp_residual(h, gam, w, n, *range, sill);
    return ORC_OK;
}
