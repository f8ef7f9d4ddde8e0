/*
 * oracle.c -- plain brute-force CPU oracle for point-in-polygon selection,
 * polygon-point join pairs and polygon-point aggregation (join-count).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The product
 * path never calls it and shares no code, header or table with it.
 *
 * What it computes (the plain definition, no canvas, no rasterisation):
 *
 *   Queries (paper Sec. 5.2 "Spatial Selection", "Spatial Joins",
 *   "Spatial Aggregations"):
 *     select(D, P)   = ascending { i : inside(p_i, P) }           (selection
 *                      with a polygonal constraint, intersection predicate;
 *                      for points intersection equals containment, Sec. 7)
 *     pairs(D, {P})  = { (i, k) : inside(p_i, P_k) } ascending by (i, k)
 *                      (polygon-point join = one selection per polygon)
 *     counts[k]      = #{ i : inside(p_i, P_k) }  (aggregation plan that
 *                      never materialises the join)
 *
 *   inside(p, P)   = XOR over every edge e=(a,b) of every ring of P of
 *                    cross(e, p)                 (even-odd crossing number)
 *   cross(e, p)    = [(a.y > p.y) != (b.y > p.y)] AND orient(lo, hi, p) > 0
 *                    with (lo, hi) = (a, b) ordered so lo.y < hi.y, and
 *   orient(a,b,c)  = (b.x-a.x)(c.y-a.y) - (b.y-a.y)(c.x-a.x)  evaluated EXACTLY.
 *
 *   The straddle test is half-open in y (lo.y <= p.y < hi.y) and a point on
 *   the supporting line of an edge is never counted as a crossing.  This is
 *   the symbolic perturbation p -> p + (eps, eps^2): a boundary point belongs
 *   to the polygon on its +x side (above, for a horizontal edge), so in a
 *   tessellation every point of the union is counted exactly once.  The paper
 *   does not fix boundary semantics; this is the reading the whole project
 *   uses.  Horizontal and zero-length edges never straddle and so never count.
 *
 * Exact orient: a floating-point filter with the a-priori error bound of
 * Shewchuk (1997, "Adaptive precision floating-point arithmetic and fast
 * robust geometric predicates", the orient2d bound (3+16 eps) eps (|l|+|r|)),
 * evaluated with contraction disabled; when the filter cannot decide, the six
 * products of the expanded determinant are summed exactly in a plain
 * big-integer accumulator (each double = integer mantissa * 2^exponent).
 * Exactness domain: finite inputs whose products neither overflow nor
 * underflow into subnormals (|coordinates| up to about 2^500).
 *
 * Pruning is limited to exact filters: a half-open bounding-box reject
 * (xmin <= x < xmax and ymin <= y < ymax is necessary for inside(): a point
 * with x >= xmax has no edge crossing strictly to its right, one with
 * y >= ymax or y < ymin straddles no edge, and one with x < xmin sees every
 * straddling edge to its right, an even number for a closed ring) and, for
 * many polygons, a uniform grid over polygon bounding boxes that only lists
 * candidates.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#pragma STDC FP_CONTRACT OFF

/* ------------------------------------------------------------------ */
/* Exact orientation sign                                              */
/* ------------------------------------------------------------------ */

/* Decompose a finite double into sign, 53-bit integer mantissa and exponent
 * so that v = sign * m * 2^e exactly (m == 0 for v == 0). */
static void split_double(double v, int *sign, uint64_t *m, int *e)
{
    if (v == 0.0) { *sign = 0; *m = 0; *e = 0; return; }
    *sign = v < 0 ? -1 : 1;
    int ex;
    double fr = frexp(fabs(v), &ex);        /* fr in [0.5, 1) */
    /* fr * 2^53 is an integer below 2^53 for normal and subnormal inputs */
    *m = (uint64_t)ldexp(fr, 53);
    *e = ex - 53;
}

#define BIG_LIMBS 80   /* 5120 bits: products span exponents -2148 .. 2046 */

typedef struct { uint64_t w[BIG_LIMBS]; } big_t;

/* acc += v * 2^shift, v an unsigned 128-bit value, shift >= 0. */
static void big_add_shifted(big_t *acc, unsigned __int128 v, int shift)
{
    int limb = shift / 64, bit = shift % 64;
    /* v << bit spans at most three limbs */
    uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
    uint64_t parts[3];
    if (bit == 0) { parts[0] = lo; parts[1] = hi; parts[2] = 0; }
    else {
        parts[0] = lo << bit;
        parts[1] = (hi << bit) | (lo >> (64 - bit));
        parts[2] = hi >> (64 - bit);
    }
    unsigned __int128 carry = 0;
    for (int k = limb; k < BIG_LIMBS; ++k) {
        unsigned __int128 s = (unsigned __int128)acc->w[k] + carry;
        if (k - limb < 3) s += parts[k - limb];
        acc->w[k] = (uint64_t)s;
        carry = s >> 64;
        if (k - limb >= 2 && carry == 0) break;
    }
}

static int big_cmp(const big_t *a, const big_t *b)
{
    for (int k = BIG_LIMBS - 1; k >= 0; --k) {
        if (a->w[k] != b->w[k]) return a->w[k] > b->w[k] ? 1 : -1;
    }
    return 0;
}

/* Sign of sum_t s_t * u_t * v_t over six products, exactly. */
static int exact_sum_of_products(const double u[6], const double v[6], const int s[6])
{
    int sg[6], ex[6];
    unsigned __int128 mag[6];
    int emin = 1 << 30, any = 0;
    for (int t = 0; t < 6; ++t) {
        int su, sv, eu, ev;
        uint64_t mu, mv;
        split_double(u[t], &su, &mu, &eu);
        split_double(v[t], &sv, &mv, &ev);
        sg[t] = su * sv * s[t];
        mag[t] = (unsigned __int128)mu * mv;
        ex[t] = eu + ev;
        if (sg[t] != 0) { any = 1; if (ex[t] < emin) emin = ex[t]; }
    }
    if (!any) return 0;
    big_t pos, neg;
    memset(&pos, 0, sizeof pos);
    memset(&neg, 0, sizeof neg);
    for (int t = 0; t < 6; ++t) {
        if (sg[t] == 0) continue;
        big_add_shifted(sg[t] > 0 ? &pos : &neg, mag[t], ex[t] - emin);
    }
    return big_cmp(&pos, &neg);
}

static int g_use_filter = 1;

/* Test hook: 0 forces every orientation through the exact big-integer path. */
void orc_set_filter(int on) { g_use_filter = on; }

/* sign of (bx-ax)(cy-ay) - (by-ay)(cx-ax), exactly. */
int orc_orient_sign(double ax, double ay, double bx, double by, double cx, double cy)
{
    if (g_use_filter) {
        double detleft = (bx - ax) * (cy - ay);
        double detright = (by - ay) * (cx - ax);
        double det = detleft - detright;
        const double eps = DBL_EPSILON * 0.5;                 /* 2^-53 */
        const double errbound = (3.0 + 16.0 * eps) * eps;
        double bound = errbound * (fabs(detleft) + fabs(detright));
        if (det > bound) return 1;
        if (-det > bound) return -1;
    }
    /* Expanded determinant: ax*by - ax*cy + bx*cy - bx*ay + cx*ay - cx*by */
    const double u[6] = { ax, ax, bx, bx, cx, cx };
    const double v[6] = { by, cy, cy, ay, ay, by };
    const int s[6] = { +1, -1, +1, -1, +1, -1 };
    return exact_sum_of_products(u, v, s);
}

/* ------------------------------------------------------------------ */
/* Crossing-number containment                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n_polys;
    const int64_t *poly_ring_off;   /* [n_polys+1] or NULL: ring i == polygon i */
    const int64_t *ring_vtx_off;    /* [n_rings+1] */
    const double *vx, *vy;
} orc_polys;

static int64_t ring_begin(const orc_polys *P, int64_t k)
{ return P->poly_ring_off ? P->poly_ring_off[k] : k; }
static int64_t ring_end(const orc_polys *P, int64_t k)
{ return P->poly_ring_off ? P->poly_ring_off[k + 1] : k + 1; }

/* cross(e, p) for the edge a->b */
static int crosses(double ax, double ay, double bx, double by, double px, double py)
{
    if ((ay > py) == (by > py)) return 0;
    if (ay < by) return orc_orient_sign(ax, ay, bx, by, px, py) > 0;
    return orc_orient_sign(bx, by, ax, ay, px, py) > 0;
}

static int inside_poly(const orc_polys *P, int64_t k, double px, double py)
{
    int par = 0;
    for (int64_t r = ring_begin(P, k); r < ring_end(P, k); ++r) {
        int64_t v0 = P->ring_vtx_off[r], v1 = P->ring_vtx_off[r + 1];
        int64_t n = v1 - v0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t a = v0 + j, b = v0 + (j + 1) % n;
            par ^= crosses(P->vx[a], P->vy[a], P->vx[b], P->vy[b], px, py);
        }
    }
    return par;
}

int orc_inside(double px, double py, int64_t n_polys, const int64_t *poly_ring_off,
               const int64_t *ring_vtx_off, const double *vx, const double *vy, int64_t k)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    return inside_poly(&P, k, px, py);
}

/* ------------------------------------------------------------------ */
/* Candidate filter: half-open bounding boxes + uniform grid           */
/* ------------------------------------------------------------------ */

static int g_use_grid = 1;

/* Test hook: 0 makes every candidate filter a single cell listing every
 * polygon (bounding-box rejects only), so the grid can be checked against it. */
void orc_set_grid(int on) { g_use_grid = on; }

typedef struct {
    double *xmin, *xmax, *ymin, *ymax;  /* per polygon */
    int G;                              /* grid is G x G over the union bbox */
    double gx0, gy0, gsx, gsy;          /* cell = floor((x-gx0)*gsx) */
    int64_t *cell_off;                  /* [G*G+1] */
    int64_t *cell_items;                /* polygon ids */
} orc_filter;

static void filter_build(const orc_polys *P, orc_filter *F)
{
    int64_t M = P->n_polys;
    F->xmin = malloc(sizeof(double) * (M ? M : 1));
    F->xmax = malloc(sizeof(double) * (M ? M : 1));
    F->ymin = malloc(sizeof(double) * (M ? M : 1));
    F->ymax = malloc(sizeof(double) * (M ? M : 1));
    double ux0 = INFINITY, ux1 = -INFINITY, uy0 = INFINITY, uy1 = -INFINITY;
    for (int64_t k = 0; k < M; ++k) {
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int64_t r = ring_begin(P, k); r < ring_end(P, k); ++r)
            for (int64_t v = P->ring_vtx_off[r]; v < P->ring_vtx_off[r + 1]; ++v) {
                if (P->vx[v] < x0) x0 = P->vx[v];
                if (P->vx[v] > x1) x1 = P->vx[v];
                if (P->vy[v] < y0) y0 = P->vy[v];
                if (P->vy[v] > y1) y1 = P->vy[v];
            }
        F->xmin[k] = x0; F->xmax[k] = x1; F->ymin[k] = y0; F->ymax[k] = y1;
        if (x0 <= x1) {
            if (x0 < ux0) ux0 = x0;
            if (x1 > ux1) ux1 = x1;
            if (y0 < uy0) uy0 = y0;
            if (y1 > uy1) uy1 = y1;
        }
    }
    /* Grid only pays for many polygons; G == 1 lists every polygon. */
    int G = 1;
    if (g_use_grid && M > 64 && ux0 < ux1 && uy0 < uy1) {
        double g = sqrt((double)M);
        G = (int)(g < 1024 ? g : 1024);
        if (G < 1) G = 1;
    }
    F->G = G;
    F->gx0 = ux0; F->gy0 = uy0;
    F->gsx = (G > 1) ? G / (ux1 - ux0) : 0.0;
    F->gsy = (G > 1) ? G / (uy1 - uy0) : 0.0;
    int64_t ncell = (int64_t)G * G;
    F->cell_off = calloc(ncell + 1, sizeof(int64_t));
    /* each bbox is listed in every cell it overlaps, widened by one cell so
       that rounding in a point's cell index can never drop a candidate */
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *fill = NULL;
        if (pass == 1) {
            for (int64_t c = 0; c < ncell; ++c) F->cell_off[c + 1] += F->cell_off[c];
            F->cell_items = malloc(sizeof(int64_t) * (F->cell_off[ncell] ? F->cell_off[ncell] : 1));
            fill = calloc(ncell, sizeof(int64_t));
        }
        for (int64_t k = 0; k < M; ++k) {
            if (!(F->xmin[k] < F->xmax[k] && F->ymin[k] < F->ymax[k])) continue;  /* empty */
            int cx0 = 0, cx1 = G - 1, cy0 = 0, cy1 = G - 1;
            if (G > 1) {
                cx0 = (int)floor((F->xmin[k] - ux0) * F->gsx) - 1;
                cx1 = (int)floor((F->xmax[k] - ux0) * F->gsx) + 1;
                cy0 = (int)floor((F->ymin[k] - uy0) * F->gsy) - 1;
                cy1 = (int)floor((F->ymax[k] - uy0) * F->gsy) + 1;
                if (cx0 < 0) cx0 = 0;
                if (cy0 < 0) cy0 = 0;
                if (cx1 > G - 1) cx1 = G - 1;
                if (cy1 > G - 1) cy1 = G - 1;
            }
            for (int cy = cy0; cy <= cy1; ++cy)
                for (int cx = cx0; cx <= cx1; ++cx) {
                    int64_t c = (int64_t)cy * G + cx;
                    if (pass == 0) F->cell_off[c + 1]++;
                    else F->cell_items[F->cell_off[c] + fill[c]++] = k;
                }
        }
        free(fill);
    }
}

static void filter_free(orc_filter *F)
{
    free(F->xmin); free(F->xmax); free(F->ymin); free(F->ymax);
    free(F->cell_off); free(F->cell_items);
}

/* Grid side the candidate filter uses for a polygon set (test hook). */
int orc_filter_grid(int64_t n_polys, const int64_t *poly_ring_off, const int64_t *ring_vtx_off,
                    const double *vx, const double *vy)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    orc_filter F;
    filter_build(&P, &F);
    int G = F.G;
    filter_free(&F);
    return G;
}

/* Candidate polygons for a point: returns the grid cell, or -1 if the point
 * lies outside the union bbox (or is NaN) and so inside no polygon. */
static int64_t filter_cell(const orc_filter *F, double x, double y)
{
    if (!(x >= F->gx0 && y >= F->gy0)) return -1;   /* also rejects NaN */
    if (F->G == 1) return 0;
    double fx = floor((x - F->gx0) * F->gsx), fy = floor((y - F->gy0) * F->gsy);
    int64_t cx = fx > F->G - 1 ? F->G - 1 : (int64_t)fx;
    int64_t cy = fy > F->G - 1 ? F->G - 1 : (int64_t)fy;
    return cy * F->G + cx;
}

/* Number of polygons containing p; writes up to cap matching ids ascending. */
static int64_t point_matches(const orc_polys *P, const orc_filter *F, double x, double y,
                             int64_t *ids, int64_t cap)
{
    int64_t c = filter_cell(F, x, y);
    if (c < 0) return 0;
    int64_t n = 0;
    /* cell lists are built in ascending polygon order, so matches come out sorted */
    for (int64_t t = F->cell_off[c]; t < F->cell_off[c + 1]; ++t) {
        int64_t k = F->cell_items[t];
        if (!(F->xmin[k] <= x && x < F->xmax[k] && F->ymin[k] <= y && y < F->ymax[k])) continue;
        if (inside_poly(P, k, x, y)) {
            if (n < cap) ids[n] = k;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Public entry points (host arrays)                                   */
/* ------------------------------------------------------------------ */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* counts[k] = number of points inside polygon k */
void orc_join_count(int64_t n, const double *x, const double *y,
                    int64_t n_polys, const int64_t *poly_ring_off, const int64_t *ring_vtx_off,
                    const double *vx, const double *vy, uint64_t *counts)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    orc_filter F;
    filter_build(&P, &F);
    for (int64_t k = 0; k < n_polys; ++k) counts[k] = 0;
    #pragma omp parallel
    {
        uint64_t *local = calloc(n_polys ? n_polys : 1, sizeof(uint64_t));
        int64_t ids[64];
        #pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = filter_cell(&F, x[i], y[i]);
            if (c < 0) continue;
            for (int64_t t = F.cell_off[c]; t < F.cell_off[c + 1]; ++t) {
                int64_t k = F.cell_items[t];
                if (!(F.xmin[k] <= x[i] && x[i] < F.xmax[k] && F.ymin[k] <= y[i] && y[i] < F.ymax[k]))
                    continue;
                local[k] += (uint64_t)inside_poly(&P, k, x[i], y[i]);
            }
            (void)ids;
        }
        #pragma omp critical
        for (int64_t k = 0; k < n_polys; ++k) counts[k] += local[k];
        free(local);
    }
    filter_free(&F);
}

/* Per-point match count (how many polygons contain point i). */
void orc_point_nmatch(int64_t n, const double *x, const double *y,
                      int64_t n_polys, const int64_t *poly_ring_off, const int64_t *ring_vtx_off,
                      const double *vx, const double *vy, int32_t *nmatch)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    orc_filter F;
    filter_build(&P, &F);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i)
        nmatch[i] = (int32_t)point_matches(&P, &F, x[i], y[i], NULL, 0);
    filter_free(&F);
}

/* Join pairs ascending by (point, polygon).  Returns the total number of
 * pairs; writes the first min(total, cap) of them. */
int64_t orc_join_pairs(int64_t n, const double *x, const double *y,
                       int64_t n_polys, const int64_t *poly_ring_off, const int64_t *ring_vtx_off,
                       const double *vx, const double *vy,
                       int64_t cap, uint32_t *out_pt, uint32_t *out_poly)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    orc_filter F;
    filter_build(&P, &F);
    int32_t *nm = malloc(sizeof(int32_t) * (n ? n : 1));
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i)
        nm[i] = (int32_t)point_matches(&P, &F, x[i], y[i], NULL, 0);
    int64_t *off = malloc(sizeof(int64_t) * (n + 1));
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + nm[i];
    int64_t total = off[n];
    #pragma omp parallel
    {
        int64_t cap_local = n_polys > 0 ? n_polys : 1;
        int64_t *ids = malloc(sizeof(int64_t) * cap_local);
        #pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i) {
            if (nm[i] == 0 || off[i] >= cap) continue;
            int64_t m = point_matches(&P, &F, x[i], y[i], ids, cap_local);
            for (int64_t t = 0; t < m && off[i] + t < cap; ++t) {
                out_pt[off[i] + t] = (uint32_t)i;
                out_poly[off[i] + t] = (uint32_t)ids[t];
            }
        }
        free(ids);
    }
    free(off);
    free(nm);
    filter_free(&F);
    return total;
}

/* Selection against polygon `k` of the set: ascending point ids inside it.
 * Returns the total; writes the first min(total, cap). */
int64_t orc_select(int64_t n, const double *x, const double *y,
                   int64_t n_polys, const int64_t *poly_ring_off, const int64_t *ring_vtx_off,
                   const double *vx, const double *vy, int64_t k,
                   int64_t cap, uint32_t *out_ids)
{
    orc_polys P = { n_polys, poly_ring_off, ring_vtx_off, vx, vy };
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t r = ring_begin(&P, k); r < ring_end(&P, k); ++r)
        for (int64_t v = ring_vtx_off[r]; v < ring_vtx_off[r + 1]; ++v) {
            if (vx[v] < x0) x0 = vx[v];
            if (vx[v] > x1) x1 = vx[v];
            if (vy[v] < y0) y0 = vy[v];
            if (vy[v] > y1) y1 = vy[v];
        }
    uint8_t *hit = malloc(n ? n : 1);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i)
        hit[i] = (x0 <= x[i] && x[i] < x1 && y0 <= y[i] && y[i] < y1) ? (uint8_t)inside_poly(&P, k, x[i], y[i]) : 0;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (hit[i]) { if (m < cap) out_ids[m] = (uint32_t)i; ++m; }
    free(hit);
    return m;
}
