/*
 * spade.h -- C ABI of the canvas point-in-polygon engine for AMD MI355X (gfx950).
 *
 * The three queries follow the paper's statement of them (Sec. 5.2):
 *   - spatial selection with a polygonal constraint: the points of a dataset
 *     that intersect one polygon (for points, intersection = containment,
 *     Sec. 7 "Containment Queries");
 *   - the polygon-point join, evaluated as a collection of selections, one
 *     per polygon of the polygon dataset ("Spatial Joins", case (1));
 *   - the polygon-point aggregation: per-polygon point counts without
 *     materialising the join ("Spatial Aggregations", second plan).
 * Polygons are rasterised into a discrete canvas (Sec. 4.1/4.2: a pixel grid
 * of polygon ids with boundary pixels pointing into a boundary index,
 * Sec. 4.3); points in non-boundary pixels take the pixel's label, points in
 * boundary pixels get an exact crossing-number test.  Results are exact.
 *
 * Containment rule (the paper fixes none): a point p is inside polygon P iff
 * an odd number of P's edges (a,b) have (a.y > p.y) != (b.y > p.y) and meet
 * the horizontal line through p strictly to the right of p, the side test
 * being the exact sign of the orientation determinant.  Equivalently p is
 * classified as p + (eps, eps^2): boundary points belong to the polygon on
 * their +x side (above, for horizontal edges), so a tessellation counts every
 * point of its union exactly once.  Rings are implicitly closed; a polygon's
 * rings combine by even-odd parity (holes, multi-polygons); horizontal and
 * zero-length edges never count.
 *
 * Conventions for every call:
 *   - Array pointers are HIP DEVICE pointers on the context's device, unless
 *     stated otherwise; scalar out-parameters (n_out, sizes) are host pointers.
 *   - The caller owns every input and output buffer; the library never frees
 *     or retains them past the call.  The context owns its scratch memory.
 *   - Work is ordered on the context's stream.  The plain query calls return
 *     after their results are complete (one stream synchronisation).
 *   - Return value: SPADE_OK (0) or a negative SPADE_E_* code; the message
 *     of the last failure on a context is available from spade_last_error.
 *   - Coordinates are IEEE float64.  Exactness holds for finite coordinates
 *     whose pairwise products neither overflow nor underflow (|c| <= 2^500).
 *     Non-finite polygon vertices are rejected (SPADE_E_INVALID); points with
 *     a NaN or infinite coordinate lie in no polygon.
 *   - Point ids are 0-based indices into the point arrays (uint32: n < 2^32);
 *     polygon ids are 0-based positions in the polygon set (< 2^31 - 1).
 *   - Calls on one context are serialised by a lock the context holds
 *     (its job worker takes it too, per job); a call made from another
 *     thread waits.  Contexts are independent: use one per stream of work.
 */
#ifndef SPADE_H
#define SPADE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPADE_OK = 0,
    SPADE_E_INVALID = -1,      /* bad argument or malformed polygon set      */
    SPADE_E_CAPACITY = -2,     /* output buffer too small; *n_out = needed   */
    SPADE_E_NOMEM = -3,        /* device allocation failed                   */
    SPADE_E_HIP = -4,          /* HIP runtime error (message has the text)   */
    SPADE_E_UNSUPPORTED = -5,  /* valid request outside the library's limits */
    SPADE_E_TOO_LARGE = -6     /* n >= 2^32 points or n_polys >= 2^31 - 1    */
};

/* Points: structure of arrays, n entries each (device pointers). */
typedef struct {
    int64_t n;
    const double *x;
    const double *y;
} spade_points;

/* Polygon set in CSR form (device pointers).
 *   poly_ring_off [n_polys + 1]: rings of polygon k are
 *                  poly_ring_off[k] .. poly_ring_off[k+1]-1; NULL means ring k
 *                  is polygon k (n_rings == n_polys).
 *   ring_vtx_off  [n_rings + 1]: vertices of ring r are ring_vtx_off[r] ..
 *                  ring_vtx_off[r+1]-1, non-decreasing, ring_vtx_off[0] == 0.
 *   vx, vy        [ring_vtx_off[n_rings]]: vertex coordinates; a ring is
 *                  closed implicitly (do not repeat the first vertex; a
 *                  repeated one is a zero-length edge and is ignored).
 * n_rings is passed explicitly so that the offsets can be validated.
 * n_vertices: the vertex count ring_vtx_off[n_rings] when the caller knows it
 * (saves reading it back from the device); <= 0 means unknown.  A positive
 * value that differs from ring_vtx_off[n_rings] is SPADE_E_INVALID.
 * bbox: optional HOST array {x_min, x_max, y_min, y_max} of the vertices
 * (NULL: computed on the device and read back).  With it, the plain calls
 * and spade_canvas_build size the canvas without waiting for the device;
 * the device still validates the offsets and the box before any kernel
 * depends on them, and a box that does not contain every vertex, like any
 * other invalid input, fails the call with SPADE_E_INVALID.  Canvas sets
 * (the batch calls) ignore it. */
typedef struct {
    int64_t n_polys;
    int64_t n_rings;
    const int64_t *poly_ring_off;
    const int64_t *ring_vtx_off;
    const double *vx;
    const double *vy;
    int64_t n_vertices;
    const double *bbox;
} spade_polys;

typedef struct spade_ctx spade_ctx;
typedef struct spade_canvas spade_canvas;

/* Create a context on HIP device `device`, ordering its work on `stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context.  Returns SPADE_E_HIP if the device cannot be selected. */
int spade_ctx_create(int device, void *stream, spade_ctx **out);

/* Destroy a context and free its scratch memory (NULL is a no-op). */
void spade_ctx_destroy(spade_ctx *ctx);

/* Change the stream later calls are ordered on (NULL = null stream). */
int spade_ctx_set_stream(spade_ctx *ctx, void *stream);

/* Message for the last failing call on ctx ("" if none).  Valid until the
 * next call on ctx. */
const char *spade_last_error(const spade_ctx *ctx);

/* Canvas resolution used by later calls on ctx: width x height pixels over
 * the polygons' bounding box (the paper's canvas resolution, Sec. 4.2).
 * 0 x 0 selects it automatically.  Results never depend on it: it only
 * changes how many points need the exact boundary test.  Limits:
 * 1 <= width <= 8192, 1 <= height <= 16384. */
int spade_ctx_set_canvas_size(spade_ctx *ctx, int32_t width, int32_t height);

/* Graph replay of canvas builds (default on).  A canvas rebuilt with the
 * same launch parameters as its previous build (same sizes, same buffers:
 * typically the same polygon set again) replays the build's kernel launches
 * from a HIP graph captured on the second such build instead of launching
 * them one by one; every kernel still runs.  on == 0 launches eagerly. */
int spade_ctx_set_graphs(spade_ctx *ctx, int on);
/* Graphs captured and replays launched on ctx so far (either may be NULL). */
int spade_ctx_graph_stats(const spade_ctx *ctx, int64_t *captures, int64_t *replays);

/* Plain-call canvas builds on ctx so far, and how many of them were redone
 * because the first row pass ran out of record capacity (either may be
 * NULL).  A redone build is probed again before the call returns. */
int spade_ctx_build_stats(const spade_ctx *ctx, int64_t *builds, int64_t *rebuilds);

/* (table chunk, query) overlaps that the last batch selection or batch join
 * pairs on ctx evaluated (each one tests the chunk's points, 4096 but in the
 * table's last chunk, against one query's canvas). */
int spade_ctx_batch_stats(const spade_ctx *ctx, int64_t *overlaps);

/* Device memory facts for admission control (any pointer may be NULL):
 * free and total bytes of ctx's device (hipMemGetInfo) and the bytes of
 * device scratch that ctx itself holds for reuse (plain-call canvas, scratch
 * slots, job result buffers; tables and canvases are reported by their own
 * info calls).  A call while the context's worker runs a job waits for it. */
int spade_mem_info(spade_ctx *ctx, size_t *free_bytes, size_t *total_bytes, size_t *ctx_bytes);

/* Phase timing (tracing aid).  on != 0 makes later query calls record HIP
 * events on ctx's stream around the rasterisation and around the probe
 * kernel (for a batch selection: its count pass; for a batch join-count or
 * join pairs: the whole evaluation); spade_ctx_last_timing waits for the
 * last probe and returns both durations in milliseconds (raster_ms is 0 when
 * the last query used a prebuilt canvas).  Either out-pointer may be NULL. */
int spade_ctx_set_timing(spade_ctx *ctx, int on);
int spade_ctx_last_timing(spade_ctx *ctx, float *raster_ms, float *probe_ms);

/* Selection (Sec. 5.2, "Spatial Selection"): ids of the points inside the
 * single polygon of `poly` (n_polys must be 1), in ascending order.
 * out_ids [cap] device buffer.  *n_out (host) receives the number of
 * matching points.  If it exceeds cap, the first cap ids are written and
 * SPADE_E_CAPACITY is returned (the paper's two-step Map, Sec. 5.1). */
int spade_select(spade_ctx *ctx, const spade_points *pts, const spade_polys *poly,
                 uint32_t *out_ids, int64_t cap, int64_t *n_out);

/* Distance selection from a point (Sec. 4.2, "Canvases for Distance-Based
 * Queries", and Sec. 5.2, "Distance-Based Queries"): ids of the points whose
 * Euclidean distance to (cx, cy) is at most r (closed disk), in ascending
 * order, decided exactly on the FP64 inputs (exact whenever no square of a
 * coordinate difference, or r^2, overflows or underflows into subnormals).
 * cx, cy and r must be finite and r >= 0 (else SPADE_E_INVALID); points with
 * a non-finite coordinate are outside.  out_ids [cap] device buffer; *n_out
 * (host, may be NULL) receives the number of selected points.  If it exceeds
 * cap, the first cap ids are written and SPADE_E_CAPACITY is returned
 * (two-step Map, Sec. 5.1). */
int spade_select_disk(spade_ctx *ctx, const spade_points *pts, double cx, double cy, double r,
                      uint32_t *out_ids, int64_t cap, int64_t *n_out);

/* Distance selection from lines (Sec. 4.2, the rounded rectangle drawn
 * around each segment of a line; Sec. 5.2, "Distance-Based Queries"): ids of
 * the points whose Euclidean distance to some segment of `lines` is at most r
 * (closed), ascending.  Every ring of `lines` is an open polyline: segments
 * join consecutive vertices, with no closing segment, and a one-vertex ring is
 * a point (n_polys and poly_ring_off are ignored; ring_vtx_off, vx, vy as for
 * a polygon set, device pointers).  Decided exactly on the FP64 inputs (see
 * the segment predicate: exact whenever no product of coordinate differences
 * overflows or underflows into subnormals).  r must be finite and >= 0;
 * invalid ring offsets or a non-finite vertex are SPADE_E_INVALID; points
 * with a non-finite coordinate are never selected.  out_ids [cap] device
 * buffer; *n_out (host, may be NULL) receives the number of selected points;
 * beyond cap the first cap ids are written and SPADE_E_CAPACITY is returned
 * (two-step Map, Sec. 5.1).  The segments are binned into a grid over their
 * box widened by r, which the context keeps in scratch memory;
 * SPADE_E_TOO_LARGE when its cell lists would exceed 2^28 entries (r far
 * larger than the spacing of the segments). */
int spade_select_near_lines(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines, double r,
                            uint32_t *out_ids, int64_t cap, int64_t *n_out);

/* Distance selection from one polygon (Sec. 4.2: the polygon drawn together
 * with the rounded rectangles of its edges): ids of the points inside the
 * polygon (decided as spade_select decides) or within closed distance r of
 * one of its edges (rings closed), ascending, exactly.  `poly` must hold
 * exactly one polygon (SPADE_E_INVALID otherwise); arguments, errors and the
 * capacity protocol as spade_select_near_lines. */
int spade_select_within_polygon(spade_ctx *ctx, const spade_points *pts, const spade_polys *poly, double r,
                                uint32_t *out_ids, int64_t cap, int64_t *n_out);

/* Distance join of the points with a set of lines (Sec. 5.2, "Distance-Based
 * Queries", join types (1) and (2) with lines as the constraint dataset):
 * every ring j of `lines` is line j, an open polyline as for
 * spade_select_near_lines; r (device, may be NULL) holds one distance per
 * line (type 2), else r_all applies to every line (type 1).  The pairs
 * (point, line) of every point within closed distance r_j of line j, decided
 * exactly, ascending by point id then line id, into out_pt / out_line
 * (device, capacity cap); *n_out (host, may be NULL) receives the number of
 * pairs, and beyond cap the first cap pairs are written and SPADE_E_CAPACITY
 * is returned.  Distances must be finite and >= 0, vertices finite and the
 * offsets valid (SPADE_E_INVALID); fewer than 2^31 - 1 lines
 * (SPADE_E_TOO_LARGE); SPADE_E_TOO_LARGE also when the grid's cell lists
 * would exceed 2^26 entries (distances far larger than the spacing of the
 * segments). */
int spade_distance_join_lines_pairs(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines,
                                    const double *r, double r_all, uint32_t *out_pt, uint32_t *out_line, int64_t cap,
                                    int64_t *n_out);

/* Aggregation over the same join: out_counts [n_rings] (device, overwritten)
 * receives the number of points within each line's distance. */
int spade_distance_join_lines_count(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines,
                                    const double *r, double r_all, uint64_t *out_counts);

/* Disks (device pointers): centres (cx[j], cy[j]) and radii r[j] (type-2
 * distance join), or one radius r_all for every disk when r is NULL (type
 * 1).  Disk ids are 0-based positions (n < 2^31 - 1). */
typedef struct {
    int64_t n;
    const double *cx;
    const double *cy;
    const double *r;
    double r_all;
} spade_disks;

/* Distance join (Sec. 4.2, "Canvases for Distance-Based Queries"; Sec. 5.2,
 * "Distance-Based Queries", joins of types (1) and (2)): every pair (point
 * id, disk id) whose distance is at most the disk's radius (closed disks,
 * decided exactly on the FP64 inputs as spade_select_disk does), ascending
 * by point id then disk id, as two device arrays of capacity cap; *n_out
 * (host) receives the number of pairs, and beyond cap the first cap pairs
 * are written and SPADE_E_CAPACITY is returned.  The disks are rasterised
 * into a grid whose cells list the disks that reach them; every listed disk
 * gets the exact test.  Non-finite centres or radii, or negative radii, are
 * SPADE_E_INVALID; points with a non-finite coordinate match nothing. */
int spade_distance_join_pairs(spade_ctx *ctx, const spade_points *pts, const spade_disks *disks,
                              uint32_t *out_pt, uint32_t *out_disk, int64_t cap, int64_t *n_out);

/* Aggregation over the distance join: out_counts [n] (device) receives the
 * number of points within each disk. */
int spade_distance_join_count(spade_ctx *ctx, const spade_points *pts, const spade_disks *disks,
                              uint64_t *out_counts);

/* kNN selection (Sec. 5.2, "kNN Queries"): the k points nearest to (px, py)
 * by exact Euclidean distance, nearest first, equal distances by ascending
 * id.  out_ids [k] (device); *n_out (host) = min(k, number of points with
 * finite coordinates).  Follows the paper's plan: an aggregation over nested
 * circles around the point whose radii halve from one to the next (here the
 * powers of two 2^j, -511 <= j <= 511, so no pass over the points is needed
 * to find the paper's outer radius r_max; only when the k points reach
 * beyond 2^511 the circles r_max / 2^i, r_max the farthest corner of the
 * points' bounding box), a distance selection with the smallest circle
 * holding k points, and a sort of those candidates by distance (exact).
 * Exact while no squared distance overflows or falls into subnormals. */
int spade_knn_select(spade_ctx *ctx, const spade_points *pts, double px, double py, int64_t k,
                     uint32_t *out_ids, int64_t *n_out);

/* Aggregation (Sec. 5.2, "Spatial Aggregations", plan over point data):
 * out_counts [n_polys] device buffer, overwritten with the number of points
 * inside each polygon.  Overlapping polygons each count the point. */
int spade_join_count(spade_ctx *ctx, const spade_points *pts, const spade_polys *polys,
                     uint64_t *out_counts);

/* Polygon-point join (Sec. 5.2, "Spatial Joins", polygon x point): every
 * pair (point id, polygon id) with the point inside the polygon, ascending by
 * point id then polygon id, as two device arrays of capacity cap.  *n_out
 * (host) receives the number of pairs; SPADE_E_CAPACITY as for select. */
int spade_join_pairs(spade_ctx *ctx, const spade_points *pts, const spade_polys *polys,
                     uint32_t *out_pt, uint32_t *out_poly, int64_t cap, int64_t *n_out);

/* ---- Resident canvases (the constraint canvas kept on the device and
 * probed many times; canvases are built on the fly from vector data,
 * Sec. 4.2).  A canvas owns device memory until spade_canvas_destroy. */

/* Rasterise `polys` into a new canvas on ctx's device (the polygon arrays
 * may be freed after the call returns). */
int spade_canvas_build(spade_ctx *ctx, const spade_polys *polys, spade_canvas **out);

/* Free a canvas (NULL is a no-op).  Must not be in use by queued work. */
void spade_canvas_destroy(spade_canvas *cv);

/* Canvas facts: width, height, polygon count, boundary-pixel count and
 * device bytes held (any pointer may be NULL).  For a batch canvas set:
 * the first canvas's width and height, totals for the rest. */
int spade_canvas_info(const spade_canvas *cv, int32_t *width, int32_t *height,
                      int64_t *n_polys, int64_t *n_boundary_pixels, int64_t *device_bytes);

/* The three queries against a prebuilt canvas; same contracts as above.
 * spade_canvas_join_count_async only enqueues (no synchronisation); its
 * counts are complete when ctx's stream reaches that point.  A batch canvas
 * set (spade_batch_build) is refused here (SPADE_E_INVALID). */
int spade_canvas_select(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                        uint32_t *out_ids, int64_t cap, int64_t *n_out);
int spade_canvas_join_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                            uint64_t *out_counts);
int spade_canvas_join_count_async(spade_ctx *ctx, const spade_canvas *cv,
                                  const spade_points *pts, uint64_t *out_counts);
int spade_canvas_join_pairs(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                            uint32_t *out_pt, uint32_t *out_poly, int64_t cap, int64_t *n_out);

/* Join-count against a prebuilt canvas that allocates nothing, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same result as
 * spade_canvas_join_count_async (counts complete when ctx's stream reaches
 * that point; no synchronisation, no hipMalloc / hipFree, no allocating
 * library routine).  Its scratch (one u64 accumulator per polygon and a
 * counter) is a fixed device array of the library, one per GPU, held until
 * the process ends: at most 65536 polygons (SPADE_E_UNSUPPORTED beyond).
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other streams, other contexts, other host threads) race and must be
 * serialised by the caller.  The canvas must have been built beforehand
 * (spade_canvas_build). */
int spade_canvas_join_count_noalloc(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                                    uint64_t *out_counts);

/* ---- Resident point tables and query batches.  Many queries share one
 * pass over a resident, spatially clustered point table (the data stays in
 * HBM; each table chunk is read once for all queries whose bounding box
 * meets it), and the query polygons of a batch are rasterised as one canvas
 * set in the same kernel launches. */
typedef struct spade_table spade_table;

/* Copy the points into a new device-resident table clustered by a grid over
 * their bounding box (the input arrays may be freed after the call).  Point
 * ids in results stay the 0-based positions in the input arrays; points with
 * a non-finite coordinate are kept and lie in no polygon.  At most 2^31 - 1
 * points (SPADE_E_TOO_LARGE beyond). */
int spade_table_create(spade_ctx *ctx, const spade_points *pts, spade_table **out);

/* Free a table (NULL is a no-op).  Must not be in use by queued work. */
void spade_table_destroy(spade_table *t);

/* Table facts: points, grid side, chunks, device bytes (NULL-able). */
int spade_table_info(const spade_table *t, int64_t *n, int32_t *grid, int64_t *chunks,
                     int64_t *device_bytes);

/* Rasterise a batch of queries into one canvas set: query q consists of
 * polygons qbound[q] .. qbound[q+1]-1 of `polys` (qbound: host array of
 * nq + 1 non-decreasing offsets, qbound[0] == 0, qbound[nq] == n_polys).
 * Each query gets its own canvas sized for its polygons. */
int spade_batch_build(spade_ctx *ctx, const spade_polys *polys, int32_t nq, const int64_t *qbound,
                      spade_canvas **out);

/* Rasterise a new batch into an existing canvas set (from spade_batch_build
 * or spade_canvas_build), reusing its device memory where it is large
 * enough: a serving loop keeps one set per worker and avoids a device
 * allocation and free per batch.  Arguments as for spade_batch_build.  The
 * set must not be in use by queued work; after a failure it holds no valid
 * canvas (rebuild or destroy it). */
int spade_batch_rebuild(spade_ctx *ctx, const spade_polys *polys, int32_t nq, const int64_t *qbound,
                        spade_canvas *set);

/* Selection for every query of a batch (each query must hold exactly one
 * polygon), over a table: the ids of the table points inside, ascending
 * within each query, queries one after another in out_ids [cap] (device).
 * out_off [nq + 1] (host) receives each query's start; out_off[nq] is the
 * total.  If the total exceeds cap, the first cap ids of that order are
 * written and SPADE_E_CAPACITY is returned with out_off filled (cap == 0:
 * the count pass alone).  Evaluated with the paper's two-step Map
 * (Sec. 5.1): a count pass, then a write pass.  The count pass keeps each
 * (table chunk, query) overlap's match bits (512 bytes per overlap) so that
 * the write pass needs no second probe, unless they would exceed the byte
 * count in the environment variable SPADE_HIT_MASK_LIMIT (default 16 GiB;
 * 0: always probe twice). */
int spade_batch_select(spade_ctx *ctx, const spade_canvas *set, const spade_table *t,
                       uint32_t *out_ids, int64_t cap, int64_t *out_off);

/* Join-count for every query of a batch over a table: out_counts [n_polys
 * of the batch] (device) receives, for each polygon of the batch polygon
 * set, the number of table points inside it (for a layered set: indexed by
 * the caller's polygon ids). */
int spade_batch_join_count(spade_ctx *ctx, const spade_canvas *set, const spade_table *t,
                           uint64_t *out_counts);

/* Join pairs over a table for every polygon of a canvas set (a batch from
 * spade_batch_build, or a layered set from spade_layered_build): every pair
 * (point id, polygon id) with the table point inside the polygon, ascending
 * by point id then polygon id, as two device arrays of capacity cap (the
 * paper's polygon-point join, Sec. 5.2 "Spatial Joins" case (1)).  Point ids
 * are the table's input positions; polygon ids are positions in the polygon
 * set the canvas set was built from (for a batch, the concatenated set).
 * *n_out (host) receives the number of pairs; beyond cap the first cap
 * pairs are written and SPADE_E_CAPACITY is returned. */
int spade_batch_join_pairs(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, uint32_t *out_pt,
                           uint32_t *out_poly, int64_t cap, int64_t *n_out);

/* ---- Layer index (Sec. 4.3 "Layer Index", created as in Sec. 5.5).  The
 * polygons are split into layers such that no two polygons of a layer cover
 * the same pixel centre of a res x res grid (aspect kept; res 0 = 1024, at
 * most 4096) over the set's bounding box.  Built by the paper's iteration:
 * each pixel keeps the highest id of the polygons not yet placed (multiway
 * blend), every such polygon whose pixels all kept its own id joins the
 * next layer (blend + mask), the others wait.  Polygons covering no pixel
 * centre join layer 0.  A tessellation is one layer.  Layers change only how
 * fast a join runs, never its result. */

/* out_layer [n_polys] (device int32) receives each polygon's layer, 0-based;
 * *n_layers (host) the number of layers. */
int spade_layer_index(spade_ctx *ctx, const spade_polys *polys, int32_t res, int32_t *out_layer,
                      int32_t *n_layers);

/* Rasterise each layer of `polys` into its own canvas of a new canvas set
 * (Sec. 5.2, "Spatial Joins" case (1): one selection per layer).  The set
 * is queried with spade_batch_join_count and spade_batch_join_pairs over a
 * table, which report the caller's polygon ids.  *n_layers may be NULL.
 * The polygon arrays may be freed after the call returns. */
int spade_layered_build(spade_ctx *ctx, const spade_polys *polys, int32_t res, spade_canvas **out,
                        int32_t *n_layers);

/* ---- Asynchronous batch jobs.  spade_batch_submit hands a batch to ctx's
 * worker thread and returns at once; the worker rasterises the batch into
 * the caller's canvas set (as spade_batch_rebuild) and evaluates it over a
 * table (selection, join-count or join pairs) on ctx's stream.  Jobs of one
 * context run in submission order; jobs of different contexts (each with
 * its own stream) overlap on the device.  Another call on a context whose
 * worker is running a job waits until that job is done (calls queued
 * behind it keep their order only per thread).  A job's canvas set, table
 * and polygon arrays must stay alive until the job is done. */
enum { SPADE_JOB_SELECT = 1, SPADE_JOB_COUNT = 2, SPADE_JOB_PAIRS = 3 };
typedef struct spade_job spade_job;
typedef struct {
    int status;          /* SPADE_OK or the job's error code */
    int64_t n_out;       /* ids (SELECT), polygons (COUNT) or pairs (PAIRS) */
    void *out0;          /* device: u32 ids / u64 counts / u32 pair point ids */
    void *out1;          /* device: u32 pair polygon ids (PAIRS), else NULL */
    const int64_t *off;  /* host: nq + 1 query offsets into out0 (SELECT), else NULL */
    int64_t n_off;
} spade_job_result;

/* polys: device CSR arrays that must stay valid until the job is done;
 * qbound: host offsets as for spade_batch_build (copied); set: a canvas set
 * from spade_batch_build (rebuilt in place; not the context's own canvas);
 * kind: SPADE_JOB_*.  *out receives the job handle.  With polys NULL the job
 * queries the set as it was last built (nq and qbound are then ignored): a
 * caller that keeps the set of a polygon set it sees again skips its
 * rasterisation. */
int spade_batch_submit(spade_ctx *ctx, spade_canvas *set, const spade_polys *polys, int32_t nq,
                       const int64_t *qbound, const spade_table *t, int kind, spade_job **out);

/* Blocks until the job is done and describes its results, which live in a
 * device buffer the context lends the job until spade_job_free (buffers
 * come back to a pool per job kind and are reused, so a loop that frees
 * each job before its next one of the kind allocates nothing per job).
 * Returns the job's status. */
int spade_batch_wait(spade_job *job, spade_job_result *res);

/* 1 if the job is done, 0 if not (never blocks). */
int spade_job_query(const spade_job *job);

/* Frees the handle (waits for the job first) and returns its result buffer
 * to the context.  Free every job of a context before destroying it. */
void spade_job_free(spade_job *job);

/* ---- Out-of-core point tables (Sec. 5.3, "Out-of-Core Queries").  The
 * points stay in host memory, clustered by a grid index (G x G cells over
 * their bounding box, each cell a contiguous block with its exact bounding
 * box).  A query filters the cells by its polygons' bounding box, then
 * streams the blocks that pass to the device in chunks through two staging
 * buffers (copies of the next chunk overlap the probe of the current one)
 * and probes each chunk with the in-memory kernels.  Results are those of
 * the in-memory calls on the original arrays. */
typedef struct spade_host_table spade_host_table;

/* x, y: HOST arrays of n points (may be freed after the call; the table
 * keeps a clustered copy in pinned host memory, 20 bytes per point, plus two
 * device staging buffers of 2^24 points).  Point ids in results are the
 * input positions (n < 2^32 - 1). */
int spade_host_table_create(spade_ctx *ctx, const double *x, const double *y, int64_t n,
                            spade_host_table **out);
void spade_host_table_destroy(spade_host_table *t);
/* Points, grid side, pinned host bytes (any pointer may be NULL). */
int spade_host_table_info(const spade_host_table *t, int64_t *n, int32_t *grid, int64_t *host_bytes);

/* Join-count of the table's points with `polys` (device CSR): out_counts
 * [n_polys] (device), as spade_join_count.  *streamed (host, may be NULL)
 * receives the number of points the cell filter let through (the points
 * copied to the device). */
int spade_host_join_count(spade_ctx *ctx, spade_host_table *t, const spade_polys *polys, uint64_t *out_counts,
                          int64_t *streamed);

/* Selection of the table's points with one polygon: ascending ids into
 * out_ids [cap] (device), capacity protocol as spade_select. */
int spade_host_select(spade_ctx *ctx, spade_host_table *t, const spade_polys *poly, uint32_t *out_ids,
                      int64_t cap, int64_t *n_out, int64_t *streamed);

/* Canvas sizing for later builds when no fixed size is set: about `ppv`
 * pixels per polygon vertex, between 64 x 64 and 4096 x 4096 pixels per
 * canvas (default 256).  The autotuner sets this. */
int spade_ctx_set_pixels_per_vertex(spade_ctx *ctx, double ppv);

/* Measurement aid: reads both coordinates of every point once and adds
 * their sum to *out_sum (device double, not cleared), with the count
 * probe's launch shape (shape 0: one 1024-thread workgroup per compute
 * unit, 8 points per thread in flight) or with 256-thread workgroups, eight
 * per compute unit (shape 1).  Timed by the phase timer as a probe. */
int spade_stream_read(spade_ctx *ctx, const spade_points *pts, int shape, double *out_sum);

/* Device-side exact predicate, exposed for testing the arithmetic in
 * isolation: for n triples (a, b, c) stored as 6 device arrays, writes
 * sign((b-a) x (c-a)) in {-1, 0, 1} to out[n] (device int32). */
int spade_orient_batch(spade_ctx *ctx, int64_t n, const double *ax, const double *ay,
                       const double *bx, const double *by, const double *cx,
                       const double *cy, int32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* SPADE_H */
