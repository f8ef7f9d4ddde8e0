// C ABI of the canvas engine: contexts, scratch memory, argument checks and
// the query entry points declared in include/spade.h.
#include "common.h"
#include "exact.h"

#include <algorithm>
#include <cstring>
#include <new>

namespace spade {

int set_error(spade_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(spade_ctx *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(ctx, e == hipErrorOutOfMemory ? SPADE_E_NOMEM : SPADE_E_HIP, m);
}

void free_buf(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Grow a device buffer to at least `bytes` (contents are not preserved).
int ensure(spade_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 1;
    if (b.cap >= bytes) return SPADE_OK;
    free_buf(b);
    size_t want = bytes + bytes / 4 + 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        e = hipMalloc(&b.p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        set_error(ctx, SPADE_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        return SPADE_E_NOMEM;
    }
    b.cap = want;
    return SPADE_OK;
}

// Grow a device buffer to at least `bytes`, keeping its contents (ordered
// on ctx's stream; the old buffer is freed once the stream has copied it).
int ensure_keep(spade_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (b.cap >= bytes) return SPADE_OK;
    DevBuf nb;
    if (ensure(ctx, nb, std::max(bytes, b.cap * 2))) return SPADE_E_NOMEM;
    if (b.p) {
        hipError_t e = hipMemcpyAsync(nb.p, b.p, b.cap, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            free_buf(nb);
            return hip_fail(ctx, e, "ensure_keep copy");
        }
    }
    free_buf(b);
    b = nb;
    return SPADE_OK;
}

int hip_fail_if(spade_ctx *ctx, hipError_t e)
{
    return e == hipSuccess ? SPADE_OK : hip_fail(ctx, e, "kernel launch");
}

void *ensure_pinned(spade_ctx *ctx, size_t bytes)
{
    if (ctx->pinned_cap >= bytes) return ctx->pinned;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
    size_t want = std::max<size_t>(bytes, 4096);
    if (hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->pinned = nullptr;
        return nullptr;
    }
    ctx->pinned_cap = want;
    return ctx->pinned;
}

static int check_ctx(spade_ctx *ctx)
{
    if (!ctx) return SPADE_E_INVALID;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    }
    return SPADE_OK;
}

static int check_points(spade_ctx *ctx, const spade_points *pts)
{
    if (!pts) return set_error(ctx, SPADE_E_INVALID, "points is NULL");
    if (pts->n < 0) return set_error(ctx, SPADE_E_INVALID, "negative point count");
    if (pts->n >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "point ids are uint32: n must be < 2^32 - 1");
    if (pts->n > 0 && (!pts->x || !pts->y)) return set_error(ctx, SPADE_E_INVALID, "point coordinate array is NULL");
    return SPADE_OK;
}

static int check_polys(spade_ctx *ctx, const spade_polys *p)
{
    if (!p) return set_error(ctx, SPADE_E_INVALID, "polygon set is NULL");
    if (p->n_polys < 0 || p->n_rings < 0) return set_error(ctx, SPADE_E_INVALID, "negative polygon or ring count");
    if (p->n_polys >= 0x7fffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "polygon ids must be < 2^31 - 1");
    if (!p->poly_ring_off && p->n_rings != p->n_polys)
        return set_error(ctx, SPADE_E_INVALID, "poly_ring_off is NULL but n_rings != n_polys");
    if (p->poly_ring_off == nullptr && p->n_polys > 0 && !p->ring_vtx_off)
        return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off is NULL");
    if (p->n_rings > 0 && (!p->ring_vtx_off || !p->vx || !p->vy))
        return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off / vx / vy is NULL");
    if (p->n_polys > 0 && !p->ring_vtx_off)
        return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off is NULL");
    if (p->n_polys > 0 && p->poly_ring_off == nullptr && p->n_rings == 0)
        return set_error(ctx, SPADE_E_INVALID, "polygons without rings");
    return SPADE_OK;
}

}  // namespace spade

using namespace spade;

extern "C" {

int spade_ctx_create(int device, void *stream, spade_ctx **out)
{
    if (!out) return SPADE_E_INVALID;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return SPADE_E_HIP;
    }
    spade_ctx *c = new (std::nothrow) spade_ctx();
    if (!c) return SPADE_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    // the device address of the no-allocation probe's scratch, once per
    // device (a failure is reported by that entry point)
    (void)noalloc_init(c);
    c->err.clear();
    *out = c;
    return SPADE_OK;
}

void spade_ctx_destroy(spade_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    jobs_shutdown(ctx);   // finishes the queued jobs first
    (void)hipDeviceSynchronize();
    for (auto &b : ctx->scratch) free_buf(b);
    if (ctx->plain) {
        free_buf(ctx->plain->cells);
        free_buf(ctx->plain->cands);
        free_buf(ctx->plain->ledges);
        free_buf(ctx->plain->pspan);
        free_buf(ctx->plain->edges);
        free_buf(ctx->plain->coarse);
        free_buf(ctx->plain->dcds);
        free_buf(ctx->plain->pid);
        free_buf(ctx->plain->qbox);
        drop_graph(ctx->plain);
        drop_batch_graph(ctx->plain);
        delete ctx->plain;
    }
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->pend) (void)hipHostFree(ctx->pend);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->join2) (void)hipEventDestroy(ctx->join2);
    if (ctx->evinfo) (void)hipEventDestroy(ctx->evinfo);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->side2) (void)hipStreamDestroy(ctx->side2);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    delete ctx;
}

int spade_ctx_set_stream(spade_ctx *ctx, void *stream)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    ctx->stream = (hipStream_t)stream;
    return SPADE_OK;
}

const char *spade_last_error(const spade_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

int spade_ctx_set_canvas_size(spade_ctx *ctx, int32_t width, int32_t height)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (width == 0 && height == 0) { ctx->canvas_w = ctx->canvas_h = 0; return SPADE_OK; }
    if (width < 1 || width > 8192 || height < 1 || height > 16384)
        return set_error(ctx, SPADE_E_INVALID, "canvas size must be 0x0 or within 1..8192 x 1..16384");
    ctx->canvas_w = width;
    ctx->canvas_h = height;
    return SPADE_OK;
}

int spade_ctx_set_graphs(spade_ctx *ctx, int on)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    ctx->graphs = on != 0;
    return SPADE_OK;
}

int spade_ctx_graph_stats(const spade_ctx *ctx, int64_t *captures, int64_t *replays)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (captures) *captures = ctx->graph_captures;
    if (replays) *replays = ctx->graph_replays;
    return SPADE_OK;
}

int spade_ctx_build_stats(const spade_ctx *ctx, int64_t *builds, int64_t *rebuilds)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (builds) *builds = ctx->builds;
    if (rebuilds) *rebuilds = ctx->rebuilds;
    return SPADE_OK;
}

int spade_ctx_batch_stats(const spade_ctx *ctx, int64_t *overlaps)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (overlaps) *overlaps = ctx->batch_overlaps;
    return SPADE_OK;
}

int spade_mem_info(spade_ctx *ctx, size_t *free_bytes, size_t *total_bytes, size_t *ctx_bytes)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    size_t fr = 0, tot = 0;
    SPADE_HIP(ctx, hipMemGetInfo(&fr, &tot));
    size_t held = 0;
    for (const auto &b : ctx->scratch) held += b.cap;
    if (ctx->plain) held += ctx->plain->bytes() + ctx->plain->edges.cap + ctx->plain->dcds.cap;
    held += jobs_bytes(ctx);
    if (free_bytes) *free_bytes = fr;
    if (total_bytes) *total_bytes = tot;
    if (ctx_bytes) *ctx_bytes = held;
    return SPADE_OK;
}

int spade_ctx_set_timing(spade_ctx *ctx, int on)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (on && !ctx->ev[0])
        for (auto &e : ctx->ev) SPADE_HIP(ctx, hipEventCreate(&e));
    ctx->timing = on != 0;
    ctx->timed_raster = false;
    return SPADE_OK;
}

int spade_ctx_last_timing(spade_ctx *ctx, float *raster_ms, float *probe_ms)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!ctx->timing) return set_error(ctx, SPADE_E_INVALID, "timing is not enabled");
    SPADE_HIP(ctx, hipEventSynchronize(ctx->ev[3]));
    float r = 0.f, p = 0.f;
    if (ctx->timed_raster) SPADE_HIP(ctx, hipEventElapsedTime(&r, ctx->ev[0], ctx->ev[1]));
    SPADE_HIP(ctx, hipEventElapsedTime(&p, ctx->ev[2], ctx->ev[3]));
    if (raster_ms) *raster_ms = r;
    if (probe_ms) *probe_ms = p;
    return SPADE_OK;
}

int spade_canvas_build(spade_ctx *ctx, const spade_polys *polys, spade_canvas **out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out) return set_error(ctx, SPADE_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((rc = check_polys(ctx, polys))) return rc;
    spade_canvas *cv = new (std::nothrow) spade_canvas();
    if (!cv) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    cv->device = ctx->device;
    rc = build_canvas(ctx, polys, cv);
    if (rc) {
        spade_canvas_destroy(cv);
        return rc;
    }
    *out = cv;
    return SPADE_OK;
}

void spade_canvas_destroy(spade_canvas *cv)
{
    if (!cv) return;
    (void)hipSetDevice(cv->device);
    free_buf(cv->cells);
    free_buf(cv->cands);
    free_buf(cv->ledges);
    free_buf(cv->pspan);
    free_buf(cv->edges);
    free_buf(cv->coarse);
    free_buf(cv->dcds);
    free_buf(cv->pid);
    free_buf(cv->qbox);
    drop_graph(cv);
    drop_batch_graph(cv);
    delete cv;
}

int spade_canvas_info(const spade_canvas *cv, int32_t *width, int32_t *height, int64_t *n_polys,
                      int64_t *n_boundary_pixels, int64_t *device_bytes)
{
    if (!cv) return SPADE_E_INVALID;
    int64_t m = 0;
    for (const auto &d : cv->descs) m += d.M;
    if (width) *width = cv->view.W;
    if (height) *height = cv->view.H;
    if (n_polys) *n_polys = m;
    if (n_boundary_pixels) *n_boundary_pixels = cv->n_boundary;
    if (device_bytes) *device_bytes = (int64_t)cv->bytes();
    return SPADE_OK;
}

int spade_layer_index(spade_ctx *ctx, const spade_polys *polys, int32_t res, int32_t *out_layer, int32_t *n_layers)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!n_layers) return set_error(ctx, SPADE_E_INVALID, "n_layers is NULL");
    *n_layers = 0;
    if ((rc = check_polys(ctx, polys))) return rc;
    if (res < 0 || res > 4096) return set_error(ctx, SPADE_E_INVALID, "res must be 0 (automatic) or 1..4096");
    if (polys->n_polys > 0 && !out_layer) return set_error(ctx, SPADE_E_INVALID, "out_layer is NULL");
    return layer_index(ctx, polys, res, out_layer, n_layers, nullptr, nullptr);
}

int spade_layered_build(spade_ctx *ctx, const spade_polys *polys, int32_t res, spade_canvas **out, int32_t *n_layers)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out) return set_error(ctx, SPADE_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((rc = check_polys(ctx, polys))) return rc;
    if (res < 0 || res > 4096) return set_error(ctx, SPADE_E_INVALID, "res must be 0 (automatic) or 1..4096");
    spade_canvas *cv = new (std::nothrow) spade_canvas();
    if (!cv) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    cv->device = ctx->device;
    int32_t L = 0;
    rc = layered_build(ctx, polys, res, cv, &L);
    if (rc) {
        spade_canvas_destroy(cv);
        return rc;
    }
    cv->n_layers = L;
    if (n_layers) *n_layers = L;
    *out = cv;
    return SPADE_OK;
}

int spade_canvas_join_count_async(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                                  uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!cv) return set_error(ctx, SPADE_E_INVALID, "canvas is NULL");
    if (cv->nc != 1) return set_error(ctx, SPADE_E_INVALID, "a batch canvas set is queried with the batch calls");
    if ((rc = check_points(ctx, pts))) return rc;
    if (cv->view.M > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    if (cv != ctx->plain) ctx->timed_raster = false;
    return probe_count(ctx, cv, pts, out_counts);
}

int spade_canvas_join_count_noalloc(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                                    uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!cv) return set_error(ctx, SPADE_E_INVALID, "canvas is NULL");
    if (cv->nc != 1) return set_error(ctx, SPADE_E_INVALID, "a batch canvas set is queried with the batch calls");
    if (cv->pending) return set_error(ctx, SPADE_E_INVALID, "the canvas's build has not completed");
    if ((rc = check_points(ctx, pts))) return rc;
    if (cv->view.M > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    if (cv != ctx->plain) ctx->timed_raster = false;
    return probe_count_noalloc(ctx, cv, pts, out_counts);
}

int spade_canvas_join_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                            uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = spade_canvas_join_count_async(ctx, cv, pts, out_counts);
    if (rc) return rc;
    SPADE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPADE_OK;
}

static int emit_common(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                       uint32_t *out_pt, uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!cv) return set_error(ctx, SPADE_E_INVALID, "canvas is NULL");
    if (cv->nc != 1) return set_error(ctx, SPADE_E_INVALID, "a batch canvas set is queried with the batch calls");
    if ((rc = check_points(ctx, pts))) return rc;
    if (!n_out) return set_error(ctx, SPADE_E_INVALID, "n_out is NULL");
    if (cap < 0) return set_error(ctx, SPADE_E_INVALID, "negative capacity");
    if (cap > 0 && !out_pt) return set_error(ctx, SPADE_E_INVALID, "output array is NULL");
    if (cv != ctx->plain) ctx->timed_raster = false;
    return probe_emit(ctx, cv, pts, out_pt, out_poly, cap, n_out);
}

int spade_canvas_select(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                        uint32_t *out_ids, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (cv && cv->nc == 1 && cv->view.M != 1) return set_error(ctx, SPADE_E_INVALID, "selection needs exactly one polygon");
    return emit_common(ctx, cv, pts, out_ids, nullptr, cap, n_out);
}

int spade_canvas_join_pairs(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                            uint32_t *out_pt, uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (cap > 0 && !out_poly) return set_error(ctx, SPADE_E_INVALID, "out_poly is NULL");
    return emit_common(ctx, cv, pts, out_pt, out_poly, cap, n_out);
}

// Plain calls: rasterise into the context's own canvas, then probe.
static int plain_build(spade_ctx *ctx, const spade_polys *polys, spade_canvas **cvo, bool defer)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_polys(ctx, polys))) return rc;
    if (!ctx->plain) {
        ctx->plain = new (std::nothrow) spade_canvas();
        if (!ctx->plain) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
        ctx->plain->device = ctx->device;
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
    rc = build_canvas(ctx, polys, ctx->plain, defer);
    if (rc) return rc;
    ctx->builds++;
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
    ctx->timed_raster = ctx->timing;
    *cvo = ctx->plain;
    return SPADE_OK;
}

// The probe is queued right behind the build, whose counters and flags are
// read at the probe's own synchronisation: a build that ran out of
// capacity is redone (with room to spare) and probed again; an invalid
// input fails the call whatever the probe returned.
extern "C++" template <typename F>
static int plain_query(spade_ctx *ctx, const spade_polys *polys, F &&probe)
{
    spade_canvas *cv = nullptr;
    int rc = plain_build(ctx, polys, &cv, true);
    if (rc) return rc;
    const int rp = probe(cv);
    if ((rc = build_flush(ctx, cv))) return rc;
    SPADE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int rf = build_finish(ctx, cv);
    if (rf == BUILD_AGAIN) {
        if ((rc = plain_build(ctx, polys, &cv, false))) return rc;
        ctx->rebuilds++;
        rc = probe(cv);
        // the probe may only have been queued (join-count): the plain calls
        // return complete results, so wait for it here as on the first path
        SPADE_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return rc;
    }
    return rf ? rf : rp;
}

int spade_select_disk(spade_ctx *ctx, const spade_points *pts, double cx, double cy, double r,
                      uint32_t *out_ids, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    return spade::select_disk(ctx, pts, cx, cy, r, out_ids, cap, n_out);
}

int spade_distance_join_pairs(spade_ctx *ctx, const spade_points *pts, const spade_disks *disks,
                              uint32_t *out_pt, uint32_t *out_disk, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    if (!n_out) return set_error(ctx, SPADE_E_INVALID, "n_out is NULL");
    if (cap < 0 || (cap > 0 && (!out_pt || !out_disk))) return set_error(ctx, SPADE_E_INVALID, "bad output buffers");
    ctx->timed_raster = false;
    return spade::distance_join(ctx, pts, disks, out_pt, out_disk, cap, n_out, nullptr);
}

int spade_distance_join_count(spade_ctx *ctx, const spade_points *pts, const spade_disks *disks,
                              uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    if (disks && disks->n > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    ctx->timed_raster = false;
    uint64_t dummy = 0;
    return spade::distance_join(ctx, pts, disks, nullptr, nullptr, 0, nullptr, out_counts ? out_counts : &dummy);
}

int spade_knn_select(spade_ctx *ctx, const spade_points *pts, double px, double py, int64_t k, uint32_t *out_ids,
                     int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    if (!n_out) return set_error(ctx, SPADE_E_INVALID, "n_out is NULL");
    ctx->timed_raster = false;
    return spade::knn_select(ctx, pts, px, py, k, out_ids, n_out);
}

int spade_select(spade_ctx *ctx, const spade_points *pts, const spade_polys *poly, uint32_t *out_ids,
                 int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    if (poly && poly->n_polys != 1) return set_error(ctx, SPADE_E_INVALID, "selection needs exactly one polygon");
    int rc = check_points(ctx, pts);
    if (rc) return rc;
    return plain_query(ctx, poly, [&](spade_canvas *cv) {
        return spade_canvas_select(ctx, cv, pts, out_ids, cap, n_out);
    });
}

int spade_join_count(spade_ctx *ctx, const spade_points *pts, const spade_polys *polys, uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_points(ctx, pts);
    if (rc) return rc;
    return plain_query(ctx, polys, [&](spade_canvas *cv) {
        return spade_canvas_join_count_async(ctx, cv, pts, out_counts);
    });
}

int spade_join_pairs(spade_ctx *ctx, const spade_points *pts, const spade_polys *polys, uint32_t *out_pt,
                     uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    int rc = check_points(ctx, pts);
    if (rc) return rc;
    return plain_query(ctx, polys, [&](spade_canvas *cv) {
        return spade_canvas_join_pairs(ctx, cv, pts, out_pt, out_poly, cap, n_out);
    });
}

int spade_select_near_lines(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines, double r,
                            uint32_t *out_ids, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    ctx->timed_raster = false;
    return spade::buffer_select(ctx, nullptr, pts, lines, r, false, out_ids, cap, n_out);
}

int spade_select_within_polygon(spade_ctx *ctx, const spade_points *pts, const spade_polys *poly, double r,
                                uint32_t *out_ids, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    if (poly && poly->n_polys != 1) return set_error(ctx, SPADE_E_INVALID, "the distance selection takes exactly one polygon");
    if (!(std::isfinite(r) && r >= 0.0)) return set_error(ctx, SPADE_E_INVALID, "the distance must be finite and >= 0");
    int rc = check_points(ctx, pts);
    if (rc) return rc;
    return plain_query(ctx, poly, [&](spade_canvas *cv) {
        return spade::buffer_select(ctx, cv, pts, poly, r, true, out_ids, cap, n_out);
    });
}

int spade_distance_join_lines_pairs(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines,
                                    const double *r, double r_all, uint32_t *out_pt, uint32_t *out_line, int64_t cap,
                                    int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (n_out) *n_out = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    ctx->timed_raster = false;
    return spade::buffer_join_lines(ctx, pts, lines, r, r_all, out_pt, out_line, cap, n_out, nullptr);
}

int spade_distance_join_lines_count(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines,
                                    const double *r, double r_all, uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    if (lines && lines->n_rings > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    ctx->timed_raster = false;
    uint64_t dummy = 0;
    return spade::buffer_join_lines(ctx, pts, lines, r, r_all, nullptr, nullptr, 0, nullptr,
                                    out_counts ? out_counts : &dummy);
}

int spade_stream_read(spade_ctx *ctx, const spade_points *pts, int shape, double *out_sum)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_points(ctx, pts))) return rc;
    if (!out_sum) return set_error(ctx, SPADE_E_INVALID, "out_sum is NULL");
    if (shape != 0 && shape != 1) return set_error(ctx, SPADE_E_INVALID, "shape must be 0 or 1");
    ctx->timed_raster = false;
    return spade::stream_read(ctx, pts, shape, out_sum);
}

// ---- exact predicate, exposed for isolated testing

__global__ void k_orient(int64_t n, const double *ax, const double *ay, const double *bx, const double *by,
                         const double *cx, const double *cy, int32_t *out)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth)
        out[i] = orient_sign(ax[i], ay[i], bx[i], by[i], cx[i], cy[i]);
}

int spade_orient_batch(spade_ctx *ctx, int64_t n, const double *ax, const double *ay, const double *bx,
                       const double *by, const double *cx, const double *cy, int32_t *out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (n < 0) return set_error(ctx, SPADE_E_INVALID, "negative count");
    if (n == 0) return SPADE_OK;
    if (!ax || !ay || !bx || !by || !cx || !cy || !out) return set_error(ctx, SPADE_E_INVALID, "NULL array");
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(k_orient, dim3(grid), dim3(256), 0, ctx->stream, n, ax, ay, bx, by, cx, cy, out);
    SPADE_HIP(ctx, hipGetLastError());
    SPADE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPADE_OK;
}

}  // extern "C"

// The context's canvas rasterised from `polys` (not deferred: complete and
// checked when this returns).
int spade::plain_canvas(spade_ctx *ctx, const spade_polys *polys, spade_canvas **cvo)
{
    return plain_build(ctx, polys, cvo, false);
}
