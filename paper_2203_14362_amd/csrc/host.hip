// Out-of-core point tables (Sec. 5.3, "Out-of-Core Queries"): points that
// stay in host memory and stream to the device per query.
//
// The table is the paper's clustered grid index: the points are sorted by
// the cell of a G x G grid over their bounding box, each cell a contiguous
// block with its exact bounding box (the paper keeps a convex hull per cell;
// a box is the same filter, a little coarser).  A query first filters the
// cells against the query's bounding box (the index-filtering step), then
// streams the blocks of the cells that pass to the device in chunks, through
// two device buffers: while the probe runs on one chunk, the copy engine
// fills the other (the I/O pipelining the paper names as future work).  Each
// chunk is probed with the in-memory kernels (the refinement step).  The
// blocks live in pinned host memory so the copies run at the link's rate.
#include "common.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

struct spade_host_table {
    int device = 0;
    int64_t n = 0, nfin = 0;
    int G = 1;
    double X0 = 0, Y0 = 0, sx = 0, sy = 0;
    double *x = nullptr, *y = nullptr;      // pinned host, clustered (finite points first)
    uint32_t *ids = nullptr;                // pinned host: input position of each point
    std::vector<int64_t> cell_off;          // [G*G + 1]
    std::vector<double> cell_bb;            // 4 per cell: x0, y0, x1, y1 (closed, of its points)
    spade::DevBuf dx[2], dy[2], did[2];     // device staging buffers
    hipStream_t copy = nullptr;
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    int64_t stage = 0;                      // points per staging buffer
    size_t host_bytes() const { return (size_t)n * 20; }
};

namespace spade {

constexpr int64_t HT_STAGE = (int64_t)1 << 24;   // points per streamed chunk

static int ht_threads()
{
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 32u));
}

template <typename F>
static void parallel_for(int64_t n, F &&f)
{
    const int T = ht_threads();
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            const int64_t a = n * t / T, b = n * (t + 1) / T;
            f(t, a, b);
        });
    for (auto &x : th) x.join();
}

int host_table_create(spade_ctx *ctx, const double *x, const double *y, int64_t n, spade_host_table *t)
{
    t->device = ctx->device;
    t->n = n;
    const int T = ht_threads();
    // bounding box of the finite points
    std::vector<double> bb((size_t)T * 4);
    parallel_for(n, [&](int th, int64_t a, int64_t b) {
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int64_t i = a; i < b; ++i) {
            const double xi = x[i], yi = y[i];
            if (!std::isfinite(xi) || !std::isfinite(yi)) continue;
            x0 = std::min(x0, xi); x1 = std::max(x1, xi);
            y0 = std::min(y0, yi); y1 = std::max(y1, yi);
        }
        bb[4 * th] = x0; bb[4 * th + 1] = x1; bb[4 * th + 2] = y0; bb[4 * th + 3] = y1;
    });
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int th = 0; th < T; ++th) {
        x0 = std::min(x0, bb[4 * th]); x1 = std::max(x1, bb[4 * th + 1]);
        y0 = std::min(y0, bb[4 * th + 2]); y1 = std::max(y1, bb[4 * th + 3]);
    }
    if (!(x0 <= x1)) { x0 = 0; x1 = 1; y0 = 0; y1 = 1; }
    // cells of about 16k points on average, at most 1024 per side
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (int64_t)std::sqrt((double)n / 16384.0)));
    t->G = G;
    t->X0 = x0;
    t->Y0 = y0;
    t->sx = x1 > x0 ? G / (x1 - x0) : 0.0;
    t->sy = y1 > y0 ? G / (y1 - y0) : 0.0;
    const int64_t ncell = (int64_t)G * G;   // cell ncell holds the non-finite points
    auto cell_of = [&](double xi, double yi) -> int64_t {
        if (!std::isfinite(xi) || !std::isfinite(yi)) return ncell;
        const int cx = (int)std::min<double>(G - 1, std::max(0.0, std::floor((xi - t->X0) * t->sx)));
        const int cy = (int)std::min<double>(G - 1, std::max(0.0, std::floor((yi - t->Y0) * t->sy)));
        return (int64_t)cy * G + cx;
    };
    // counting sort by cell: per-thread histograms, prefix, scatter
    std::vector<std::vector<int64_t>> hist((size_t)T, std::vector<int64_t>((size_t)ncell + 1, 0));
    parallel_for(n, [&](int th, int64_t a, int64_t b) {
        auto &h = hist[(size_t)th];
        for (int64_t i = a; i < b; ++i) h[(size_t)cell_of(x[i], y[i])]++;
    });
    t->cell_off.assign((size_t)ncell + 2, 0);
    {
        int64_t run = 0;
        for (int64_t c = 0; c <= ncell; ++c) {
            t->cell_off[(size_t)c] = run;
            for (int th = 0; th < T; ++th) {
                const int64_t v = hist[(size_t)th][(size_t)c];
                hist[(size_t)th][(size_t)c] = run;
                run += v;
            }
        }
        t->cell_off[(size_t)ncell + 1] = run;
    }
    t->nfin = t->cell_off[(size_t)ncell];
    if (hipHostMalloc((void **)&t->x, sizeof(double) * (size_t)std::max<int64_t>(n, 1), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&t->y, sizeof(double) * (size_t)std::max<int64_t>(n, 1), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&t->ids, sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, SPADE_E_NOMEM, "pinned host allocation of the table failed");
    }
    parallel_for(n, [&](int th, int64_t a, int64_t b) {
        auto &h = hist[(size_t)th];
        for (int64_t i = a; i < b; ++i) {
            const int64_t at = h[(size_t)cell_of(x[i], y[i])]++;
            t->x[at] = x[i];
            t->y[at] = y[i];
            t->ids[at] = (uint32_t)i;
        }
    });
    // exact box of every cell's points
    t->cell_bb.assign((size_t)ncell * 4, 0.0);
    parallel_for(ncell, [&](int, int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            double bx0 = INFINITY, bx1 = -INFINITY, by0 = INFINITY, by1 = -INFINITY;
            for (int64_t i = t->cell_off[(size_t)c]; i < t->cell_off[(size_t)c + 1]; ++i) {
                bx0 = std::min(bx0, t->x[i]); bx1 = std::max(bx1, t->x[i]);
                by0 = std::min(by0, t->y[i]); by1 = std::max(by1, t->y[i]);
            }
            double *o = &t->cell_bb[(size_t)c * 4];
            o[0] = bx0; o[1] = by0; o[2] = bx1; o[3] = by1;
        }
    });
    // staging buffers, copy stream, events
    t->stage = std::min<int64_t>(HT_STAGE, std::max<int64_t>(n, 1));
    for (int b = 0; b < 2; ++b)
        if (ensure(ctx, t->dx[b], 8 * (size_t)t->stage) || ensure(ctx, t->dy[b], 8 * (size_t)t->stage) ||
            ensure(ctx, t->did[b], 4 * (size_t)t->stage))
            return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipStreamCreateWithFlags(&t->copy, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        SPADE_HIP(ctx, hipEventCreateWithFlags(&t->ready[b], hipEventDisableTiming));
        SPADE_HIP(ctx, hipEventCreateWithFlags(&t->freed[b], hipEventDisableTiming));
    }
    return SPADE_OK;
}

void host_table_free(spade_host_table *t)
{
    if (t->copy) (void)hipStreamSynchronize(t->copy);
    for (int b = 0; b < 2; ++b) {
        free_buf(t->dx[b]);
        free_buf(t->dy[b]);
        free_buf(t->did[b]);
        if (t->ready[b]) (void)hipEventDestroy(t->ready[b]);
        if (t->freed[b]) (void)hipEventDestroy(t->freed[b]);
    }
    if (t->copy) (void)hipStreamDestroy(t->copy);
    if (t->x) (void)hipHostFree(t->x);
    if (t->y) (void)hipHostFree(t->y);
    if (t->ids) (void)hipHostFree(t->ids);
}

// Ranges of clustered points in the cells whose box meets the query's
// half-open box [bx0, bx1) x [by0, by1), merged when adjacent.
static std::vector<std::pair<int64_t, int64_t>> filter_cells(const spade_host_table *t, const CanvasView &v)
{
    std::vector<std::pair<int64_t, int64_t>> out;
    const int64_t ncell = (int64_t)t->G * t->G;
    for (int64_t c = 0; c < ncell; ++c) {
        const int64_t a = t->cell_off[(size_t)c], b = t->cell_off[(size_t)c + 1];
        if (a == b) continue;
        const double *o = &t->cell_bb[(size_t)c * 4];
        if (!(o[2] >= v.bx0 && o[0] < v.bx1 && o[3] >= v.by0 && o[1] < v.by1)) continue;
        if (!out.empty() && out.back().second == a) out.back().second = b;
        else out.push_back({a, b});
    }
    return out;
}

__global__ void k_add_counts(int64_t M, const unsigned long long *part, unsigned long long *out)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M; k += (int64_t)gridDim.x * blockDim.x)
        out[k] += part[k];
}

__global__ void k_zero_u64(int64_t M, unsigned long long *out)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = 0ull;
}

__global__ void k_map_ids(int64_t m, const uint32_t *local, const uint32_t *ids, uint32_t *out)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = ids[local[k]];
}

static int ht_grid(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

// Streams the point ranges in chunks of at most t->stage points through the
// two staging buffers; probe(x, y, ids, m, chunk) runs on ctx's stream.
template <typename Probe>
static int stream_chunks(spade_ctx *ctx, spade_host_table *t, const std::vector<std::pair<int64_t, int64_t>> &ranges,
                         Probe &&probe, int64_t *streamed)
{
    hipStream_t st = ctx->stream;
    struct Piece { int64_t a, m; };
    std::vector<std::vector<Piece>> chunks;
    {
        std::vector<Piece> cur;
        int64_t fill = 0;
        for (auto r : ranges) {
            int64_t a = r.first;
            while (a < r.second) {
                const int64_t take = std::min(r.second - a, t->stage - fill);
                cur.push_back({a, take});
                fill += take;
                a += take;
                if (fill == t->stage) {
                    chunks.push_back(cur);
                    cur.clear();
                    fill = 0;
                }
            }
        }
        if (!cur.empty()) chunks.push_back(cur);
    }
    int64_t total = 0;
    // the copy stream may reuse a buffer once the compute stream has passed it
    for (int b = 0; b < 2; ++b) SPADE_HIP(ctx, hipEventRecord(t->freed[b], st));
    std::vector<int64_t> filled(chunks.size(), 0);
    auto enqueue_copy = [&](size_t k) -> int {
        const int b = (int)(k & 1);
        SPADE_HIP(ctx, hipStreamWaitEvent(t->copy, t->freed[b], 0));
        int64_t off = 0;
        for (const Piece &p : chunks[k]) {
            SPADE_HIP(ctx, hipMemcpyAsync((double *)t->dx[b].p + off, t->x + p.a, 8 * (size_t)p.m,
                                          hipMemcpyHostToDevice, t->copy));
            SPADE_HIP(ctx, hipMemcpyAsync((double *)t->dy[b].p + off, t->y + p.a, 8 * (size_t)p.m,
                                          hipMemcpyHostToDevice, t->copy));
            SPADE_HIP(ctx, hipMemcpyAsync((uint32_t *)t->did[b].p + off, t->ids + p.a, 4 * (size_t)p.m,
                                          hipMemcpyHostToDevice, t->copy));
            off += p.m;
        }
        SPADE_HIP(ctx, hipEventRecord(t->ready[b], t->copy));
        filled[k] = off;
        return SPADE_OK;
    };
    if (!chunks.empty()) {
        int rc = enqueue_copy(0);
        if (rc) return rc;
    }
    for (size_t k = 0; k < chunks.size(); ++k) {
        const int b = (int)(k & 1);
        // the next chunk's copies are queued before this chunk's probe, which
        // may wait on the host, so that they overlap it
        if (k + 1 < chunks.size()) {
            int rc = enqueue_copy(k + 1);
            if (rc) return rc;
        }
        SPADE_HIP(ctx, hipStreamWaitEvent(st, t->ready[b], 0));
        int rc = probe((const double *)t->dx[b].p, (const double *)t->dy[b].p, (const uint32_t *)t->did[b].p,
                       filled[k], (int64_t)k);
        if (rc) {
            (void)hipStreamSynchronize(t->copy);
            return rc;
        }
        SPADE_HIP(ctx, hipEventRecord(t->freed[b], st));
        total += filled[k];
    }
    if (streamed) *streamed = total;
    return SPADE_OK;
}

int host_join_count(spade_ctx *ctx, spade_host_table *t, const spade_canvas *cv, uint64_t *out_counts,
                    int64_t *streamed)
{
    hipStream_t st = ctx->stream;
    const int64_t M = cv->view.M;
    if (M == 0) return SPADE_OK;
    hipLaunchKernelGGL(k_zero_u64, dim3(ht_grid(M)), dim3(256), 0, st, M, (unsigned long long *)out_counts);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &bp = ctx->scratch[S_MISC];
    if (ensure(ctx, bp, 8 * (size_t)M)) return SPADE_E_NOMEM;
    const auto ranges = filter_cells(t, cv->view);
    return stream_chunks(ctx, t, ranges, [&](const double *X, const double *Y, const uint32_t *, int64_t m, int64_t) {
        spade_points p{m, X, Y};
        int rc = probe_count(ctx, cv, &p, (uint64_t *)bp.p);
        if (rc) return rc;
        hipLaunchKernelGGL(k_add_counts, dim3(ht_grid(M)), dim3(256), 0, st, M, (const unsigned long long *)bp.p,
                           (unsigned long long *)out_counts);
        return hip_fail_if(ctx, hipGetLastError());
    }, streamed);
}

int host_select(spade_ctx *ctx, spade_host_table *t, const spade_canvas *cv, uint32_t *out_ids, int64_t cap,
                int64_t *n_out, int64_t *streamed)
{
    hipStream_t st = ctx->stream;
    *n_out = 0;
    DevBuf &acc = ctx->scratch[S_ENTC], &loc = ctx->scratch[S_ENTF];
    int64_t have = 0;
    const auto ranges = filter_cells(t, cv->view);
    int rc = stream_chunks(ctx, t, ranges, [&](const double *X, const double *Y, const uint32_t *ids, int64_t m,
                                                int64_t) {
        spade_points p{m, X, Y};
        if (ensure_keep(ctx, loc, 4 * (size_t)std::max<int64_t>(m, 1))) return (int)SPADE_E_NOMEM;
        int64_t got = 0;
        int r = probe_emit(ctx, cv, &p, (uint32_t *)loc.p, nullptr, m, &got);   // synchronises
        if (r) return r;
        if (got == 0) return (int)SPADE_OK;
        if (ensure_keep(ctx, acc, 4 * (size_t)(have + got))) return (int)SPADE_E_NOMEM;
        hipLaunchKernelGGL(k_map_ids, dim3(ht_grid(got)), dim3(256), 0, st, got, (const uint32_t *)loc.p, ids,
                           (uint32_t *)acc.p + have);
        have += got;
        return hip_fail_if(ctx, hipGetLastError());
    }, streamed);
    if (rc) return rc;
    *n_out = have;
    if (have == 0) return SPADE_OK;
    // ascending input positions: one radix sort of the selected ids
    DevBuf &tmp = ctx->scratch[S_KEYS2], &cub = ctx->scratch[S_CUBTMP];
    if (ensure(ctx, tmp, 4 * (size_t)have)) return SPADE_E_NOMEM;
    int bits = 1;
    while (bits < 32 && ((uint64_t)(t->n - 1) >> bits) != 0) ++bits;
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(nullptr, tb, (const uint32_t *)acc.p, (uint32_t *)tmp.p,
                                                     (int)have, 0, bits, st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(cub.p, tb, (const uint32_t *)acc.p, (uint32_t *)tmp.p,
                                                     (int)have, 0, bits, st));
    const int64_t nw = std::min(have, cap);
    if (nw > 0) SPADE_HIP(ctx, hipMemcpyAsync(out_ids, tmp.p, 4 * (size_t)nw, hipMemcpyDeviceToDevice, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (have > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // namespace spade

using namespace spade;

extern "C" {

int spade_host_table_create(spade_ctx *ctx, const double *x, const double *y, int64_t n, spade_host_table **out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !out) return SPADE_E_INVALID;
    *out = nullptr;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    if (n < 0 || (n > 0 && (!x || !y))) return set_error(ctx, SPADE_E_INVALID, "invalid host point arrays");
    if (n >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "point ids are uint32: n must be < 2^32 - 1");
    spade_host_table *t = new (std::nothrow) spade_host_table();
    if (!t) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    const int rc = host_table_create(ctx, x, y, n, t);
    if (rc) {
        host_table_free(t);
        delete t;
        return rc;
    }
    *out = t;
    return SPADE_OK;
}

void spade_host_table_destroy(spade_host_table *t)
{
    if (!t) return;
    (void)hipSetDevice(t->device);
    host_table_free(t);
    delete t;
}

int spade_host_table_info(const spade_host_table *t, int64_t *n, int32_t *grid, int64_t *host_bytes)
{
    if (!t) return SPADE_E_INVALID;
    if (n) *n = t->n;
    if (grid) *grid = t->G;
    if (host_bytes) *host_bytes = (int64_t)t->host_bytes();
    return SPADE_OK;
}

int spade_host_join_count(spade_ctx *ctx, spade_host_table *t, const spade_polys *polys, uint64_t *out_counts,
                          int64_t *streamed)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (streamed) *streamed = 0;
    if (!t) return set_error(ctx, SPADE_E_INVALID, "table is NULL");
    spade_canvas *cv = nullptr;
    int rc = plain_canvas(ctx, polys, &cv);
    if (rc) return rc;
    if (cv->view.M > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    if ((rc = host_join_count(ctx, t, cv, out_counts, streamed))) return rc;
    SPADE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPADE_OK;
}

int spade_host_select(spade_ctx *ctx, spade_host_table *t, const spade_polys *poly, uint32_t *out_ids, int64_t cap,
                      int64_t *n_out, int64_t *streamed)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (streamed) *streamed = 0;
    if (n_out) *n_out = 0;
    if (!t || !n_out) return set_error(ctx, SPADE_E_INVALID, "table or n_out is NULL");
    if (poly && poly->n_polys != 1) return set_error(ctx, SPADE_E_INVALID, "selection needs exactly one polygon");
    if (cap < 0 || (cap > 0 && !out_ids)) return set_error(ctx, SPADE_E_INVALID, "bad output buffer");
    spade_canvas *cv = nullptr;
    int rc = plain_canvas(ctx, poly, &cv);
    if (rc) return rc;
    return host_select(ctx, t, cv, out_ids, cap, n_out, streamed);
}

}  // extern "C"
