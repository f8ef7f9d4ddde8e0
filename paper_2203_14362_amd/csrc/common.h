// Internal declarations of the canvas engine (device structs, context,
// scratch management).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spade.h"

namespace spade {

// Canvas word (one uint32 per pixel):
//   0                  : the pixel lies in no polygon
//   1 .. 2^31-1        : every point of the pixel lies in polygon (word - 1)
//                        and in no other
//   BFLAG | r          : boundary pixel; its candidate records start at index
//                        r of the record array and run up to a record flagged
//                        LAST.
// This is the paper's discrete canvas (Sec. 4.1: an object id plus a pointer
// v_b into the boundary index) restricted to polygons.
constexpr uint32_t BFLAG = 0x80000000u;

// Candidate record of a boundary pixel for one polygon (the boundary index
// entry, Sec. 4.3).  A point p of the pixel is inside polygon `poly` iff
//     S  XOR  (XOR over partial-right edges e of straddle(e, p.y))
//        XOR  (XOR over local edges e of cross(e, p))
// where local edges touch the (margin-dilated) pixel, partial-right edges lie
// entirely to its right but end inside the pixel row, and S is the parity of
// the edges entirely to the right that span the whole row.  Local edges are
// stored with their coordinates: the first inside the record, the others
// contiguous from eoff; partial-right edges only need their y-range
// (contiguous from poff, the first repeated inside the record).  A record of
// one local edge and at most one partial-right range is a single 64-byte
// read.
struct Edge {
    double xlo, ylo, xhi, yhi;
};
struct Cand {
    uint32_t poly;
    uint32_t meta;   // bit 0: S, bit 1: last record of the pixel,
                     // bits 2..16: n_local, bits 17..31: n_partial
    uint32_t eoff;   // second local edge in the local-edge array
    uint32_t poff;   // first partial-right y-range in the span array
    Edge e0;         // the first local edge (when n_local > 0)
    double2 s0;      // partial-right range poff (when n_partial > 0)
};
static_assert(sizeof(Cand) == 64, "a candidate record is one 64-byte read");
constexpr uint32_t CAND_S = 1u;
constexpr uint32_t CAND_LAST = 2u;
// Coarse canvas word (one per 2^blog x 2^blog block of pixels):
//   label + 1 (0: in no polygon) when every pixel of the block carries that
//   same non-boundary canvas word;
//   COARSE_FULL otherwise: the point's word is read from the full canvas.
// (An intermediate level of per-pixel codes for blocks of few labels costs
// every wave that meets one a further dependent read; it measured slower
// than reading the full canvas word directly.)
constexpr uint16_t COARSE_FULL = 0xffffu;
// A single canvas of at most COARSE_BYTE_MAXM polygons stores its coarse
// words as bytes, half the LDS for the same block size: label + 1 below
// COARSE_BYTE_FULL.  A uniform block of a larger label is stored as full.
constexpr uint32_t COARSE_BYTE_FULL = 255u;
constexpr int64_t COARSE_BYTE_MAXM = 512;

// Edge in world coordinates with lo.y <= hi.y.
// One canvas of a canvas set: its world->pixel map, bounding box, size and
// where its words live in the set's shared arrays.  A set rasterises many
// polygon groups (one per canvas) in the same kernel launches; canvas q owns
// polygons [poly_base, poly_base + M) and labels them 0..M-1.
struct CanvasDesc {
    double X0, Y0, sx, sy, hy;    // pixel u = (x - X0) * sx, v = (y - Y0) * sy; hy = 1 / sy
    double bx0, by0, bx1, by1;    // half-open bounding box of the canvas's polygons
    int32_t W, H, Wt, Wc, Hc, blog;
    int32_t empty;                // no polygon area: every point is outside
    int32_t cbyte;                // coarse words are bytes (see COARSE_BYTE_*)
    int64_t poly_base, M;
    int64_t row_base;             // first global row of the set
    int64_t cell_off;             // first canvas word (tile-major, 16 x 16 tiles)
    int64_t coarse_off;           // first coarse word
};

// Everything a probe kernel needs, passed by value.
struct CanvasView {
    double X0, Y0, sx, sy;        // pixel u = (x - X0) * sx, v = (y - Y0) * sy
    double bx0, by0, bx1, by1;    // half-open bounding box of all polygons
    int32_t W, H;
    int32_t Wt;                   // 16 x 16 pixel tiles per canvas row
    int32_t Wc, Hc, blog;         // coarse grid: one word per 2^blog x 2^blog pixels
    int32_t cbyte;                // coarse words are bytes (see COARSE_BYTE_*)
    int64_t M;                    // number of polygons
    const uint32_t *cells;        // canvas words, tile-major (16 x 16 tiles)
    const uint16_t *coarse;       // Wc * Hc coarse words, row-major
    const Cand *cands;
    const Edge *ledges;           // local edges of the records
    const double2 *pspan;         // (ylo, yhi) of partial-right edges
};

// Growable device buffer owned by a context or canvas.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

}  // namespace spade

struct spade_canvas {
    int device = 0;
    int nc = 1;                               // canvases in the set
    std::vector<spade::CanvasDesc> descs;     // host copy of the canvas descriptors
    spade::DevBuf dcds;                       // device copy
    spade::CanvasView view{};                 // probe view of canvas 0
    int64_t n_boundary = 0;
    int64_t n_cands = 0;
    int64_t n_elist = 0;
    int64_t n_edges = 0;
    spade::DevBuf cells, cands, ledges, pspan, edges, coarse;
    spade::DevBuf pid;                        // layered set: caller's polygon id of each set polygon
    bool layered = false;
    int32_t n_layers = 0;
    std::vector<uint64_t> gkey;               // launch parameters of the last build
    hipGraphExec_t gexec = nullptr;           // its captured launches (second build on)
    std::vector<uint64_t> bkey;               // batch join-count: launch parameters of the last call
    hipGraphExec_t bexec = nullptr;           // its captured launches (second call on)
    spade::DevBuf qbox;                       // per-canvas boxes for the batch join-count
    bool pending = false;                     // built, counters and flags not yet read
    const void *pend_src = nullptr;           // their device block, until build_flush copies it
    size_t bytes() const
    {
        return cells.cap + cands.cap + ledges.cap + pspan.cap + coarse.cap;
    }
};

struct spade_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int32_t canvas_w = 0, canvas_h = 0;     // 0 = automatic
    double ppv = 256.0;                     // automatic sizing: pixels per vertex
    spade::DevBuf scratch[22];              // reusable scratch slots (spade::S_NSLOTS)
    void *pinned = nullptr;                 // small pinned host staging area
    void *pend = nullptr;                   // pinned counters and flags of a deferred build
    spade_canvas *plain = nullptr;          // canvas reused by the plain query calls
    bool timing = false;                    // record phase events (raster, probe)
    bool timed_raster = false;              // last query rasterised under timing
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t pinned_cap = 0;
    hipStream_t side = nullptr;             // internal streams for overlapped launches
    hipStream_t side2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
    hipEvent_t evinfo = nullptr;            // a build's row totals reached the host
    hipStream_t capture = nullptr;          // internal stream graphs are captured on
    bool graphs = true;                     // replay repeated canvas builds from graphs
    int64_t graph_captures = 0, graph_replays = 0;
    int64_t builds = 0, rebuilds = 0;       // plain-call canvas builds, and those redone for capacity
    int64_t batch_overlaps = 0;             // last batch selection / join pairs: (chunk, query) overlaps
    void *jobs = nullptr;                   // asynchronous batch jobs: queue and worker thread
    // Held by every call that uses the context's stream, scratch or state,
    // and by the job worker while it runs a job: a call made while a job
    // runs waits for it instead of sharing scratch buffers with it.
    mutable std::recursive_mutex mu;
};

#define SPADE_CTX_LOCK(c) std::lock_guard<std::recursive_mutex> spade_ctx_guard_((c)->mu)

namespace spade {

// Scratch slot ids inside a context.
enum Slot {
    S_BLOCKRED = 0, S_RINGPOLY, S_NROWS, S_ROWOFF, S_KEYS, S_KEYS2, S_VALS, S_VALS2,
    S_ENTC, S_ENTF, S_CUBTMP, S_ROWCNT, S_NEXTP, S_PROBE, S_LOOKBACK, S_MISC, S_ROWSCAN,
    S_BITS,     // per-point result bits of the ordered emits (count pass to write pass)
    S_BUF_SEGS, S_BUF_GRID, S_BUF_LIST, S_BUF_TMP,   // distance selection from lines / a polygon
    S_NSLOTS
};

static_assert(S_NSLOTS == 22, "scratch slot count of spade_ctx");

// Points per segment of the ordered emit (bits: EMIT_SEG / 64 words each).
constexpr int EMIT_SEG = 1024;
// Write pass of an ordered selection from per-point result bits: segment sg
// of EMIT_SEG points writes its ids from offs[sg] on (below cap).
__global__ void k_emit_bits(int64_t nseg, const unsigned long long *offs, const unsigned long long *bits,
                            uint32_t *out_pt, uint32_t *out_poly, int64_t cap);

int set_error(spade_ctx *ctx, int code, const std::string &msg);
int hip_fail(spade_ctx *ctx, hipError_t e, const char *what);
int ensure(spade_ctx *ctx, DevBuf &b, size_t bytes);
void *ensure_pinned(spade_ctx *ctx, size_t bytes);
int ensure_keep(spade_ctx *ctx, DevBuf &b, size_t bytes);
int hip_fail_if(spade_ctx *ctx, hipError_t e);
int plain_canvas(spade_ctx *ctx, const spade_polys *polys, spade_canvas **cvo);
void jobs_shutdown(spade_ctx *ctx);
size_t jobs_bytes(const spade_ctx *ctx);
void free_buf(DevBuf &b);

// `defer`: leave the build's counters and flags on the device instead of
// waiting for them; build_flush queues their copy to the host (after the
// caller's own launches) and build_finish reads it after the caller's next
// synchronisation.
int build_canvas(spade_ctx *ctx, const spade_polys *polys, spade_canvas *cv, bool defer = false);
int build_flush(spade_ctx *ctx, spade_canvas *cv);
// Completes a deferred build; returns BUILD_AGAIN when the single row pass
// ran out of capacity (grown by now: build again, non-deferred).
constexpr int BUILD_AGAIN = 1;
int build_finish(spade_ctx *ctx, spade_canvas *cv);
void drop_graph(spade_canvas *cv);
void drop_batch_graph(spade_canvas *cv);
// Rasterises polygons [pbound[q], pbound[q+1]) into canvas q, q < nc.
int build_set(spade_ctx *ctx, const spade_polys *polys, int nc, const int64_t *pbound, spade_canvas *cv,
              bool defer = false);
CanvasView view_of(const spade_canvas *cv, int q);
// Layer index of a polygon set (layer of each polygon in d_layer, device)
// and a canvas set with one canvas per layer.
struct HostSet;
int layer_index(spade_ctx *ctx, const spade_polys *polys, int res, int32_t *d_layer, int32_t *n_layers,
                std::vector<int32_t> *host_layer, HostSet *hs_out);
int layered_build(spade_ctx *ctx, const spade_polys *polys, int res, spade_canvas *cv, int32_t *n_layers);

// Distance selection: the points within closed distance r of a segment of
// `geom`'s rings (open polylines, or closed rings when `closed`), or kept by
// the one-polygon canvas `cv` when it is not NULL; ascending ids.
int buffer_select(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, const spade_polys *geom, double r,
                  bool closed, uint32_t *out_ids, int64_t cap, int64_t *n_out);

// Distance join with lines: pairs (point, line) of the points within r[line]
// (or r_all when r is NULL) of each ring of `lines` as an open polyline, in
// (point, line) order; or, with out_counts, the pairs per line.
int buffer_join_lines(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines, const double *r,
                      double r_all, uint32_t *out_pt, uint32_t *out_line, int64_t cap, int64_t *n_out,
                      uint64_t *out_counts);

// LDS bytes the count probe leaves for the coarse canvas, given the polygon
// count (its histogram shares the LDS).
size_t coarse_lds_budget(int64_t M);

int probe_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                uint64_t *out_counts);
// Plain read of every point (bandwidth reference for the probe).
int stream_read(spade_ctx *ctx, const spade_points *pts, int shape, double *out);
// The same probe with its scratch in a fixed device array (no allocation);
// noalloc_init looks the array's address up for ctx's device.
int noalloc_init(spade_ctx *ctx);
int probe_count_noalloc(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
                        uint64_t *out_counts);
int select_disk(spade_ctx *ctx, const spade_points *pts, double cx, double cy, double r, uint32_t *out_ids,
                int64_t cap, int64_t *n_out);
// Distance joins of points with disks (pairs, or per-disk counts when
// out_counts is given) and kNN selection.
int distance_join(spade_ctx *ctx, const spade_points *pts, const spade_disks *dk, uint32_t *out_pt,
                  uint32_t *out_disk, int64_t cap, int64_t *n_out, uint64_t *out_counts);
int knn_select(spade_ctx *ctx, const spade_points *pts, double px, double py, int64_t k, uint32_t *out_ids,
               int64_t *n_out);
int probe_emit(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts,
               uint32_t *out_pt, uint32_t *out_poly, int64_t cap, int64_t *n_out);

}  // namespace spade

#define SPADE_HIP(ctx, call)                                               \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return spade::hip_fail((ctx), e_, #call);    \
    } while (0)
