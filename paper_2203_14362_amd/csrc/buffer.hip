// Distance selection from lines and from a polygon: the rounded rectangles
// of Sec. 4.2 (every position within distance r of a segment) drawn around
// every segment of a set of polylines, or around every edge of a polygon
// together with the polygon itself, and the distance selection of Sec. 5.2
// over that shape.
//
// Instead of rasterising the rounded rectangles, the segments are binned
// into a uniform grid over their box widened by r: a cell lists every
// segment whose widened box meets it (count, scan, fill).  One pass over the
// points then keeps, per 1024-point segment of the stream, one result bit
// per point: for a polygon, the canvas of the polygon answers first (coarse
// level in LDS, full canvas, exact records, as the selection probe does);
// a point not yet kept that lies in the grid's box is tested exactly against
// the segments its cell lists, until one is within r.  The tests of a
// wavefront's 64 points are spread over its lanes (buf_wave_walk), so that a
// wavefront takes about as many rounds as its points have candidates in
// total / 64 rather than as many as its longest list.  The ordered ids are
// then written from the bits (the two-step Map of the selection).
#include "common.h"
#include "lookup.h"
#include "segdist.h"
#include "wavewalk.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace spade {

constexpr int BUF_GRID_MAX = 4096;            // cells per side
constexpr int BUF_THREADS = 1024;
constexpr int BUF_WORDS = EMIT_SEG / 64;      // bit words per point segment

// Order-preserving 64-bit key of a double (minima by atomicMin).
__device__ __forceinline__ unsigned long long buf_key(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

static double buf_from_key(unsigned long long k)
{
    const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// The grid: cells of side `cell` (1 / inv) from (X0, Y0); (X1, Y1) closes
// the box.
struct BufGrid {
    double X0, Y0, X1, Y1, inv, cell;
    int gx, gy;
};

__device__ __forceinline__ int buf_cell(double v, double v0, double inv, int g)
{
    const double u = __dmul_rn(__dsub_rn(v, v0), inv);
    return (int)fmin(fmax(floor(u), 0.0), (double)(g - 1));
}

// One segment slot per vertex: vertex v of its ring to the next one (the
// ring's first vertex after the last when `closed`; a one-vertex ring is a
// point).  Validates the offsets and the vertices on the way (err bit 1:
// offsets, bit 2: a non-finite vertex) and reduces the segments' box into
// bb (min x, -max x, min y, -max y as ordered keys); sums the segments'
// lengths (an FP64 estimate, only for the grid's cell size) into *len.
__global__ void k_buf_segs(int64_t R, const int64_t *rvo, int64_t V, const double *vx, const double *vy,
                           int closed, Seg *segs, uint8_t *valid, unsigned long long *bb, unsigned *err,
                           double *len)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = gid; k <= R; k += nth) {
        const int64_t o = rvo[k];
        if ((k == 0 && o != 0) || (k == R && o != V) || (k < R && rvo[k + 1] < o)) atomicOr(err, 1u);
    }
    unsigned long long k0 = ~0ull, k1 = ~0ull, k2 = ~0ull, k3 = ~0ull;
    double lsum = 0.0;
    for (int64_t v = gid; v < V; v += nth) {
        valid[v] = 0;
        // ring of v: the last ring whose first vertex is <= v
        int64_t lo = 0, hi = R - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (rvo[mid] <= v) lo = mid; else hi = mid - 1;
        }
        const int64_t o = rvo[lo], e = rvo[lo + 1];
        if (!(o >= 0 && o <= v && v < e && e <= V)) {
            atomicOr(err, 1u);
            continue;
        }
        int64_t w;
        if (e - o == 1) w = v;
        else if (v + 1 < e) w = v + 1;
        else if (closed) w = o;
        else continue;
        const double ax = vx[v], ay = vy[v], bx = vx[w], by = vy[w];
        if (!(isfinite(ax) && isfinite(ay) && isfinite(bx) && isfinite(by))) {
            atomicOr(err, 2u);
            continue;
        }
        segs[v] = Seg{ax, ay, bx, by};
        valid[v] = 1;
        lsum += hypot(bx - ax, by - ay);
        k0 = min(k0, min(buf_key(ax), buf_key(bx))); k1 = min(k1, min(buf_key(-ax), buf_key(-bx)));
        k2 = min(k2, min(buf_key(ay), buf_key(by))); k3 = min(k3, min(buf_key(-ay), buf_key(-by)));
    }
    for (int d = 32; d > 0; d >>= 1) {
        k0 = min(k0, (unsigned long long)__shfl_xor((long long)k0, d, 64));
        k1 = min(k1, (unsigned long long)__shfl_xor((long long)k1, d, 64));
        k2 = min(k2, (unsigned long long)__shfl_xor((long long)k2, d, 64));
        k3 = min(k3, (unsigned long long)__shfl_xor((long long)k3, d, 64));
    }
    for (int d = 32; d > 0; d >>= 1) lsum += __shfl_xor(lsum, d, 64);
    if ((threadIdx.x & 63) == 0 && k0 != ~0ull) {
        atomicMin(&bb[0], k0); atomicMin(&bb[1], k1); atomicMin(&bb[2], k2); atomicMin(&bb[3], k3);
        atomicAdd(len, lsum);
    }
}

// Cells that may hold a point within r of each valid segment: the cells of
// its box widened by pad whose centre lies within r + half the cell diagonal
// of the segment (FP64 distance, with a relative margin of 1e-9 and the
// absolute part of pad, far above its rounding and that of the point-to-cell
// mapping), counted (FILL false, with the number of list entries summed into
// *tot) or listed (FILL true: a copy of the segment in a per-cell slot from
// off[] claimed with cursor[], so that a point reads its cell's candidates
// contiguously, with no index to follow).
template <bool FILL>
__global__ void k_buf_bin(int64_t V, const Seg *segs, const uint8_t *valid, BufGrid g, double pad, uint32_t *cnt,
                          const uint32_t *off, Seg *list, unsigned long long *tot)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += nth) {
        if (!valid[v]) continue;
        const Seg s = segs[v];
        const int x0 = buf_cell(fmin(s.ax, s.bx) - pad, g.X0, g.inv, g.gx);
        const int x1 = buf_cell(fmax(s.ax, s.bx) + pad, g.X0, g.inv, g.gx);
        const int y0 = buf_cell(fmin(s.ay, s.by) - pad, g.Y0, g.inv, g.gy);
        const int y1 = buf_cell(fmax(s.ay, s.by) + pad, g.Y0, g.inv, g.gy);
        const double ex = s.bx - s.ax, ey = s.by - s.ay, l2 = ex * ex + ey * ey;
        const double reach = (pad + 0.7071067811865476 * g.cell) * (1.0 + 1e-9);
        const double reach2 = reach * reach;
        unsigned long long nlisted = 0;
        for (int cy = y0; cy <= y1; ++cy)
            for (int cx = x0; cx <= x1; ++cx) {
                const double px = g.X0 + (cx + 0.5) * g.cell, py = g.Y0 + (cy + 0.5) * g.cell;
                double t = l2 > 0.0 ? ((px - s.ax) * ex + (py - s.ay) * ey) / l2 : 0.0;
                t = fmin(fmax(t, 0.0), 1.0);
                const double dx = px - (s.ax + t * ex), dy = py - (s.ay + t * ey);
                if (dx * dx + dy * dy > reach2) continue;
                const int64_t c = (int64_t)cy * g.gx + cx;
                if (FILL) list[off[c] + atomicAdd(&cnt[c], 1u)] = s;
                else atomicAdd(&cnt[c], 1u);
                ++nlisted;
            }
        if (!FILL) atomicAdd(tot, nlisted);
    }
}

// The candidate tests of one wavefront's points, balanced over its lanes
// (wave_round): lane i's point has the candidates list[k, k + rem) left, and
// a point any of whose candidates in a round was within r drops the rest.
// Returns whether this lane's point was hit.  Called by every lane of the
// wavefront.
__device__ __forceinline__ bool buf_wave_walk(double x, double y, uint32_t k, uint32_t rem, const Seg *list,
                                              double r, double r2, double pad, int lane)
{
    bool hit = false;
    while (__ballot(rem != 0u)) {
        const WaveRound w = wave_round(rem, lane);
        const uint32_t ok = __shfl(k, w.o, 64);
        const double ox = __shfl(x, w.o, 64), oy = __shfl(y, w.o, 64);
        bool h = false;
        if ((uint32_t)lane < w.ntake) {
            const Seg s = list[ok + ((uint32_t)lane - w.opre)];
            // outside the segment's box widened by pad: farther than r
            if (!(ox < fmin(s.ax, s.bx) - pad || ox > fmax(s.ax, s.bx) + pad || oy < fmin(s.ay, s.by) - pad ||
                  oy > fmax(s.ay, s.by) + pad))
                h = seg_near(ox, oy, s, r, r2);
        }
        const unsigned long long hm = __ballot(h);
        const uint32_t len = wave_round_len(w);
        if (hm & wave_round_mask(w)) {
            hit = true;
            rem = 0u;
        } else {
            k += len;
            rem -= len;
        }
    }
    return hit;
}

// One result bit per point (layout of the ordered emit: word j of segment sg
// holds points sg * EMIT_SEG + 64 j + lane) and the count per segment.
template <bool POLY>
__global__ __launch_bounds__(BUF_THREADS) void k_buf_bits(CanvasView cv, int64_t n, const double *X, const double *Y,
                                                          BufGrid g, const Seg *segs, const uint32_t *off,
                                                          const Seg *list, double r, double r2, double pad,
                                                          int64_t nseg, unsigned long long *counts,
                                                          unsigned long long *bits)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *coarse = (uint16_t *)smem;
    if (POLY) {
        load_coarse(cv, coarse, BUF_THREADS);
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * BUF_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * BUF_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        unsigned long long total = 0, segw = 0;
        for (int j = 0; j < BUF_WORDS; ++j) {
            const int64_t i = sg * EMIT_SEG + 64 * j + lane;
            const double x = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            const double y = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
            bool hit = false;
            if (POLY) {
                const uint32_t w = lookup(cv, coarse, x, y);
                if (w != 0u && !(w & BFLAG)) {
                    hit = true;
                } else if (w & BFLAG) {
                    uint32_t rec = w & ~BFLAG;
                    while (true) {
                        const Cand c = cv.cands[rec];
                        if (cand_inside(cv, c, x, y)) { hit = true; break; }
                        if (c.meta & CAND_LAST) break;
                        ++rec;
                    }
                }
            }
            // NaN fails the box test
            uint32_t k = 0u, rem = 0u;
            if (!hit && x >= g.X0 && x <= g.X1 && y >= g.Y0 && y <= g.Y1) {
                const int64_t c = (int64_t)buf_cell(y, g.Y0, g.inv, g.gy) * g.gx + buf_cell(x, g.X0, g.inv, g.gx);
                k = off[c];
                rem = off[c + 1] - k;
            }
            if (buf_wave_walk(x, y, k, rem, list, r, r2, pad, lane)) hit = true;
            const unsigned long long word = __ballot(hit);
            total += (unsigned long long)__popcll(word);
            if (lane == j) segw = word;
        }
        if (lane < BUF_WORDS) bits[sg * BUF_WORDS + lane] = segw;
        if (lane == 0) counts[sg] = total;
    }
}

__global__ void k_buf_zero(unsigned long long *p) { *p = 0ull; }

int buffer_select(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, const spade_polys *geom, double r,
                  bool closed, uint32_t *out_ids, int64_t cap, int64_t *n_out)
{
    hipStream_t st = ctx->stream;
    if (n_out) *n_out = 0;
    if (!(std::isfinite(r) && r >= 0.0)) return set_error(ctx, SPADE_E_INVALID, "the distance must be finite and >= 0");
    if (cap < 0) return set_error(ctx, SPADE_E_INVALID, "negative capacity");
    if (cap > 0 && !out_ids) return set_error(ctx, SPADE_E_INVALID, "out_ids is NULL");
    if (!geom) return set_error(ctx, SPADE_E_INVALID, "geometry is NULL");
    const int64_t R = geom->n_rings;
    if (R < 0) return set_error(ctx, SPADE_E_INVALID, "negative ring count");
    if (R > 0 && (!geom->ring_vtx_off || !geom->vx || !geom->vy))
        return set_error(ctx, SPADE_E_INVALID, "geometry array is NULL");
    // vertex count: given, else read back
    int64_t V = 0;
    if (R > 0) {
        if (geom->n_vertices > 0) {
            V = geom->n_vertices;
        } else {
            int64_t *h = (int64_t *)ensure_pinned(ctx, 64);
            if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
            SPADE_HIP(ctx, hipMemcpyAsync(h, geom->ring_vtx_off + R, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SPADE_HIP(ctx, hipStreamSynchronize(st));
            V = h[0];
        }
        if (V < 0 || V >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_INVALID, "bad vertex count");
    }
    const int64_t n = pts->n;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        cus = 256;

    // segments, their box, validation
    DevBuf &bs = ctx->scratch[S_BUF_SEGS], &bg = ctx->scratch[S_BUF_GRID];
    if (ensure(ctx, bs, sizeof(Seg) * (size_t)std::max<int64_t>(V, 1) + (size_t)V + 16) || ensure(ctx, bg, 256))
        return SPADE_E_NOMEM;
    Seg *segs = (Seg *)bs.p;
    uint8_t *valid = (uint8_t *)(segs + std::max<int64_t>(V, 1));
    unsigned long long *bb = (unsigned long long *)bg.p;
    unsigned *err = (unsigned *)(bb + 4);
    double *dlen = (double *)(bb + 6);
    SPADE_HIP(ctx, hipMemsetAsync(bb, 0xff, 4 * sizeof(unsigned long long), st));
    SPADE_HIP(ctx, hipMemsetAsync(err, 0, sizeof(unsigned), st));
    SPADE_HIP(ctx, hipMemsetAsync(dlen, 0, sizeof(double), st));
    if (R > 0) {
        const int sgrid = (int)std::max<int64_t>(1, std::min<int64_t>((std::max(V, R + 1) + 255) / 256, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_buf_segs, dim3(sgrid), dim3(256), 0, st, R, geom->ring_vtx_off, V, geom->vx, geom->vy,
                           closed ? 1 : 0, segs, valid, bb, err, dlen);
        SPADE_HIP(ctx, hipGetLastError());
    }
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, bb, 7 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const unsigned ef = (unsigned)(h[4] & 0xffffffffu);
    if (ef & 1u) return set_error(ctx, SPADE_E_INVALID, "ring offsets are not a valid CSR array");
    if (ef & 2u) return set_error(ctx, SPADE_E_INVALID, "a vertex coordinate is not finite");
    const bool any = h[0] != ~0ull;
    double len_sum;
    std::memcpy(&len_sum, &h[6], sizeof len_sum);
    if (n == 0) return SPADE_OK;

    // the grid over the segments' box widened by r (and a relative margin,
    // so that rounding never drops a position within r)
    BufGrid grid{0.0, 0.0, -1.0, -1.0, 1.0, 1.0, 1, 1};   // empty box: no point is tested
    double pad = 0.0;
    uint32_t *off = nullptr;
    Seg *list = nullptr;
    if (any) {
        const double x0 = buf_from_key(h[0]), x1 = -buf_from_key(h[1]);
        const double y0 = buf_from_key(h[2]), y1 = -buf_from_key(h[3]);
        const double mag = std::fabs(x0) + std::fabs(x1) + std::fabs(y0) + std::fabs(y1);
        pad = r * (1.0 + 0x1p-40) + mag * 0x1p-40 + 1e-300;
        const double X0 = x0 - pad, X1 = x1 + pad, Y0 = y0 - pad, Y1 = y1 + pad;
        const double w = X1 - X0, hgt = Y1 - Y0;
        // cells as wide as r or the mean segment length, whichever is
        // larger (a segment then meets a few cells, a cell a few segments),
        // at most BUF_GRID_MAX per side
        const double lmean = std::isfinite(len_sum) ? len_sum / (double)std::max<int64_t>(V, 1) : 0.0;
        double cell = std::max(r, std::min(lmean, std::sqrt(w * hgt / (2.0 * (double)std::max<int64_t>(V, 1)))));
        cell = std::max(cell, std::max(w, hgt) / BUF_GRID_MAX);
        if (!(cell > 1e-290)) cell = 1.0;
        grid.X0 = X0; grid.Y0 = Y0; grid.X1 = X1; grid.Y1 = Y1;
        grid.inv = 1.0 / cell;
        grid.cell = cell;
        grid.gx = (int)std::min<double>(BUF_GRID_MAX, std::max(1.0, std::ceil(w * grid.inv)));
        grid.gy = (int)std::min<double>(BUF_GRID_MAX, std::max(1.0, std::ceil(hgt * grid.inv)));
        const int64_t G = (int64_t)grid.gx * grid.gy;
        DevBuf &bt = ctx->scratch[S_BUF_TMP];
        if (ensure(ctx, bg, 256 + sizeof(uint32_t) * 3 * (size_t)(G + 1))) return SPADE_E_NOMEM;
        bb = (unsigned long long *)bg.p;
        uint32_t *cnt = (uint32_t *)((unsigned char *)bg.p + 256);
        off = cnt + (G + 1);
        uint32_t *cursor = off + (G + 1);
        unsigned long long *tot = bb + 5;
        SPADE_HIP(ctx, hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)(G + 1), st));
        SPADE_HIP(ctx, hipMemsetAsync(tot, 0, sizeof(unsigned long long), st));
        const int bgrid = (int)std::max<int64_t>(1, std::min<int64_t>((V + 255) / 256, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_buf_bin<false>, dim3(bgrid), dim3(256), 0, st, V, (const Seg *)segs,
                           (const uint8_t *)valid, grid, pad, cnt, (const uint32_t *)nullptr, (Seg *)nullptr,
                           tot);
        SPADE_HIP(ctx, hipGetLastError());
        size_t tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)(G + 1), st));
        if (ensure(ctx, bt, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(bt.p, tb, cnt, off, (int)(G + 1), st));
        // the 64-bit entry count first: the cell lists (32 bytes an entry)
        // stay below 2^28 entries, so their 32-bit offsets are exact
        SPADE_HIP(ctx, hipMemcpyAsync(h, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        if (h[0] >= ((unsigned long long)1 << 28))
            return set_error(ctx, SPADE_E_TOO_LARGE, "too many (segment, cell) entries: the distance is too large "
                                                     "for the segments' spread");
        const uint64_t total = h[0];
        DevBuf &bl = ctx->scratch[S_BUF_LIST];
        if (ensure(ctx, bl, sizeof(Seg) * (size_t)std::max<uint64_t>(total, 1))) return SPADE_E_NOMEM;
        list = (Seg *)bl.p;
        SPADE_HIP(ctx, hipMemsetAsync(cursor, 0, sizeof(uint32_t) * (size_t)(G + 1), st));
        hipLaunchKernelGGL(k_buf_bin<true>, dim3(bgrid), dim3(256), 0, st, V, (const Seg *)segs,
                           (const uint8_t *)valid, grid, pad, cursor, (const uint32_t *)off, list,
                           (unsigned long long *)nullptr);
        SPADE_HIP(ctx, hipGetLastError());
    }

    // result bits and per-segment counts, then the ordered write pass
    const int64_t nseg = (n + EMIT_SEG - 1) / EMIT_SEG;
    DevBuf &lb = ctx->scratch[S_LOOKBACK], &bbits = ctx->scratch[S_BITS];
    if (ensure(ctx, lb, sizeof(unsigned long long) * 2 * (size_t)(nseg + 1)) ||
        ensure(ctx, bbits, sizeof(unsigned long long) * BUF_WORDS * (size_t)nseg))
        return SPADE_E_NOMEM;
    unsigned long long *counts = (unsigned long long *)lb.p;
    unsigned long long *offs = counts + (nseg + 1);
    unsigned long long *bits = (unsigned long long *)bbits.p;
    const double r2 = r * r;
    const int64_t wpb = BUF_THREADS / 64;
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (cv) {
        const CanvasView &v = cv->view;
        const size_t lds = ((size_t)v.Wc * v.Hc * (v.cbyte ? 1 : 2) + 15) & ~(size_t)15;
        if (lds + 2048 > 160 * 1024) return set_error(ctx, SPADE_E_HIP, "internal: coarse level exceeds the LDS");
        const int per_cu = std::max<int>(1, (int)((160 * 1024) / (lds + 2048)));
        const int grid_b = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + wpb - 1) / wpb, (int64_t)cus * std::min(per_cu, 2)));
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_buf_bits<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_buf_bits<true>, dim3(grid_b), dim3(BUF_THREADS), lds, st, v, n, pts->x, pts->y, grid,
                           (const Seg *)segs, (const uint32_t *)off, (const Seg *)list, r, r2, pad, nseg, counts,
                           bits);
    } else {
        const int grid_b = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + wpb - 1) / wpb, (int64_t)cus * 2));
        hipLaunchKernelGGL(k_buf_bits<false>, dim3(grid_b), dim3(BUF_THREADS), 0, st, CanvasView{}, n, pts->x, pts->y,
                           grid, (const Seg *)segs, (const uint32_t *)off, (const Seg *)list, r, r2, pad, nseg,
                           counts, bits);
    }
    hipLaunchKernelGGL(k_buf_zero, dim3(1), dim3(1), 0, st, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &bt = ctx->scratch[S_BUF_TMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, bt, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(bt.p, tb, counts, offs, (int)(nseg + 1), st));
    if (cap > 0) {
        const int eg = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + 3) / 4, (int64_t)cus * 16));
        hipLaunchKernelGGL(k_emit_bits, dim3(eg), dim3(256), 0, st, nseg, (const unsigned long long *)offs,
                           (const unsigned long long *)bits, out_ids, (uint32_t *)nullptr, cap);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (n_out) *n_out = (int64_t)h[0];
    if ((int64_t)h[0] > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}


// ------------------------------------------------------------ distance join with lines
//
// Sec. 5.2's distance joins of types (1) and (2) with lines as the
// constraint dataset: every ring of the line set is one line object j (an
// open polyline) with its distance r_j (type 2) or one distance for all
// (type 1), and the join returns the pairs (point, line) of the points within
// r_j of line j.  The segments, each with its line and distance, are binned
// as for the selection; each cell's list is then sorted by segment id, so
// that a line's segments are consecutive in it and a point meets each of its
// lines once, in ascending line order: the first segment of a line within
// that line's distance emits the pair, the rest of the line is skipped.

struct JSeg {
    double ax, ay, bx, by, r;
    uint32_t line, pad_;
};

// Segment slot v of a set of open polylines: its line (ring) and far end,
// or false (last vertex of a ring, or malformed offsets: err bit 1).
__device__ __forceinline__ bool line_seg_of(int64_t R, const int64_t *rvo, int64_t V, int64_t v, int64_t &ring,
                                            int64_t &w, unsigned *err)
{
    int64_t lo = 0, hi = R - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rvo[mid] <= v) lo = mid; else hi = mid - 1;
    }
    const int64_t o = rvo[lo], e = rvo[lo + 1];
    if (!(o >= 0 && o <= v && v < e && e <= V)) {
        atomicOr(err, 1u);
        return false;
    }
    ring = lo;
    if (e - o == 1) w = v;
    else if (v + 1 < e) w = v + 1;
    else return false;
    return true;
}

// Segments with their line and distance; validates offsets (err bit 1),
// vertices (bit 2) and distances (bit 4); reduces the segments' box into bb
// and the largest distance into bb[7] (as the ordered key of -r).
__global__ void k_bufj_segs(int64_t R, const int64_t *rvo, int64_t V, const double *vx, const double *vy,
                            const double *rline, double r_all, JSeg *segs, uint8_t *valid,
                            unsigned long long *bb, unsigned *err, double *len)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t k = gid; k <= R; k += nth) {
        const int64_t o = rvo[k];
        if ((k == 0 && o != 0) || (k == R && o != V) || (k < R && rvo[k + 1] < o)) atomicOr(err, 1u);
        if (k < R && rline && !(isfinite(rline[k]) && rline[k] >= 0.0)) atomicOr(err, 4u);
    }
    unsigned long long k0 = ~0ull, k1 = ~0ull, k2 = ~0ull, k3 = ~0ull, kr = ~0ull;
    double lsum = 0.0;
    for (int64_t v = gid; v < V; v += nth) {
        valid[v] = 0;
        int64_t ring, w;
        if (!line_seg_of(R, rvo, V, v, ring, w, err)) continue;
        const double ax = vx[v], ay = vy[v], bx = vx[w], by = vy[w];
        const double r = rline ? rline[ring] : r_all;
        if (!(isfinite(ax) && isfinite(ay) && isfinite(bx) && isfinite(by))) {
            atomicOr(err, 2u);
            continue;
        }
        if (!(isfinite(r) && r >= 0.0)) continue;   // reported through bit 4
        segs[v] = JSeg{ax, ay, bx, by, r, (uint32_t)ring, 0u};
        valid[v] = 1;
        lsum += hypot(bx - ax, by - ay);
        k0 = min(k0, min(buf_key(ax), buf_key(bx))); k1 = min(k1, min(buf_key(-ax), buf_key(-bx)));
        k2 = min(k2, min(buf_key(ay), buf_key(by))); k3 = min(k3, min(buf_key(-ay), buf_key(-by)));
        kr = min(kr, buf_key(-r));
    }
    for (int d = 32; d > 0; d >>= 1) {
        k0 = min(k0, (unsigned long long)__shfl_xor((long long)k0, d, 64));
        k1 = min(k1, (unsigned long long)__shfl_xor((long long)k1, d, 64));
        k2 = min(k2, (unsigned long long)__shfl_xor((long long)k2, d, 64));
        k3 = min(k3, (unsigned long long)__shfl_xor((long long)k3, d, 64));
        kr = min(kr, (unsigned long long)__shfl_xor((long long)kr, d, 64));
        lsum += __shfl_xor(lsum, d, 64);
    }
    if ((threadIdx.x & 63) == 0 && k0 != ~0ull) {
        atomicMin(&bb[0], k0); atomicMin(&bb[1], k1); atomicMin(&bb[2], k2); atomicMin(&bb[3], k3);
        atomicMin(&bb[7], kr);
        atomicAdd(len, lsum);
    }
}

// Cells that may hold a point within a segment's own distance of it (as
// k_buf_bin, with the segment's pad r (1 + 2^-40) + magpad): counted
// (FILL false, entries summed into *tot) or listed as sort keys
// (cell << 32 | segment) with the segment as value.
template <bool FILL>
__global__ void k_bufj_bin(int64_t V, const JSeg *segs, const uint8_t *valid, BufGrid g, double magpad,
                           uint32_t *cnt, const uint32_t *off, unsigned long long *keys, uint32_t *vals,
                           unsigned long long *tot)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += nth) {
        if (!valid[v]) continue;
        const JSeg s = segs[v];
        const double pad = s.r * (1.0 + 0x1p-40) + magpad;
        const int x0 = buf_cell(fmin(s.ax, s.bx) - pad, g.X0, g.inv, g.gx);
        const int x1 = buf_cell(fmax(s.ax, s.bx) + pad, g.X0, g.inv, g.gx);
        const int y0 = buf_cell(fmin(s.ay, s.by) - pad, g.Y0, g.inv, g.gy);
        const int y1 = buf_cell(fmax(s.ay, s.by) + pad, g.Y0, g.inv, g.gy);
        const double ex = s.bx - s.ax, ey = s.by - s.ay, l2 = ex * ex + ey * ey;
        const double reach = (pad + 0.7071067811865476 * g.cell) * (1.0 + 1e-9);
        const double reach2 = reach * reach;
        unsigned long long nlisted = 0;
        for (int cy = y0; cy <= y1; ++cy)
            for (int cx = x0; cx <= x1; ++cx) {
                const double px = g.X0 + (cx + 0.5) * g.cell, py = g.Y0 + (cy + 0.5) * g.cell;
                double t = l2 > 0.0 ? ((px - s.ax) * ex + (py - s.ay) * ey) / l2 : 0.0;
                t = fmin(fmax(t, 0.0), 1.0);
                const double dx = px - (s.ax + t * ex), dy = py - (s.ay + t * ey);
                if (dx * dx + dy * dy > reach2) continue;
                const int64_t c = (int64_t)cy * g.gx + cx;
                if (FILL) {
                    const uint32_t at = off[c] + atomicAdd(&cnt[c], 1u);
                    keys[at] = ((unsigned long long)c << 32) | (unsigned long long)v;
                    vals[at] = (uint32_t)v;
                } else {
                    atomicAdd(&cnt[c], 1u);
                }
                ++nlisted;
            }
        if (!FILL) atomicAdd(tot, nlisted);
    }
}

// Cell lists in sorted order: copies of the segments.
__global__ void k_bufj_gather(int64_t ntot, const uint32_t *vals, const JSeg *segs, JSeg *list)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += nth) list[i] = segs[vals[i]];
}

// The cell's candidates of a point: list[k, k + rem), or none outside the
// grid's box (NaN fails the test too).
__device__ __forceinline__ void bufj_range(double x, double y, const BufGrid &g, const uint32_t *off, uint32_t &k,
                                           uint32_t &rem)
{
    k = 0u;
    rem = 0u;
    if (x >= g.X0 && x <= g.X1 && y >= g.Y0 && y <= g.Y1) {
        const int64_t c = (int64_t)buf_cell(y, g.Y0, g.inv, g.gy) * g.gx + buf_cell(x, g.X0, g.inv, g.gx);
        k = off[c];
        rem = off[c + 1] - k;
    }
}

// The (point, line) pairs of a wavefront's points, with the candidate tests
// balanced over the lanes (wave_round).  A cell's list is sorted by segment,
// so a line's segments are consecutive in it, and a hit repeats its point's
// previous hit exactly when it has the same line: the previous hit is found
// among the round's earlier positions of the same point, else it is the last
// line the point met in earlier rounds.  A repeated line is not tested again
// once its point has met it in an earlier round.  For each new pair the
// testing lane calls pair(o, slot, line) with o the point's lane and slot =
// base of lane o + the pair's rank among the point's pairs (ascending line
// order); on return cnt holds the number of pairs of this lane's point.
// Called by every lane of the wavefront.
template <typename Pair>
__device__ __forceinline__ void bufj_wave_walk(double x, double y, uint32_t k, uint32_t rem, const JSeg *list,
                                               double magpad, uint32_t base, int lane, uint32_t &cnt, Pair &&pair)
{
    uint32_t last = 0xffffffffu;
    cnt = 0u;
    while (__ballot(rem != 0u)) {
        const WaveRound w = wave_round(rem, lane);
        const uint32_t ok = __shfl(k, w.o, 64);
        const uint32_t olast = __shfl(last, w.o, 64);
        const uint32_t ocnt = __shfl(cnt, w.o, 64);
        const uint32_t obase = __shfl(base, w.o, 64);
        const double ox = __shfl(x, w.o, 64), oy = __shfl(y, w.o, 64);
        bool h = false;
        uint32_t line = 0xffffffffu;
        if ((uint32_t)lane < w.ntake) {
            const JSeg sg = list[ok + ((uint32_t)lane - w.opre)];
            line = sg.line;
            if (line != olast) {
                const double pad = sg.r * (1.0 + 0x1p-40) + magpad;
                if (!(ox < fmin(sg.ax, sg.bx) - pad || ox > fmax(sg.ax, sg.bx) + pad ||
                      oy < fmin(sg.ay, sg.by) - pad || oy > fmax(sg.ay, sg.by) + pad))
                    h = seg_near(ox, oy, Seg{sg.ax, sg.ay, sg.bx, sg.by}, sg.r, sg.r * sg.r);
            }
        }
        const unsigned long long hm = __ballot(h);
        // the previous hit of the same point in this round, if any
        const unsigned long long own = wave_round_before(w, lane);
        const unsigned long long ph = hm & own;
        const uint32_t pline = __shfl(line, ph ? 63 - __clzll((long long)ph) : lane, 64);
        const bool fresh = h && line != (ph ? pline : olast);
        const unsigned long long nm = __ballot(fresh);
        if (fresh) pair(w.o, obase + ocnt + (uint32_t)__popcll(nm & own), line);
        // this point's pairs of the round, and its last hit line
        const unsigned long long mine = wave_round_mask(w);
        const unsigned long long myh = hm & mine;
        const uint32_t hline = __shfl(line, myh ? 63 - __clzll((long long)myh) : lane, 64);
        if (myh) last = hline;
        cnt += (uint32_t)__popcll(nm & mine);
        const uint32_t len = wave_round_len(w);
        k += len;
        rem -= len;
    }
}

// MODE 0: pairs per 1024-point segment (counts[sg]; with pcount, also the
// pairs of every point, so that the write pass walks once); MODE 1: the pairs, from
// offs[sg] on (below cap; the first cap in (point, line) order); MODE 2:
// pairs per line added into lcount (an LDS histogram when nlines <= hist).
template <int MODE>
__global__ __launch_bounds__(BUF_THREADS) void k_bufj_pairs(int64_t n, const double *X, const double *Y, BufGrid g,
                                                            const uint32_t *off, const JSeg *list, double magpad,
                                                            int64_t nseg, unsigned long long *counts,
                                                            const unsigned long long *offs, uint32_t *out_pt,
                                                            uint32_t *out_line, int64_t cap,
                                                            unsigned long long *lcount, int nlines, int hist,
                                                            uint32_t *pcount)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *h = (uint32_t *)smem;
    const bool lds = MODE == 2 && nlines <= hist;
    if (lds) {
        for (int k = threadIdx.x; k < nlines; k += BUF_THREADS) h[k] = 0u;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * BUF_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * BUF_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        unsigned long long total = 0;
        int64_t pos = MODE == 1 ? (int64_t)offs[sg] : 0;
        for (int j = 0; j < BUF_WORDS; ++j) {
            const int64_t i = sg * EMIT_SEG + 64 * j + lane;
            const double x = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            const double y = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
            uint32_t k, rem, cnt;
            bufj_range(x, y, g, off, k, rem);
            if (MODE == 2) {
                bufj_wave_walk(x, y, k, rem, list, magpad, 0u, lane, cnt, [&](int, uint32_t, uint32_t line) {
                    if (lds) atomicAdd(&h[line], 1u);
                    else atomicAdd(&lcount[line], 1ull);
                });
                continue;
            }
            if (MODE == 1 && pcount) {
                cnt = i < n ? pcount[i] : 0u;   // the count pass's pairs of this point
            } else {
                bufj_wave_walk(x, y, k, rem, list, magpad, 0u, lane, cnt, [](int, uint32_t, uint32_t) {});
                if (MODE == 0 && pcount && i < n) pcount[i] = cnt;
            }
            // the wavefront's pairs of this word, in lane order
            uint32_t pre = cnt;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)pre, d, 64);
                if (lane >= d) pre += t;
            }
            const uint32_t wsum = (uint32_t)__shfl((int)pre, 63, 64);
            if (MODE == 1 && wsum) {
                // again, writing each pair at pos + (pairs of earlier lanes) + rank
                const int64_t w0 = sg * EMIT_SEG + 64 * j;
                uint32_t c2;
                bufj_wave_walk(x, y, k, cnt ? rem : 0u, list, magpad, pre - cnt, lane, c2,
                               [&](int o, uint32_t slot, uint32_t line) {
                                   const int64_t p = pos + (int64_t)slot;
                                   if (p < cap) {
                                       out_pt[p] = (uint32_t)(w0 + o);
                                       out_line[p] = line;
                                   }
                               });
            }
            pos += wsum;
            total += wsum;
        }
        if (MODE == 0 && lane == 0) counts[sg] = total;
    }
    if (lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < nlines; k += BUF_THREADS)
            if (h[k]) atomicAdd(&lcount[k], (unsigned long long)h[k]);
    }
}

__global__ void k_bufj_zero(int64_t n, unsigned long long *p)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) p[i] = 0ull;
}

int buffer_join_lines(spade_ctx *ctx, const spade_points *pts, const spade_polys *lines, const double *r,
                      double r_all, uint32_t *out_pt, uint32_t *out_line, int64_t cap, int64_t *n_out,
                      uint64_t *out_counts)
{
    hipStream_t st = ctx->stream;
    if (n_out) *n_out = 0;
    const bool counting = out_counts != nullptr;
    if (!r && !(std::isfinite(r_all) && r_all >= 0.0))
        return set_error(ctx, SPADE_E_INVALID, "the distance must be finite and >= 0");
    if (!counting) {
        if (cap < 0) return set_error(ctx, SPADE_E_INVALID, "negative capacity");
        if (cap > 0 && (!out_pt || !out_line)) return set_error(ctx, SPADE_E_INVALID, "output array is NULL");
    }
    if (!lines) return set_error(ctx, SPADE_E_INVALID, "line set is NULL");
    const int64_t R = lines->n_rings;
    if (R < 0) return set_error(ctx, SPADE_E_INVALID, "negative ring count");
    if (R >= 0x7fffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "line ids must be < 2^31 - 1");
    if (R > 0 && (!lines->ring_vtx_off || !lines->vx || !lines->vy))
        return set_error(ctx, SPADE_E_INVALID, "line array is NULL");
    int64_t V = 0;
    if (R > 0) {
        if (lines->n_vertices > 0) {
            V = lines->n_vertices;
        } else {
            int64_t *hv = (int64_t *)ensure_pinned(ctx, 64);
            if (!hv) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
            SPADE_HIP(ctx, hipMemcpyAsync(hv, lines->ring_vtx_off + R, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SPADE_HIP(ctx, hipStreamSynchronize(st));
            V = hv[0];
        }
        if (V < 0 || V >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_INVALID, "bad vertex count");
    }
    const int64_t n = pts->n;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        cus = 256;
    if (counting && R > 0)
        hipLaunchKernelGGL(k_bufj_zero, dim3((unsigned)std::min<int64_t>((R + 255) / 256, 4096)), dim3(256), 0, st, R,
                           (unsigned long long *)out_counts);

    DevBuf &bs = ctx->scratch[S_BUF_SEGS], &bg = ctx->scratch[S_BUF_GRID];
    if (ensure(ctx, bs, sizeof(JSeg) * (size_t)std::max<int64_t>(V, 1) + (size_t)V + 16) || ensure(ctx, bg, 256))
        return SPADE_E_NOMEM;
    JSeg *segs = (JSeg *)bs.p;
    uint8_t *valid = (uint8_t *)(segs + std::max<int64_t>(V, 1));
    unsigned long long *bb = (unsigned long long *)bg.p;
    unsigned *err = (unsigned *)(bb + 4);
    double *dlen = (double *)(bb + 6);
    SPADE_HIP(ctx, hipMemsetAsync(bb, 0xff, 8 * sizeof(unsigned long long), st));
    SPADE_HIP(ctx, hipMemsetAsync(bb + 4, 0, 3 * sizeof(unsigned long long), st));
    if (R > 0) {
        const int sgrid = (int)std::max<int64_t>(1, std::min<int64_t>((std::max(V, R + 1) + 255) / 256, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_bufj_segs, dim3(sgrid), dim3(256), 0, st, R, lines->ring_vtx_off, V, lines->vx, lines->vy,
                           r, r_all, segs, valid, bb, err, dlen);
        SPADE_HIP(ctx, hipGetLastError());
    }
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, bb, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const unsigned ef = (unsigned)(h[4] & 0xffffffffu);
    if (ef & 1u) return set_error(ctx, SPADE_E_INVALID, "ring offsets are not a valid CSR array");
    if (ef & 2u) return set_error(ctx, SPADE_E_INVALID, "a vertex coordinate is not finite");
    if (ef & 4u) return set_error(ctx, SPADE_E_INVALID, "a line's distance is not finite and >= 0");
    const bool any = h[0] != ~0ull;
    double len_sum;
    std::memcpy(&len_sum, &h[6], sizeof len_sum);
    const double rmax = any ? -buf_from_key(h[7]) : 0.0;
    if (n == 0) return SPADE_OK;

    BufGrid grid{0.0, 0.0, -1.0, -1.0, 1.0, 1.0, 1, 1};   // empty box: no point is tested
    double magpad = 0.0;
    uint32_t *off = nullptr;
    JSeg *list = nullptr;
    if (any) {
        const double x0 = buf_from_key(h[0]), x1 = -buf_from_key(h[1]);
        const double y0 = buf_from_key(h[2]), y1 = -buf_from_key(h[3]);
        const double mag = std::fabs(x0) + std::fabs(x1) + std::fabs(y0) + std::fabs(y1);
        magpad = mag * 0x1p-40 + 1e-300;
        const double pad = rmax * (1.0 + 0x1p-40) + magpad;
        const double X0 = x0 - pad, X1 = x1 + pad, Y0 = y0 - pad, Y1 = y1 + pad;
        const double w = X1 - X0, hgt = Y1 - Y0;
        const double lmean = std::isfinite(len_sum) ? len_sum / (double)std::max<int64_t>(V, 1) : 0.0;
        double cell = std::max(rmax, std::min(lmean, std::sqrt(w * hgt / (2.0 * (double)std::max<int64_t>(V, 1)))));
        cell = std::max(cell, std::max(w, hgt) / BUF_GRID_MAX);
        if (!(cell > 1e-290)) cell = 1.0;
        grid.X0 = X0; grid.Y0 = Y0; grid.X1 = X1; grid.Y1 = Y1;
        grid.inv = 1.0 / cell;
        grid.cell = cell;
        grid.gx = (int)std::min<double>(BUF_GRID_MAX, std::max(1.0, std::ceil(w * grid.inv)));
        grid.gy = (int)std::min<double>(BUF_GRID_MAX, std::max(1.0, std::ceil(hgt * grid.inv)));
        const int64_t G = (int64_t)grid.gx * grid.gy;
        if (ensure(ctx, bg, 256 + sizeof(uint32_t) * 3 * (size_t)(G + 1))) return SPADE_E_NOMEM;
        bb = (unsigned long long *)bg.p;
        uint32_t *cnt = (uint32_t *)((unsigned char *)bg.p + 256);
        off = cnt + (G + 1);
        uint32_t *cursor = off + (G + 1);
        unsigned long long *tot = bb + 5;
        SPADE_HIP(ctx, hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)(G + 1), st));
        SPADE_HIP(ctx, hipMemsetAsync(tot, 0, sizeof(unsigned long long), st));
        const int bgrid = (int)std::max<int64_t>(1, std::min<int64_t>((V + 255) / 256, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_bufj_bin<false>, dim3(bgrid), dim3(256), 0, st, V, (const JSeg *)segs,
                           (const uint8_t *)valid, grid, magpad, cnt, (const uint32_t *)nullptr,
                           (unsigned long long *)nullptr, (uint32_t *)nullptr, tot);
        SPADE_HIP(ctx, hipGetLastError());
        DevBuf &bt = ctx->scratch[S_BUF_TMP];
        size_t tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)(G + 1), st));
        if (ensure(ctx, bt, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(bt.p, tb, cnt, off, (int)(G + 1), st));
        SPADE_HIP(ctx, hipMemcpyAsync(h, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        if (h[0] >= ((unsigned long long)1 << 26))
            return set_error(ctx, SPADE_E_TOO_LARGE, "too many (segment, cell) entries: the distances are too "
                                                     "large for the segments' spread");
        const int64_t total = (int64_t)h[0];
        // cell lists: sort keys and values, sorted copies of the segments
        DevBuf &bl = ctx->scratch[S_BUF_LIST];
        const size_t keyb = sizeof(unsigned long long) * (size_t)std::max<int64_t>(total, 1);
        const size_t valb = sizeof(uint32_t) * (size_t)std::max<int64_t>(total, 1);
        const size_t listb = sizeof(JSeg) * (size_t)std::max<int64_t>(total, 1);
        if (ensure(ctx, bl, 2 * keyb + 2 * valb + listb + 64)) return SPADE_E_NOMEM;
        unsigned long long *k1 = (unsigned long long *)bl.p, *k2 = k1 + std::max<int64_t>(total, 1);
        uint32_t *v1 = (uint32_t *)(k2 + std::max<int64_t>(total, 1)), *v2 = v1 + std::max<int64_t>(total, 1);
        list = (JSeg *)(((uintptr_t)(v2 + std::max<int64_t>(total, 1)) + 15) & ~(uintptr_t)15);
        SPADE_HIP(ctx, hipMemsetAsync(cursor, 0, sizeof(uint32_t) * (size_t)(G + 1), st));
        hipLaunchKernelGGL(k_bufj_bin<true>, dim3(bgrid), dim3(256), 0, st, V, (const JSeg *)segs,
                           (const uint8_t *)valid, grid, magpad, cursor, (const uint32_t *)off, k1, v1,
                           (unsigned long long *)nullptr);
        SPADE_HIP(ctx, hipGetLastError());
        if (total > 0) {
            int cb = 1;
            while (cb < 40 && ((uint64_t)(G - 1) >> cb) != 0) ++cb;
            size_t sb = 0;
            SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, sb, (const unsigned long long *)k1, k2,
                                                              (const uint32_t *)v1, v2, (int)total, 0, 32 + cb, st));
            if (ensure(ctx, bt, std::max<size_t>(sb, 1))) return SPADE_E_NOMEM;
            SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(bt.p, sb, (const unsigned long long *)k1, k2,
                                                              (const uint32_t *)v1, v2, (int)total, 0, 32 + cb, st));
            const int ggrid = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, (int64_t)cus * 8));
            hipLaunchKernelGGL(k_bufj_gather, dim3(ggrid), dim3(256), 0, st, (int64_t)total, (const uint32_t *)v2,
                               (const JSeg *)segs, list);
            SPADE_HIP(ctx, hipGetLastError());
        }
    }

    const int64_t nseg = (n + EMIT_SEG - 1) / EMIT_SEG;
    const int64_t wpb = BUF_THREADS / 64;
    const int gridp = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + wpb - 1) / wpb, (int64_t)cus * 2));
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (counting) {
        constexpr int HIST = 16384;
        const size_t lds = R <= HIST ? sizeof(uint32_t) * (size_t)std::max<int64_t>(R, 1) : 0;
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_bufj_pairs<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)std::max<size_t>(lds, 4)));
        hipLaunchKernelGGL(k_bufj_pairs<2>, dim3(gridp), dim3(BUF_THREADS), lds, st, n, pts->x, pts->y, grid,
                           (const uint32_t *)off, (const JSeg *)list, magpad, nseg, (unsigned long long *)nullptr,
                           (const unsigned long long *)nullptr, (uint32_t *)nullptr, (uint32_t *)nullptr, (int64_t)0,
                           (unsigned long long *)out_counts, (int)R, HIST, (uint32_t *)nullptr);
        SPADE_HIP(ctx, hipGetLastError());
        if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        return SPADE_OK;
    }
    DevBuf &lb = ctx->scratch[S_LOOKBACK];
    if (ensure(ctx, lb, sizeof(unsigned long long) * 2 * (size_t)(nseg + 1))) return SPADE_E_NOMEM;
    unsigned long long *counts = (unsigned long long *)lb.p;
    unsigned long long *offs = counts + (nseg + 1);
    // pairs per point, kept by the count pass for the write pass (without the
    // room, the write pass counts again)
    DevBuf &pb = ctx->scratch[S_BITS];
    uint32_t *pcount = nullptr;
    if (cap > 0) {
        if (ensure(ctx, pb, sizeof(uint32_t) * (size_t)n) == SPADE_OK) pcount = (uint32_t *)pb.p;
        else ctx->err.clear();
    }
    hipLaunchKernelGGL(k_bufj_pairs<0>, dim3(gridp), dim3(BUF_THREADS), 0, st, n, pts->x, pts->y, grid,
                       (const uint32_t *)off, (const JSeg *)list, magpad, nseg, counts,
                       (const unsigned long long *)nullptr, (uint32_t *)nullptr, (uint32_t *)nullptr, (int64_t)0,
                       (unsigned long long *)nullptr, (int)R, 0, pcount);
    hipLaunchKernelGGL(k_buf_zero, dim3(1), dim3(1), 0, st, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &bt = ctx->scratch[S_BUF_TMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, bt, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(bt.p, tb, counts, offs, (int)(nseg + 1), st));
    if (cap > 0) {
        hipLaunchKernelGGL(k_bufj_pairs<1>, dim3(gridp), dim3(BUF_THREADS), 0, st, n, pts->x, pts->y, grid,
                           (const uint32_t *)off, (const JSeg *)list, magpad, nseg, (unsigned long long *)nullptr,
                           (const unsigned long long *)offs, out_pt, out_line, cap, (unsigned long long *)nullptr,
                           (int)R, 0, pcount);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (n_out) *n_out = (int64_t)h[0];
    if ((int64_t)h[0] > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // namespace spade
