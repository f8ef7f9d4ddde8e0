// Canvas construction: polygons -> discrete canvas + boundary index.
//
// This is the paper's canvas creation for polygons (Sec. 4.2: polygons drawn
// into a pixel grid of object ids, boundary pixels found by conservative
// rasterisation of the boundary lines) and its boundary index (Sec. 4.3),
// re-designed for a compute GPU:
//   * no triangulation: a scanline rasteriser works on edge lists per pixel
//     row;
//   * conservative marking: every pixel whose square, dilated by MARGIN
//     pixels, meets an edge is a boundary pixel (the dilation absorbs the
//     rounding of the world->pixel map on both edges and points);
//   * the boundary index of a boundary pixel lists, per candidate polygon,
//     the edges needed for an exact crossing-number test of any point of the
//     pixel (local edges, partial edges to the right, parity of spanning
//     edges to the right) instead of one triangle per pixel, which is exact
//     for any number of edges in a pixel.
//
// Pipeline (all on the context's stream):
//   k_validate   offsets / finiteness checks, ring -> polygon map, bbox
//                (k_canvas_bbox: per-canvas boxes of a canvas set)
//   k_edges      one thread per vertex: edge record, pixel row range
//   scan         edge -> first (edge,row) entry
//   k_entries    one (edge,row) entry per row an edge touches: footprint
//                columns [c0,c1], spanning flag, parity weight at the row centre
//   radix sort   entries by (row, polygon, c0)
//   k_gather     sorted payload, row -> first entry
//   k_rows<1>    per row, in LDS: write canvas words, records, edge ids into
//                ranges reserved with atomics (k_rows<0> + scans + k_rows<1>
//                with exact sizes when the reserved capacity runs out)
//   k_compact    coarse level over the canvas words
#include "common.h"
#include "exact.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace spade {

constexpr double MARGIN = 1.0 / 4096.0;       // pixels
constexpr double SLOP = 1.0 / 1073741824.0;   // pixels, covers clipping round-off
constexpr int MAXW = 8192;
constexpr int ROW_THREADS = 256;
constexpr int ROW_THREADS_MAX = 512;
constexpr size_t ROW_LDS_PER_CU = 160 * 1024;   // LDS of one CU
constexpr int RED_BLOCKS = 256;

constexpr uint8_t F_SPAN = 1;    // edge spans the whole dilated row band
constexpr uint8_t F_W = 2;       // edge straddles the row-centre line
constexpr uint8_t F_HORIZ = 4;   // horizontal edge (never crosses)

// Canvas of polygon k: canvases own contiguous polygon ranges.
__device__ __forceinline__ int canvas_of_poly(const CanvasDesc *cds, int nc, int64_t k)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cds[mid].poly_base <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Canvas holding global row r (rows of all canvases are concatenated).
__device__ __forceinline__ int canvas_of_row(const CanvasDesc *cds, int nc, int64_t r)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cds[mid].row_base <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Order-preserving map of a double to an unsigned integer (for atomic min/max).
__device__ __forceinline__ unsigned long long dkey(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// ------------------------------------------------------------ validation

// Clears the build's flags and counters in one launch: error flags, the
// per-canvas box keys (to the maximum key), the row-pass counters.
// Output ranges of the single row pass come from NSHARD independent
// allocators (row r uses allocator r mod NSHARD, each owning an equal slice
// of every output array), each counter on a cache line of its own, so that
// the rows' reservations do not queue on one address.
constexpr int NSHARD = 16;
constexpr int GSTRIDE = 16;                        // words between counters
constexpr int NGCTR = NSHARD * 4 * GSTRIDE;        // counter block, 8 KB
__host__ __device__ inline int gctr_at(int shard, int c) { return (shard * 4 + c) * GSTRIDE; }

__global__ void k_init(unsigned *errflags, unsigned long long *bb, int64_t nbb, unsigned long long *gctr)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) *errflags = 0u;
    for (int64_t i = tid; i < NGCTR; i += nth) gctr[i] = 0ull;
    for (int64_t i = tid; i < nbb; i += nth) bb[i] = ~0ull;
}

__global__ __launch_bounds__(256) void k_validate(int64_t M, int64_t R, const int64_t *pro,
                                                  const int64_t *rvo, int64_t V, const double *vx,
                                                  const double *vy, int32_t *ring_poly,
                                                  double *blockred, unsigned *errflags,
                                                  unsigned long long *bb)
{
    // (per-canvas boxes are computed by k_canvas_bbox once ring_poly is known)
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    // the vertex arrays hold ring_vtx_off[R] entries: never read past them,
    // whatever the caller's count says (a mismatch is reported)
    const int64_t Vend = rvo[R];
    if (tid == 0 && Vend != V) atomicOr(errflags, 64u);
    V = min(V, Vend);
    for (int64_t k = tid; k < M; k += nth) {
        int64_t r0 = pro ? pro[k] : k, r1 = pro ? pro[k + 1] : k + 1;
        if (r0 < 0 || r1 < r0 || r1 > R) { atomicOr(errflags, 2u); continue; }
        for (int64_t r = r0; r < r1; ++r) ring_poly[r] = (int32_t)k;
    }
    if (tid == 0) {
        if (pro && (pro[0] != 0 || pro[M] != R)) atomicOr(errflags, 2u);
        if (rvo[0] != 0) atomicOr(errflags, 1u);
    }
    for (int64_t r = tid; r < R; r += nth)
        if (rvo[r + 1] < rvo[r]) atomicOr(errflags, 1u);

    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t v = tid; v < V; v += nth) {
        double x = vx[v], y = vy[v];
        if (!isfinite(x) || !isfinite(y)) { atomicOr(errflags, 4u); continue; }
        x0 = fmin(x0, x); x1 = fmax(x1, x);
        y0 = fmin(y0, y); y1 = fmax(y1, y);
    }
    __shared__ double s[4][256];
    s[0][threadIdx.x] = x0; s[1][threadIdx.x] = -x1;
    s[2][threadIdx.x] = y0; s[3][threadIdx.x] = -y1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = fmin(s[q][threadIdx.x], s[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) blockred[blockIdx.x * 4 + q] = s[q][0];
    // one canvas: its box is the box of all vertices (keys as in k_canvas_bbox)
    if (bb && threadIdx.x < 4) atomicMin(&bb[threadIdx.x], dkey(s[threadIdx.x][0]));
}

// Per-canvas bounding boxes: bb[4 q + 0..3] = keys of min x, -max x, min y,
// -max y over the vertices of canvas q's polygons (ordered-key atomics).
// Each thread reduces a run of BB_SPAN consecutive vertices, flushing when
// the canvas changes; a wave whose runs all end in one canvas merges them
// before its atomics, so one canvas of many vertices costs few atomics.
constexpr int BB_SPAN = 32;

__device__ __forceinline__ void bb_flush(unsigned long long *bb, int q, const unsigned long long k[4])
{
    atomicMin(&bb[4 * q + 0], k[0]);
    atomicMin(&bb[4 * q + 1], k[1]);
    atomicMin(&bb[4 * q + 2], k[2]);
    atomicMin(&bb[4 * q + 3], k[3]);
}

__global__ __launch_bounds__(256) void k_canvas_bbox(int64_t R, const int64_t *rvo, int64_t V,
                                                     const double *vx, const double *vy,
                                                     const int32_t *ring_poly, const CanvasDesc *cds,
                                                     int nc, unsigned long long *bb)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    V = min(V, rvo[R]);
    const int64_t nspan = (V + BB_SPAN - 1) / BB_SPAN;
    // every lane runs the same number of iterations (the wave merge below)
    const int64_t iters = (nspan + nth - 1) / nth;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t sp = it * nth + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        int q = -1;
        unsigned long long k[4] = {~0ull, ~0ull, ~0ull, ~0ull};
        if (sp < nspan) {
            const int64_t j0 = sp * BB_SPAN, j1 = min(V, j0 + BB_SPAN);
            int64_t lo = 0, hi = R;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (rvo[mid] <= j0) lo = mid; else hi = mid;
            }
            int64_t r = lo;
            q = canvas_of_poly(cds, nc, ring_poly[r]);
            for (int64_t j = j0; j < j1; ++j) {
                if (j >= rvo[r + 1]) {
                    while (j >= rvo[r + 1]) ++r;
                    const int qn = canvas_of_poly(cds, nc, ring_poly[r]);
                    if (qn != q) {
                        bb_flush(bb, q, k);
                        k[0] = k[1] = k[2] = k[3] = ~0ull;
                        q = qn;
                    }
                }
                const double x = vx[j], y = vy[j];
                k[0] = min(k[0], dkey(x)); k[1] = min(k[1], dkey(-x));
                k[2] = min(k[2], dkey(y)); k[3] = min(k[3], dkey(-y));
            }
        }
        const int q0 = __shfl(q, 0, 64);
        if (__all(q == q0 || q == -1) && q0 != -1) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                for (int d = 32; d > 0; d >>= 1) k[t] = min(k[t], (unsigned long long)__shfl_xor(k[t], d, 64));
            if ((threadIdx.x & 63) == 0) bb_flush(bb, q0, k);
        } else if (q != -1) {
            bb_flush(bb, q, k);
        }
    }
}

// ------------------------------------------------------------ edges

// Conservative footprint of an edge in pixel row r: the columns [c0, c1]
// its part inside the row band, dilated by MARGIN, can touch.  (ulo, vlo)
// and (uhi, vhi) are the edge's end points in pixel coordinates.
// inv_dv = 1 / (vhi - vlo), computed once per edge: the product differs
// from the quotient by a few units in the last place of t, far below SLOP.
__device__ __forceinline__ void row_footprint(const CanvasDesc &m, double ulo, double uhi, double vlo, double vhi,
                                              double inv_dv, int32_t r, int32_t &c0, int32_t &c1)
{
    const double b0 = (double)r - MARGIN, b1 = (double)r + 1.0 + MARGIN;
    double xa, xb;
    if (vlo == vhi) {
        xa = ulo; xb = uhi;
    } else {
        const double ta = fmin(1.0, fmax(0.0, (b0 - vlo) * inv_dv));
        const double tb = fmin(1.0, fmax(0.0, (b1 - vlo) * inv_dv));
        xa = ulo + ta * (uhi - ulo);
        xb = ulo + tb * (uhi - ulo);
    }
    const double xmn = fmin(xa, xb) - SLOP, xmx = fmax(xa, xb) + SLOP;
    c0 = (int32_t)fmax(0.0, fmin(floor(xmn - MARGIN), (double)(m.W - 1)));
    c1 = (int32_t)fmax(0.0, fmin(floor(xmx + MARGIN), (double)(m.W - 1)));
}

constexpr int ROW_WIN = 4096;   // rows of a workgroup's LDS row window
constexpr int LANE_ROWS_W = 16; // rows an edge's own lane walks; longer edges are walked by the wave

// Calls fn(row) for every row of the (edge, row) entries of this thread's
// edge (rows g0 .. g0 + nr - 1); edges of more than LANE_ROWS_W rows are
// walked by their whole wave.
template <typename Fn>
__device__ __forceinline__ void for_entry_rows(int64_t g0, int nr, Fn fn)
{
    const int lane = threadIdx.x & 63;
    if (nr > 0 && nr <= LANE_ROWS_W)
        for (int t = 0; t < nr; ++t) fn(g0 + t);
    unsigned long long longs = __ballot(nr > LANE_ROWS_W);
    while (longs) {
        const int src = __ffsll((long long)longs) - 1;
        longs &= longs - 1;
        const int64_t gg = __shfl(g0, src, 64);
        const int nn = __shfl(nr, src, 64);
        for (int t = lane; t < nn; t += 64) fn(gg + t);
    }
}

// Per-row entry counts of a workgroup's edges added to global counters
// (one every rstride words): counted in LDS over the rows the workgroup
// touches, then one global atomic per touched row.  Returns true with the
// counters' old values (each touched row's first slot for this workgroup)
// in hist[row - *s_lo].  When the rows span more than ROW_WIN it returns
// false having added nothing if `base`, per entry otherwise.  Every thread
// of the block calls it (barriers).
__device__ bool block_row_counts(int64_t g0, int nr, uint32_t *ctr, int rstride, uint32_t *hist,
                                 int *s_lo, int *s_hi, bool base)
{
    const int tid = threadIdx.x;
    if (tid == 0) { *s_lo = 0x7fffffff; *s_hi = -1; }
    __syncthreads();
    if (nr > 0) { atomicMin(s_lo, (int)g0); atomicMax(s_hi, (int)(g0 + nr - 1)); }
    __syncthreads();
    const int lo = *s_lo, n = *s_hi - *s_lo + 1;
    if (n > 0 && n <= ROW_WIN) {
        for (int k = tid; k < n; k += blockDim.x) hist[k] = 0u;
        __syncthreads();
        for_entry_rows(g0, nr, [&](int64_t g) { atomicAdd(&hist[g - lo], 1u); });
        __syncthreads();
        for (int k = tid; k < n; k += blockDim.x) {
            const uint32_t c = hist[k];
            if (c) {
                const uint32_t old = atomicAdd(&ctr[(int64_t)(lo + k) * rstride], c);
                if (base) hist[k] = old;
            }
        }
        __syncthreads();
        return true;
    }
    if (n > 0 && !base) for_entry_rows(g0, nr, [&](int64_t g) { atomicAdd(&ctr[g * rstride], 1u); });
    __syncthreads();
    return false;
}

__device__ __forceinline__ double undkey(unsigned long long k)
{
    const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Edges, their canvas rows and the row histogram.  With `guard` (a canvas
// sized from the caller's bounding box before the validation was read), the
// kernel first checks the validation flags and that the vertices' box lies
// inside the given one; otherwise it flags 128 and emits no entries, so
// nothing downstream reads the polygon arrays.
__global__ __launch_bounds__(256) void k_edges(int64_t R, const int64_t *rvo, int64_t V,
                                               const double *vx, const double *vy,
                                               const int32_t *ring_poly, const CanvasDesc *cds, int nc,
                                               Edge *edges, uint32_t *epoly, int32_t *erow0,
                                               uint64_t *nrows, uint32_t *rcount, int rstride, int guard,
                                               unsigned *errflags, const unsigned long long *bbk,
                                               double hx0, double hx1, double hy0, double hy1)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) nrows[V] = 0;   // zero tail of the row-count scan
    if (guard) {
        __shared__ int s_ok;
        if (threadIdx.x == 0) {
            const unsigned f = __hip_atomic_load(errflags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool ok = !(f & (1u | 2u | 4u | 64u));
            if (ok && V > 0) {
                const double x0 = undkey(bbk[0]), x1 = -undkey(bbk[1]);
                const double y0 = undkey(bbk[2]), y1 = -undkey(bbk[3]);
                ok = x0 >= hx0 && x1 <= hx1 && y0 >= hy0 && y1 <= hy1;
                if (!ok && blockIdx.x == 0) atomicOr(errflags, 128u);
            }
            s_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (!s_ok) {
            for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < V; j += nth) {
                nrows[j] = 0;
                erow0[j] = 0;
            }
            return;   // (every block returns: the verdict is the same for all)
        }
    }
    __shared__ uint32_t hist[ROW_WIN];
    __shared__ int s_lo, s_hi;
    // one edge per even lane: twice the waves for the latency-bound work
    const int64_t per = nth >> 1;
    const int64_t iters = (V + per - 1) / per;   // the same for every thread (block barriers)
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t j = (threadIdx.x & 1) ? V : it * per + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1);
        int64_t g0 = 0;
        int nr = 0;
        if (j < V) {
            // ring of vertex j: rvo[r] <= j < rvo[r+1]
            int64_t lo = 0, hi = R;
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) >> 1;
                if (rvo[mid] <= j) lo = mid; else hi = mid;
            }
            const int64_t r = lo;
            const int64_t nx = (j + 1 < rvo[r + 1]) ? j + 1 : rvo[r];
            double ax = vx[j], ay = vy[j], bx = vx[nx], by = vy[nx];
            epoly[j] = (uint32_t)ring_poly[r];
            const CanvasDesc &m = cds[canvas_of_poly(cds, nc, ring_poly[r])];
            Edge e;
            if (ay <= by) { e.xlo = ax; e.ylo = ay; e.xhi = bx; e.yhi = by; }
            else          { e.xlo = bx; e.ylo = by; e.xhi = ax; e.yhi = ay; }
            edges[j] = e;
            if ((ax == bx && ay == by) || m.empty) {   // zero length
                nrows[j] = 0;
                erow0[j] = 0;
            } else {
                double vlo = __dmul_rn(__dsub_rn(e.ylo, m.Y0), m.sy);
                double vhi = __dmul_rn(__dsub_rn(e.yhi, m.Y0), m.sy);
                double f0 = floor(vlo - MARGIN), f1 = floor(vhi + MARGIN);
                int32_t r0 = (int32_t)fmax(0.0, fmin(f0, (double)(m.H - 1)));
                int32_t r1 = (int32_t)fmax(0.0, fmin(f1, (double)(m.H - 1)));
                erow0[j] = r0;
                nrows[j] = (uint64_t)(r1 - r0 + 1);
                g0 = m.row_base + r0;
                nr = r1 - r0 + 1;
            }
        }
        // one entry per row r0..r1: counted per row of the block's window
        // in LDS, then one global atomic per row the block touches
        (void)block_row_counts(g0, nr, rcount, rstride, hist, &s_lo, &s_hi, false);
    }
}

__global__ void k_zero_u32(int64_t n, uint32_t *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ------------------------------------------------------------ row buckets

constexpr int SCAN_THREADS = 1024;

// Exclusive prefix sum over the block of one value per thread.
__device__ long long block_excl_sum(long long v, long long *wtot)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    long long inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    long long pre = 0;
    for (int q = 0; q < wv; ++q) pre += wtot[q];
    __syncthreads();
    return pre + inc - v;
}

// One block: from the per-row entry counts (one word every `rstride`, so
// that the edges' atomics spread over cache lines) the row offsets
// (row_off[Htot] = total), insertion cursors starting at the offsets (same
// stride), and two row lists: rows with more than capA and at most capB
// entries (longrows[0..)), rows with more than capB entries
// (longrows[Htot..)).
// info = {total entries, longest row, rows of the first list, of the second}.
__global__ __launch_bounds__(SCAN_THREADS) void k_rowscan(int64_t Htot, const uint32_t *rcount, int rstride,
                                                          int capA, int capB, uint32_t *row_off,
                                                          uint32_t *cursor, uint32_t *longrows,
                                                          unsigned long long *info)
{
    __shared__ long long wtot[SCAN_THREADS / 64];
    __shared__ unsigned s_nb, s_nc;
    __shared__ int s_max;
    const int tid = threadIdx.x;
    if (tid == 0) { s_nb = 0; s_nc = 0; s_max = 0; }
    const int64_t per = (Htot + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b = min(Htot, (int64_t)tid * per), e = min(Htot, b + per);
    // up to RS_REG counts per thread are loaded together and kept in
    // registers for the second pass (one memory round trip instead of one
    // per row and pass)
    constexpr int RS_REG = 8;
    uint32_t rc[RS_REG];
    const bool inreg = per <= RS_REG;
    long long tot = 0;
    if (inreg) {
#pragma unroll
        for (int k = 0; k < RS_REG; ++k) rc[k] = b + k < e ? rcount[(b + k) * rstride] : 0u;
#pragma unroll
        for (int k = 0; k < RS_REG; ++k) tot += rc[k];
    } else {
        for (int64_t r = b; r < e; ++r) tot += rcount[r * rstride];
    }
    long long off = block_excl_sum(tot, wtot);
    int mx = 0;
    auto visit = [&](int64_t r, long long cnt) {
        row_off[r] = (uint32_t)off;
        cursor[r * rstride] = (uint32_t)off;
        off += cnt;
        mx = max(mx, (int)min(cnt, (long long)0x7fffffff));
        if (cnt > capB) longrows[Htot + atomicAdd(&s_nc, 1u)] = (uint32_t)r;
        else if (cnt > capA) longrows[atomicAdd(&s_nb, 1u)] = (uint32_t)r;
    };
    if (inreg) {
#pragma unroll
        for (int k = 0; k < RS_REG; ++k)
            if (b + k < e) visit(b + k, rc[k]);
    } else {
        for (int64_t r = b; r < e; ++r) visit(r, rcount[r * rstride]);
    }
    atomicMax(&s_max, mx);
    __syncthreads();
    if (tid == SCAN_THREADS - 1) {
        row_off[Htot] = (uint32_t)off;
        info[0] = (unsigned long long)off;
        info[1] = (unsigned long long)s_max;
        info[2] = s_nb;
        info[3] = s_nc;
    }
}

// ------------------------------------------------------------ (edge,row) entries

// One entry per (edge, row): footprint, flags, sort key, edge id and the
// identity permutation.  Edges spanning few rows are expanded by their own
// lane; an edge spanning many rows (a long vertical boundary) is expanded by
// its whole wave, so no lane walks thousands of rows alone.
constexpr uint64_t LANE_ROWS = 16;

__global__ __launch_bounds__(256) void k_entries(int64_t V, const Edge *edges, const uint32_t *epoly,
                                                 const int32_t *erow0, const uint64_t *nrows,
                                                 const uint64_t *off, const CanvasDesc *cds, int nc,
                                                 int cbits, int pbits,
                                                 uint64_t *keys, uint32_t *vals, uint32_t *ent_c,
                                                 uint8_t *ent_f, uint32_t *perm)
{
    const int lane = threadIdx.x & 63;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    auto expand = [&](int64_t j, uint64_t t0, uint64_t dt, uint64_t nr) {
        const Edge e = edges[j];
        const bool horiz = (e.ylo == e.yhi);
        const CanvasDesc &m = cds[canvas_of_poly(cds, nc, epoly[j])];
        const double ulo = __dmul_rn(__dsub_rn(e.xlo, m.X0), m.sx);
        const double uhi = __dmul_rn(__dsub_rn(e.xhi, m.X0), m.sx);
        const double vlo = __dmul_rn(__dsub_rn(e.ylo, m.Y0), m.sy);
        const double vhi = __dmul_rn(__dsub_rn(e.yhi, m.Y0), m.sy);
        const double inv = vhi > vlo ? 1.0 / (vhi - vlo) : 0.0;
        const uint64_t poly = (uint64_t)((int64_t)epoly[j] - m.poly_base);
        const uint64_t base = off[j];
        for (uint64_t t = t0; t < nr; t += dt) {
            const int32_t r = erow0[j] + (int32_t)t;
            const double b0 = (double)r - MARGIN, b1 = (double)r + 1.0 + MARGIN;
            int32_t c0, c1;
            row_footprint(m, ulo, uhi, vlo, vhi, inv, r, c0, c1);
            const bool span = !horiz && vlo <= b0 && vhi >= b1;
            const double yc = m.Y0 + ((double)r + 0.5) * m.hy;
            const bool w = !horiz && straddles(e.ylo, e.yhi, yc);
            const uint64_t idx = base + t;
            keys[idx] = ((uint64_t)(m.row_base + r) << (pbits + cbits)) | (poly << cbits) | (uint64_t)c0;
            vals[idx] = (uint32_t)j;
            perm[idx] = (uint32_t)idx;
            ent_c[idx] = (uint32_t)c0 | ((uint32_t)c1 << 16);
            ent_f[idx] = (span ? F_SPAN : 0) | (w ? F_W : 0) | (horiz ? F_HORIZ : 0);
        }
    };
    // every lane runs the same number of iterations (the wave steps below)
    const int64_t iters = (V + nth - 1) / nth;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t j = it * nth + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const uint64_t nr = j < V ? nrows[j] : 0;
        if (nr > 0 && nr <= LANE_ROWS) expand(j, 0, 1, nr);
        unsigned long long longs = __ballot(nr > LANE_ROWS);
        while (longs) {
            const int src = __ffsll((long long)longs) - 1;
            longs &= longs - 1;
            const int64_t jj = __shfl(j, src, 64);
            const uint64_t nn = __shfl(nr, src, 64);
            expand(jj, (uint64_t)lane, 64, nn);
        }
    }
}

// Entries written straight into their row's bucket with the key
// (polygon, first column, edge id) that orders them inside the row.  A
// workgroup reserves, per row it touches, one range of slots with one
// global atomic on the row's cursor and hands them out from LDS (so the
// order inside a row is arbitrary until the row sort).
__global__ __launch_bounds__(256) void k_entries_rows(int64_t V, const Edge *edges, const uint32_t *epoly,
                                                      const int32_t *erow0, const uint64_t *nrows,
                                                      const CanvasDesc *cds, int nc, int ebits,
                                                      int ckshift, uint32_t *cursor, int rstride,
                                                      uint64_t *ukey, uint32_t *uc, uint8_t *uf,
                                                      const unsigned long long *tinfo, uint64_t tcap)
{
    // launched before the host has read the entry total: buffers hold tcap
    // entries, and a larger total leaves everything to a later launch
    if (tinfo && tinfo[0] > tcap) return;
    __shared__ uint32_t hist[ROW_WIN];
    __shared__ int s_lo, s_hi;
    const int lane = threadIdx.x & 63;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    auto entry = [&](int64_t j, const CanvasDesc &m, double ulo, double uhi, double vlo, double vhi,
                     double inv, bool horiz, const Edge &e, uint64_t poly, int32_t r, uint32_t pos) {
        const double b0 = (double)r - MARGIN, b1 = (double)r + 1.0 + MARGIN;
        int32_t c0, c1;
        row_footprint(m, ulo, uhi, vlo, vhi, inv, r, c0, c1);
        const bool span = !horiz && vlo <= b0 && vhi >= b1;
        const double yc = m.Y0 + ((double)r + 0.5) * m.hy;
        const bool w = !horiz && straddles(e.ylo, e.yhi, yc);
        ukey[pos] = (poly << ckshift) | ((uint64_t)c0 << ebits) | (uint64_t)j;
        uc[pos] = (uint32_t)c0 | ((uint32_t)c1 << 16);
        uf[pos] = (span ? F_SPAN : 0) | (w ? F_W : 0) | (horiz ? F_HORIZ : 0);
    };
    // one edge per fourth lane: four times the waves, a quarter of the
    // entries per wave
    const int64_t per = nth >> 2;
    const int64_t iters = (V + per - 1) / per;   // the same for every thread (block barriers)
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t j = (lane & 3) ? V : it * per + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2);
        const int nr = j < V ? (int)nrows[j] : 0;
        int64_t g0 = 0;
        int q = 0;
        if (nr > 0) {
            q = canvas_of_poly(cds, nc, epoly[j]);
            g0 = cds[q].row_base + erow0[j];
        }
        const bool win = block_row_counts(g0, nr, cursor, rstride, hist, &s_lo, &s_hi, true);
        const int lo = s_lo;
        auto slot = [&](int64_t g) -> uint32_t {
            return win ? atomicAdd(&hist[g - lo], 1u) : atomicAdd(&cursor[g * rstride], 1u);
        };
        // the wave's entries spread evenly over its lanes: entry k of the
        // wave belongs to the lane whose inclusive row-count prefix first
        // exceeds k (found by a binary search over the lanes)
        int incl = nr;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(incl, d, 64);
            if (lane >= d) incl += t;
        }
        const int E = __shfl(incl, 63, 64);
        for (int k = lane; k - lane < E; k += 64) {
            int src = 0;
#pragma unroll
            for (int b = 32; b > 0; b >>= 1) {
                const int probe = __shfl(incl, src + b - 1, 64);
                if (probe <= k) src += b;
            }
            const int before = __shfl(incl, src, 64) - __shfl(nr, src, 64);
            const int64_t jj = __shfl(j, src, 64);
            const int qq = __shfl(q, src, 64);
            if (k >= E) continue;
            const int t = k - before;
            const Edge e = edges[jj];
            const CanvasDesc &m = cds[qq];
            const bool horiz = (e.ylo == e.yhi);
            const double ulo = __dmul_rn(__dsub_rn(e.xlo, m.X0), m.sx);
            const double uhi = __dmul_rn(__dsub_rn(e.xhi, m.X0), m.sx);
            const double vlo = __dmul_rn(__dsub_rn(e.ylo, m.Y0), m.sy);
            const double vhi = __dmul_rn(__dsub_rn(e.yhi, m.Y0), m.sy);
            const double inv = vhi > vlo ? 1.0 / (vhi - vlo) : 0.0;
            const uint64_t poly = (uint64_t)((int64_t)epoly[jj] - m.poly_base);
            const int32_t r = erow0[jj] + t;
            entry(jj, m, ulo, uhi, vlo, vhi, inv, horiz, e, poly, r, slot(m.row_base + r));
        }
        __syncthreads();   // the window's slots are handed out before the next round
    }
}

// Longest row the in-row sort takes (its keys twice in LDS).
constexpr int ROWSORT_MAX = 4096;
constexpr int SORT_THREADS = 1024;
constexpr int SORT_CHUNKS = ROWSORT_MAX / SORT_THREADS;

// Sorts every row's entries by key and writes them in that order: polygon
// and edge from the key, footprint and flags from the source slot.  Keys
// are unique.  The row is cut into chunks of one key per thread; a key's
// rank in its chunk is the count of smaller keys there (the chunk is then
// stored sorted), and its rank in the row adds, for every other chunk, the
// count of smaller keys found by binary search.  The listed long rows
// (nB + nC of them, with more than `cap` entries) come first, so that the
// longest sorts do not start last.
__global__ __launch_bounds__(SORT_THREADS) void k_rowsort(int64_t Htot, const uint32_t *row_off,
                                                          const uint64_t *ukey, const uint32_t *uc,
                                                          const uint8_t *uf, int pshift, uint64_t emask,
                                                          uint32_t *s_poly, uint32_t *s_edge, uint32_t *s_c,
                                                          uint8_t *s_f, int pmax, const uint32_t *longrows,
                                                          int64_t nB, int64_t nC, int cap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *kk = (uint64_t *)smem;      // keys in bucket order
    uint64_t *sk = kk + pmax;             // keys, each chunk sorted
    const int tid = threadIdx.x;
    const int64_t items = nC + nB + Htot;
    for (int64_t k = blockIdx.x; k < items; k += gridDim.x) {
        const int64_t r = k < nC ? (int64_t)longrows[Htot + k] : k < nC + nB ? (int64_t)longrows[k - nC] : k - nC - nB;
        const uint32_t s = row_off[r];
        const int n = (int)(row_off[r + 1] - s);
        if (n == 0 || (k >= nC + nB && n > cap)) continue;
        const int C = (n + SORT_THREADS - 1) / SORT_THREADS;
        for (int i = tid; i < n; i += SORT_THREADS) kk[i] = ukey[s + i];
        __syncthreads();
        int lr[SORT_CHUNKS];
#pragma unroll
        for (int c = 0; c < SORT_CHUNKS; ++c) {
            const int i = c * SORT_THREADS + tid;
            lr[c] = 0;
            if (c < C && i < n) {
                const uint64_t x = kk[i];
                const int cb = c * SORT_THREADS, ce = min(n, cb + SORT_THREADS);
                int rank = 0;
#pragma unroll 8
                for (int q = cb; q < ce; ++q) rank += (kk[q] < x) ? 1 : 0;
                lr[c] = rank;
                sk[cb + rank] = x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < SORT_CHUNKS; ++c) {
            const int i = c * SORT_THREADS + tid;
            if (c < C && i < n) {
                const uint64_t x = kk[i];
                int g = lr[c];
                for (int o = 0; o < C; ++o) {
                    if (o == c) continue;
                    int lo = o * SORT_THREADS, hi = min(n, lo + SORT_THREADS);   // at most 1024 keys
                    const int b = lo;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (sk[mid] < x) lo = mid + 1; else hi = mid;
                    }
                    g += lo - b;
                }
                s_poly[s + g] = (uint32_t)(x >> pshift);
                s_edge[s + g] = (uint32_t)(x & emask);
                s_c[s + g] = uc[s + i];
                s_f[s + g] = uf[s + i];
            }
        }
        __syncthreads();
    }
}

// After the sort: per sorted entry, its footprint, flags, polygon and edge
// id in sorted order, and the first entry of every row (rows between the
// previous entry's row and this one's start here).
__global__ void k_gather(int64_t T, const uint32_t *perm, const uint32_t *ent_c, const uint8_t *ent_f,
                         const uint32_t *vals, const uint64_t *skeys, int cbits, uint64_t pmask, int rshift,
                         int64_t H, uint32_t *s_c, uint8_t *s_f, uint32_t *s_poly, uint32_t *s_edge,
                         uint32_t *row_off)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= T; i += nth) {
        if (i < T) {
            const uint32_t p = perm[i];
            s_c[i] = ent_c[p];
            s_f[i] = ent_f[p];
            s_edge[i] = vals[p];
            s_poly[i] = (uint32_t)((skeys[i] >> cbits) & pmask);
        }
        const int64_t ri = (i < T) ? (int64_t)(skeys[i] >> rshift) : H;
        const int64_t rp = (i == 0) ? -1 : (int64_t)(skeys[i - 1] >> rshift);
        for (int64_t rr = rp + 1; rr <= ri; ++rr) row_off[rr] = (uint32_t)i;
    }
}

// ------------------------------------------------------------ per-row scanline

// Column arrays of a row live in LDS with one pad word per 32 so that the
// contiguous per-thread chunks of the scans do not collide in LDS banks.
__device__ __forceinline__ int cix(int c) { return c + (c >> 5); }
__host__ __device__ inline int col_words(int W) { return W + 1 + (W + 1) / 32 + 1; }

// Threads of a row workgroup: ROW_THREADS, or ROW_THREADS_MAX where the
// row stage leaves room for at most two workgroups per CU.
__device__ __forceinline__ int row_threads() { return (int)blockDim.x; }

// Block-wide in-place inclusive scan of a[cix(0..n)) with row_threads()
// threads: contiguous per-thread chunks, wave-level shuffle scan of the
// chunk totals, one LDS word per wave.  `op` must be associative and
// commutative.
template <typename T, typename Op>
__device__ void block_scan(T *a, int n, T *wtot, Op op, T ident)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + row_threads() - 1) / row_threads();
    const int b = min(n, tid * per), e = min(n, b + per);
    T acc = ident;
    for (int i = b; i < e; ++i) acc = op(acc, a[cix(i)]);   // chunk total: loads only
    T inc = acc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(inc, d, 64);
        if (lane >= d) inc = op(inc, t);
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    T pre = ident;
    for (int q = 0; q < wv; ++q) pre = op(pre, wtot[q]);
    T prev = __shfl_up(inc, 1, 64);
    if (lane > 0) pre = op(pre, prev);
    for (int i = b; i < e; ++i) { pre = op(pre, a[cix(i)]); a[cix(i)] = pre; }
    __syncthreads();
}

struct RowArgs {
    const CanvasDesc *cds;   // canvases of the set
    int nc;
    int maxW;                // widest canvas (LDS column arrays)
    int cls16;              // pixel classes in 16 bits (every canvas has < 2^15 polygons)
    int64_t Htot;            // rows of all canvases
    int cap;                 // entries of one row staged in LDS
    const uint32_t *row_off;
    const uint32_t *spoly;   // polygon per sorted entry
    const uint32_t *sedge;   // edge id per sorted entry
    const uint32_t *sc;      // c0 | c1 << 16
    const uint8_t *sf;
    const Edge *edges;
    uint32_t *gaux;          // 6 words per entry for rows too long to stage
    int min_n;               // this launch handles rows with min_n <= entries (<= max_n)
    int max_n;
    const uint32_t *rows;    // rows of this launch (nullptr: all rows)
    int64_t nlist;
    const uint32_t *first;   // with rows == nullptr: nfirst rows taken before all others,
    int64_t nfirst;          // which then skip those of more than `cap` entries
    // single-pass allocation: per-row output ranges reserved with atomics
    int alloc;
    unsigned long long *gctr;    // per shard: records, local edges, partial spans, boundary pixels
    unsigned long long cap_rec, cap_loc, cap_part;   // per shard
    // count pass
    uint64_t *row_nrec, *row_nloc, *row_npart, *row_nbp;
    // emit pass
    const uint64_t *rec_base, *loc_base, *part_base;
    uint32_t *cells;
    Cand *cands;
    Edge *ledges;
    double2 *pspan;
    unsigned *errflags;
};

// Entries of one row, relative to its first entry, with their per-row
// auxiliary arrays (LDS when the row is staged, global memory otherwise).
struct RowData {
    const uint32_t *poly;
    const uint32_t *c;
    const uint8_t *f;
    const uint32_t *edge;
    uint32_t *pm;     // running max over the run up to q of (c1 + 1): low 16 bits all
                      // entries, high 16 bits non-horizontal entries (0: none)
    uint32_t *pre;    // inclusive row prefix: partial count (bits 0..30, sum) and
                      // spanning parity (bit 31, xor)
    uint32_t *ihead;  // footprint-union intervals of the runs: run start, run end,
    uint32_t *iend;   // first column, inclusive prefix of interval lengths
    uint32_t *icol;
    uint32_t *ilen;
    int n;
};

// Row-level LDS state shared by the run workers.
struct RowShared {
    int32_t *sa;        // footprint counts -> per-column record counts / bases
    int32_t *sb;        // claim counts -> per-column fill counters
    void *sx;           // claimant xor -> pixel class (16 or 32 bits per column)
    uint32_t *locfill;  // row-local fill counter of the local-edge array
    uint32_t *nint;     // number of footprint-union intervals of the row
    uint32_t *nlong;    // long runs deferred to whole waves, and their starts
    uint32_t *longq;
    const unsigned long long *nrec;   // records of the row (set by the count phase)
    int W;              // width of the row's canvas
    bool cls16;        // sx in 16 bits: labels + 1 below 2^15, boundary flag in bit 15

    __device__ __forceinline__ uint32_t sx_flag() const { return cls16 ? 0x8000u : BFLAG; }
    __device__ __forceinline__ uint32_t sx_get(int e) const
    {
        return cls16 ? (uint32_t)((const uint16_t *)sx)[e] : ((const uint32_t *)sx)[e];
    }
    __device__ __forceinline__ void sx_set(int e, uint32_t v) const
    {
        if (cls16) ((uint16_t *)sx)[e] = (uint16_t)v;
        else ((uint32_t *)sx)[e] = v;
    }
    // xor into element e (two 16-bit elements share an LDS word)
    __device__ __forceinline__ void sx_xor(int e, uint32_t v) const
    {
        if (cls16) atomicXor((uint32_t *)sx + (e >> 1), v << ((e & 1) * 16));
        else atomicXor((uint32_t *)sx + e, v);
    }
};

// Runs longer than this are processed by a whole wave (lane-parallel scans)
// instead of one thread; up to LONGQ of them per row, the rest serially.
constexpr int LONG_RUN = 8;
constexpr int LONGQ = 128;

__device__ __forceinline__ size_t tile_index(int Wt, int c, int r)
{
    return ((size_t)(r >> 4) * Wt + (c >> 4)) * 256 + ((r & 15) << 4) + (c & 15);
}

__device__ __forceinline__ bool is_partial(uint8_t f) { return !(f & F_SPAN) && !(f & F_HORIZ); }
__device__ __forceinline__ bool is_spanning(uint8_t f) { return (f & F_SPAN) && !(f & F_HORIZ); }

__device__ __forceinline__ uint32_t pre_own(uint8_t f)
{
    return (is_partial(f) ? 1u : 0u) | (is_spanning(f) ? 0x80000000u : 0u);
}

// Combines two prefix words: 31-bit sum of partial counts, xor of parities.
__device__ __forceinline__ uint32_t pre_op(uint32_t a, uint32_t b)
{
    return ((a + b) & 0x7fffffffu) | ((a ^ b) & 0x80000000u);
}

// Exclusive row prefix at q (q may be n).
__device__ __forceinline__ uint32_t pre_excl(const RowData &D, int q)
{
    return q == 0 ? 0u : D.pre[q - 1];
}

// Slot of a new record of column col (sa holds the inclusive prefix of the
// row's per-column record counts, sb the fill counters), and CAND_LAST when
// it takes the column's last slot.  A pixel's records are in no particular
// polygon order; the probes order their matches where order matters.
__device__ __forceinline__ uint64_t rec_slot(const RowShared &L, int col, uint64_t rec_base_r, uint32_t &last)
{
    const int32_t k = atomicAdd(&L.sb[cix(col)], 1);
    const int32_t b = col ? L.sa[cix(col - 1)] : 0;
    const int32_t e = L.sa[cix(col)];
    last = (k == e - b - 1) ? CAND_LAST : 0u;
    return rec_base_r + (uint64_t)b + (uint64_t)k;
}

// Records of one run at one column.  A point p of the pixel is inside the
// run's polygon iff  S ^ XOR(partial-right straddles) ^ XOR(local crosses),
// with S the parity of the run's spanning entries starting right of col,
// partial-right entries those partial entries starting right of col, and
// local entries the non-horizontal entries whose footprint contains col.
template <bool EMIT>
__device__ __forceinline__ void column_record(const RowArgs &A, const RowData &D, const RowShared &L,
                                              int i, int je, int col, uint64_t rec_base_r,
                                              uint64_t loc_base_r, uint64_t part_base_r,
                                              uint64_t &nloc_tot)
{
    // sp: first entry of the run whose footprint starts right of col
    int lo = i, hi = je;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)(D.c[mid] & 0xffff) <= col) lo = mid + 1; else hi = mid;
    }
    const int sp = lo;
    if (sp == i || (int)(D.pm[sp - 1] & 0xffff) <= col) return;   // col outside the run's footprints
    const uint32_t pe = pre_excl(D, je), ps = pre_excl(D, sp);
    const uint32_t S = ((pe ^ ps) >> 31) & 1u;
    const uint32_t npart = (pe & 0x7fffffffu) - (ps & 0x7fffffffu);
    uint32_t nloc = 0;
    uint32_t id0 = 0, id1 = 0, id2 = 0, id3 = 0;   // the last four local edges met
    for (int q = sp - 1; q >= i && (int)(D.pm[q] >> 16) > col; --q)
        if ((int)(D.c[q] >> 16) >= col && !(D.f[q] & F_HORIZ)) {
            if (EMIT) { id3 = id2; id2 = id1; id1 = id0; id0 = D.edge[q]; }
            ++nloc;
        }
    if (nloc > 0x7fffu || npart > 0x7fffu) atomicOr(A.errflags, 16u);
    if (!EMIT) {
        atomicAdd(&L.sa[cix(col)], 1);
        nloc_tot += nloc ? nloc - 1 : 0;   // the first local edge lives in the record
        return;
    }
    uint32_t last;
    const uint64_t slot = rec_slot(L, col, rec_base_r, last);
    uint64_t eoff = 0;
    Cand cd{};
    // the record repeats its first partial-right range: that of the run's
    // first partial entry from sp on
    uint32_t pid = 0;
    if (npart) {
        int q = sp;
        while (!is_partial(D.f[q])) ++q;
        pid = D.edge[q];
    }
    if (nloc) {
        // the first local edge goes into the record, the others to the
        // local-edge array from eoff
        if (nloc > 1) eoff = loc_base_r + atomicAdd(L.locfill, nloc - 1);
        if (nloc <= 4) {
            // up to four edges: all loads in flight before the stores (a
            // pixel's local edges are tested in any order)
            const Edge e0 = A.edges[id0];
            const Edge e1 = A.edges[nloc > 1 ? id1 : id0];
            const Edge e2 = A.edges[nloc > 2 ? id2 : id0];
            const Edge e3 = A.edges[nloc > 3 ? id3 : id0];
            const Edge ep = A.edges[pid];
            if (nloc > 1) A.ledges[eoff] = e1;
            if (nloc > 2) A.ledges[eoff + 1] = e2;
            if (nloc > 3) A.ledges[eoff + 2] = e3;
            cd.e0 = e0;
            if (npart) cd.s0 = make_double2(ep.ylo, ep.yhi);
        } else {
            uint64_t o = eoff;
            bool first = true;
            for (int q = sp - 1; q >= i && (int)(D.pm[q] >> 16) > col; --q)
                if ((int)(D.c[q] >> 16) >= col && !(D.f[q] & F_HORIZ)) {
                    const Edge e = A.edges[D.edge[q]];
                    if (first) cd.e0 = e;
                    else A.ledges[o++] = e;
                    first = false;
                }
        }
    }
    if (npart && !(nloc && nloc <= 4)) {
        const Edge ep = A.edges[pid];
        cd.s0 = make_double2(ep.ylo, ep.yhi);
    }
    cd.poly = D.poly[i];
    cd.meta = S | last | ((nloc & 0x7fffu) << 2) | ((npart & 0x7fffu) << 17);
    cd.eoff = (uint32_t)eoff;
    cd.poff = (uint32_t)(part_base_r + (ps & 0x7fffffffu));
    A.cands[slot] = cd;
}

// Claimant records of a run in rows where interiors overlap: every boundary
// column inside the run's interior spans gets (S = 1, no edges).
template <bool EMIT>
__device__ void claimant_walk(const RowArgs &A, const RowData &D, const RowShared &L, int i, int je,
                              uint64_t rec_base_r, int W)
{
    uint32_t par = 0;
    for (int q = i; q < je; ++q) par ^= (D.f[q] & F_W) ? 1u : 0u;
    auto emit = [&](int col) {
        if (!EMIT) { atomicAdd(&L.sa[cix(col)], 1); return; }
        uint32_t last;
        const uint64_t slot = rec_slot(L, col, rec_base_r, last);
        Cand cd{};
        cd.poly = D.poly[i];
        cd.meta = CAND_S | last;
        cd.eoff = 0;
        cd.poff = 0;
        A.cands[slot] = cd;
    };
    int mx = -1;
    const int c0first = (int)(D.c[i] & 0xffff);
    if (par)
        for (int col = 0; col < c0first; ++col)
            if (L.sx_get(cix(col)) & L.sx_flag()) emit(col);
    for (int q = i; q < je; ++q) {
        const uint32_t c = D.c[q];
        mx = max(mx, (int)(c >> 16));
        if (D.f[q] & F_W) par ^= 1u;
        const int nc0 = (q + 1 < je) ? (int)(D.c[q + 1] & 0xffff) : W;
        const int lo = max((int)(c & 0xffff), mx + 1), hi = nc0 - 1;
        if (par)
            for (int col = lo; col <= hi; ++col)
                if (L.sx_get(cix(col)) & L.sx_flag()) emit(col);
    }
}

// Calls fn(i, je) for every run (maximal block of entries of one polygon)
// whose first entry this thread owns.
template <typename Fn>
__device__ __forceinline__ void for_each_run(const RowData &D, Fn fn)
{
    for (int i = threadIdx.x; i < D.n; i += row_threads()) {
        const uint32_t k = D.poly[i];
        if (i != 0 && D.poly[i - 1] == k) continue;
        int je = i + 1;
        while (je < D.n && D.poly[je] == k) ++je;
        fn(i, je);
    }
}

// The five inclusive scans of phase 2 in one pass: footprint counts (sum),
// claim counts (sum) and claimant xor over the row's columns, the per-entry
// partial/spanning prefix (pre_op) and the interval lengths (sum).  Each
// thread takes a contiguous chunk of every array: chunk totals first (loads
// only, so they overlap), wave scans of the five totals, one barrier, then
// the chunks rewritten from their running prefixes.  wt holds 5 words per
// wave.
__device__ void row_scans(const RowShared &L, int W, uint32_t *pre, int n, uint32_t *ilen, int ni, uint32_t *wt)
{
    int32_t *sa = L.sa, *sb = L.sb;
    const int NW = row_threads() >> 6;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int pc = (W + row_threads() - 1) / row_threads(), pp = (n + row_threads() - 1) / row_threads();
    const int pi = (ni + row_threads() - 1) / row_threads();
    const int cb = min(W, tid * pc), ce = min(W, cb + pc);
    const int qb = min(n, tid * pp), qe = min(n, qb + pp);
    const int ib = min(ni, tid * pi), ie = min(ni, ib + pi);
    uint32_t ta = 0, tb = 0, tx = 0, tp = 0, ti = 0;
    for (int c = cb; c < ce; ++c) {
        ta += (uint32_t)sa[cix(c)];
        tb += (uint32_t)sb[cix(c)];
        tx ^= L.sx_get(cix(c));
    }
    for (int q = qb; q < qe; ++q) tp = pre_op(tp, pre[q]);
    for (int q = ib; q < ie; ++q) ti += ilen[q];
    // inclusive wave scans of the chunk totals
    uint32_t ia = ta, ibb = tb, ix = tx, ip = tp, ii = ti;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t a = __shfl_up(ia, d, 64), b = __shfl_up(ibb, d, 64), x = __shfl_up(ix, d, 64);
        const uint32_t pq = __shfl_up(ip, d, 64), iq = __shfl_up(ii, d, 64);
        if (lane >= d) { ia += a; ibb += b; ix ^= x; ip = pre_op(ip, pq); ii += iq; }
    }
    if (lane == 63) {
        wt[0 * NW + wv] = ia; wt[1 * NW + wv] = ibb; wt[2 * NW + wv] = ix;
        wt[3 * NW + wv] = ip; wt[4 * NW + wv] = ii;
    }
    __syncthreads();
    // exclusive prefix of this thread's chunks
    uint32_t ra = ia - ta, rb = ibb - tb, rx = ix ^ tx, ri = ii - ti;
    uint32_t rp = __shfl_up(ip, 1, 64);
    if (lane == 0) rp = 0u;
    for (int w = 0; w < wv; ++w) {
        ra += wt[0 * NW + w]; rb += wt[1 * NW + w]; rx ^= wt[2 * NW + w];
        rp = pre_op(wt[3 * NW + w], rp); ri += wt[4 * NW + w];
    }
    for (int c = cb; c < ce; ++c) {
        const uint32_t a = (uint32_t)sa[cix(c)], b = (uint32_t)sb[cix(c)], x = L.sx_get(cix(c));
        ra += a; rb += b; rx ^= x;
        sa[cix(c)] = (int32_t)ra; sb[cix(c)] = (int32_t)rb; L.sx_set(cix(c), rx);
    }
    for (int q = qb; q < qe; ++q) { rp = pre_op(rp, pre[q]); pre[q] = rp; }
    for (int q = ib; q < ie; ++q) { ri += ilen[q]; ilen[q] = ri; }
    __syncthreads();
}

// Runs every (run, footprint column) item of the row through column_record.
template <bool EMIT>
__device__ void all_column_records(const RowArgs &A, const RowData &D, const RowShared &L,
                                   uint64_t rec_base_r, uint64_t loc_base_r, uint64_t part_base_r,
                                   uint64_t &nloc_tot)
{
    const int ni = (int)*L.nint;
    if (ni == 0) return;
    const uint32_t total = D.ilen[ni - 1];
    for (uint32_t t = threadIdx.x; t < total; t += row_threads()) {
        int lo = 0, hi = ni - 1;            // first interval with prefix > t
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (D.ilen[mid] > t) hi = mid; else lo = mid + 1;
        }
        const uint32_t before = lo ? D.ilen[lo - 1] : 0u;
        const int col = (int)D.icol[lo] + (int)(t - before);
        column_record<EMIT>(A, D, L, (int)D.ihead[lo], (int)D.iend[lo], col, rec_base_r, loc_base_r,
                            part_base_r, nloc_tot);
    }
}

// 32-bit words of the pixel-class column array (16-bit elements when cls16).
__host__ __device__ inline int sx_words(int cw, bool cls16) { return cls16 ? (cw + 1) / 2 : cw; }

// Dynamic LDS: three padded column arrays (the pixel classes in 16 bits with
// cls16), then `cap` staged entries with their auxiliary words and up to
// `cap` footprint intervals.
__host__ __device__ inline size_t row_lds_bytes(int W, int cap, bool cls16)
{
    const int cw = col_words(W);
    return (size_t)(2 * cw + sx_words(cw, cls16)) * 4 + (size_t)cap * 37 + 32;
}

// Phase 1 for one run by one thread: footprint counts, interior spans with
// their claimant xor, running footprint maxima, footprint-union intervals.
__device__ void run_serial(const RowData &D, const RowShared &L, int i, int je, int W)
{
    const uint32_t lab = D.poly[i] + 1;
    uint32_t wtot = 0;
    for (int q = i; q < je; ++q) wtot ^= (D.f[q] & F_W) ? 1u : 0u;
    uint32_t par = wtot;
    int mx = -1;
    uint32_t mall = 0, mnh = 0;
    const int c0first = (int)(D.c[i] & 0xffff);
    if (par && c0first > 0) {
        atomicAdd(&L.sb[cix(0)], 1); atomicSub(&L.sb[cix(c0first)], 1);
        L.sx_xor(cix(0), lab); L.sx_xor(cix(c0first), lab);
    }
    for (int q = i; q < je; ++q) {
        const uint32_t c = D.c[q];
        const int c0 = (int)(c & 0xffff), c1 = (int)(c >> 16);
        const uint8_t f = D.f[q];
        atomicAdd(&L.sa[cix(c0)], 1);
        atomicSub(&L.sa[cix(c1 + 1)], 1);
        mx = max(mx, c1);
        mall = max(mall, (uint32_t)c1 + 1u);
        if (!(f & F_HORIZ)) mnh = max(mnh, (uint32_t)c1 + 1u);
        D.pm[q] = mall | (mnh << 16);
        if (f & F_W) par ^= 1u;
        const int nc0 = (q + 1 < je) ? (int)(D.c[q + 1] & 0xffff) : W;
        const int lo = max(c0, mx + 1), hi = nc0 - 1;
        if (par && lo <= hi) {
            atomicAdd(&L.sb[cix(lo)], 1); atomicSub(&L.sb[cix(hi + 1)], 1);
            L.sx_xor(cix(lo), lab); L.sx_xor(cix(hi + 1), lab);
        }
    }
    // footprint-union intervals of the run
    int ulo = c0first, uhi = (int)(D.c[i] >> 16);
    for (int q = i + 1; q <= je; ++q) {
        const int c0 = q < je ? (int)(D.c[q] & 0xffff) : W + 1;
        if (q < je && c0 <= uhi + 1) { uhi = max(uhi, (int)(D.c[q] >> 16)); continue; }
        const uint32_t j = atomicAdd(L.nint, 1u);
        D.ihead[j] = (uint32_t)i;
        D.iend[j] = (uint32_t)je;
        D.icol[j] = (uint32_t)ulo;
        D.ilen[j] = (uint32_t)(uhi - ulo + 1);
        if (q < je) { ulo = c0; uhi = (int)(D.c[q] >> 16); }
    }
}

__device__ __forceinline__ int wave_incl_max(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v = max(v, t);
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_xor(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v ^= t;
    }
    return v;
}

// Phase 1 for one long run by a whole wave, 64 entries at a time: the
// serial recurrences (parity after each entry, running maxima, interval
// starts) become wave scans with carries between chunks.  Same results as
// run_serial.
__device__ void run_wave(const RowData &D, const RowShared &L, int i, int W)
{
    const int lane = threadIdx.x & 63;
    const uint32_t k = D.poly[i];
    const uint32_t lab = k + 1;
    int je = D.n;
    for (int b = i;; b += 64) {
        const int q = b + lane;
        const bool same = q < D.n && D.poly[q] == k;
        const unsigned long long m = __ballot(!same);
        if (m) { je = b + __ffsll((long long)m) - 1; break; }
    }
    uint32_t nw = 0;
    for (int b = i; b < je; b += 64) {
        const int q = b + lane;
        nw += (uint32_t)__popcll(__ballot(q < je && (D.f[q] & F_W)));
    }
    const uint32_t wtot = nw & 1u;
    const int c0first = (int)(D.c[i] & 0xffff);
    if (lane == 0 && wtot && c0first > 0) {
        atomicAdd(&L.sb[cix(0)], 1); atomicSub(&L.sb[cix(c0first)], 1);
        L.sx_xor(cix(0), lab); L.sx_xor(cix(c0first), lab);
    }
    uint32_t par_c = wtot;
    int mx_c = -1, mall_c = 0, mnh_c = 0, ulo_c = c0first;
    for (int b = i; b < je; b += 64) {
        const int q = b + lane;
        const bool valid = q < je;
        const uint32_t c = valid ? D.c[q] : 0u;
        const int c0 = (int)(c & 0xffff), c1 = (int)(c >> 16);
        const uint8_t f = valid ? D.f[q] : (uint8_t)0;
        if (valid) { atomicAdd(&L.sa[cix(c0)], 1); atomicSub(&L.sa[cix(c1 + 1)], 1); }
        const uint32_t par = par_c ^ wave_incl_xor((f & F_W) ? 1u : 0u);
        const int mxs = wave_incl_max(valid ? c1 : -1);
        const int mx = max(mx_c, mxs);
        const int mall = max(mall_c, wave_incl_max(valid ? c1 + 1 : 0));
        const int mnh = max(mnh_c, wave_incl_max(valid && !(f & F_HORIZ) ? c1 + 1 : 0));
        if (valid) D.pm[q] = (uint32_t)mall | ((uint32_t)mnh << 16);
        const int nc0 = (q + 1 < je) ? (int)(D.c[q + 1] & 0xffff) : W;
        const int lo = max(c0, mx + 1), hi = nc0 - 1;
        if (valid && par && lo <= hi) {
            atomicAdd(&L.sb[cix(lo)], 1); atomicSub(&L.sb[cix(hi + 1)], 1);
            L.sx_xor(cix(lo), lab); L.sx_xor(cix(hi + 1), lab);
        }
        // footprint-union intervals: an entry starts one when it begins more
        // than a column right of every earlier footprint of the run
        const int prev = __shfl_up(mxs, 1, 64);
        const int mx_excl = lane ? max(mx_c, prev) : mx_c;
        const bool start = valid && (q == i || c0 > mx_excl + 1);
        const int ulo = max(ulo_c, wave_incl_max(start ? c0 : -1));
        const bool last = valid && (q + 1 == je || nc0 > mx + 1);
        if (last) {
            const uint32_t j = atomicAdd(L.nint, 1u);
            D.ihead[j] = (uint32_t)i;
            D.iend[j] = (uint32_t)je;
            D.icol[j] = (uint32_t)ulo;
            D.ilen[j] = (uint32_t)(mx - ulo + 1);
        }
        par_c = __shfl(par, 63, 64);
        mx_c = __shfl(mx, 63, 64);
        mall_c = __shfl(mall, 63, 64);
        mnh_c = __shfl(mnh, 63, 64);
        ulo_c = __shfl(ulo, 63, 64);
    }
}

template <bool EMIT>
__device__ void process_row(const RowArgs &A, const RowData &D, const RowShared &L, int64_t r, int W,
                            int Wt, uint32_t *cells_q, int r_local,
                            int32_t *wtoti, uint32_t *wtotu, uint32_t *s_nbp, uint32_t *s_multi,
                            unsigned long long *s_nloc, unsigned long long *s_nrec,
                            unsigned long long *s_base)
{
    const int tid = threadIdx.x;

    // phase 1: per run, footprints (boundary counts), interior claims, the
    //          running footprint maxima and the run list; per entry, the
    //          partial / spanning indicators to be scanned
    for (int q = tid; q < D.n; q += row_threads()) D.pre[q] = pre_own(D.f[q]);
    for_each_run(D, [&](int i, int je) {
        if (je - i > LONG_RUN) {
            const uint32_t j = atomicAdd(L.nlong, 1u);
            if (j < (uint32_t)LONGQ) { L.longq[j] = (uint32_t)i; return; }
        }
        run_serial(D, L, i, je, W);
    });
    __syncthreads();
    {
        const uint32_t nl = min(*L.nlong, (uint32_t)LONGQ);
        for (uint32_t k = (uint32_t)(tid >> 6); k < nl; k += (row_threads() >> 6)) run_wave(D, L, (int)L.longq[k], W);
    }
    __syncthreads();

    // phase 2: prefix scans -> per-pixel boundary count, claim count,
    //          claimant; per-entry partial/spanning prefixes; run spans
    row_scans(L, W, D.pre, D.n, D.ilen, (int)*L.nint, wtotu);

    // phase 3: classify pixels.  sx := 0 (no polygon), label + 1, or for a
    // boundary pixel BFLAG | (label + 1 of its single interior claimant, or 0);
    // sa := per-column record counters, starting with the claimant record.
    uint32_t nb = 0, multi = 0;
    for (int c = tid; c < W; c += row_threads()) {
        const int32_t bc = L.sa[cix(c)], cc = L.sb[cix(c)];
        const uint32_t xc = L.sx_get(cix(c));
        const bool bnd = bc > 0 || cc >= 2;
        L.sx_set(cix(c), bnd ? (L.sx_flag() | (cc == 1 ? xc : 0u)) : (cc == 1 ? xc : 0u));
        L.sa[cix(c)] = (bnd && cc == 1) ? 1 : 0;
        L.sb[cix(c)] = 0;
        nb += bnd ? 1u : 0u;
        multi |= (cc >= 2) ? 1u : 0u;
    }
    atomicAdd(s_nbp, nb);
    if (multi) atomicOr(s_multi, 1u);
    __syncthreads();
    const bool rmulti = *s_multi != 0;
    if (rmulti) {
        // overlapping interiors: every claimant record comes from the run walk
        for (int c = tid; c < W; c += row_threads()) L.sa[cix(c)] = 0;
        __syncthreads();
    }

    // phase 4: count records per column (and local-edge totals)
    uint64_t nloc = 0;
    all_column_records<false>(A, D, L, 0, 0, 0, nloc);
    if (rmulti) for_each_run(D, [&](int i, int je) { claimant_walk<false>(A, D, L, i, je, 0, W); });
    atomicAdd(s_nloc, (unsigned long long)nloc);
    __syncthreads();

    {
        uint32_t nrec = 0;
        for (int c = tid; c < W; c += row_threads()) nrec += (uint32_t)L.sa[cix(c)];
        atomicAdd(s_nrec, (unsigned long long)nrec);
        __syncthreads();
    }
    const uint32_t npart_r = D.n ? (D.pre[D.n - 1] & 0x7fffffffu) : 0u;
    if (EMIT && A.alloc) {
        // reserve this row's output ranges; an overflow abandons the row and
        // the host redoes the canvas with exact sizes
        if (tid == 0) {
            const int sh = (int)(r % NSHARD);
            const unsigned long long b0 = atomicAdd(&A.gctr[gctr_at(sh, 0)], *s_nrec);
            const unsigned long long b1 = atomicAdd(&A.gctr[gctr_at(sh, 1)], *s_nloc);
            const unsigned long long b2 = atomicAdd(&A.gctr[gctr_at(sh, 2)], (unsigned long long)npart_r);
            atomicAdd(&A.gctr[gctr_at(sh, 3)], (unsigned long long)*s_nbp);
            const bool over = b0 + *s_nrec > A.cap_rec || b1 + *s_nloc > A.cap_loc || b2 + npart_r > A.cap_part;
            if (over) atomicOr(A.errflags, 32u);
            s_base[0] = (unsigned long long)sh * A.cap_rec + b0;
            s_base[1] = (unsigned long long)sh * A.cap_loc + b1;
            s_base[2] = (unsigned long long)sh * A.cap_part + b2;
            s_base[3] = over ? 1ull : 0ull;
        }
        __syncthreads();
        if (s_base[3]) {
            // abandoned: an empty row, so that a probe run before the host
            // has seen the flag reads no stale record index
            for (int c = tid; c < W; c += row_threads()) cells_q[tile_index(Wt, c, r_local)] = 0u;
            return;
        }
    }
    if (!EMIT) {
        if (tid == 0) {
            A.row_nrec[r] = *s_nrec;
            A.row_nloc[r] = *s_nloc;
            A.row_npart[r] = npart_r;
            A.row_nbp[r] = *s_nbp;
        }
        return;
    }

    // record ranges of the row's columns: sa := inclusive prefix of the
    // per-column record counts (column c owns [sa[c-1], sa[c])), sb := 0
    block_scan(L.sa, W, wtoti, [](int32_t a, int32_t b) { return a + b; }, 0);
    for (int c = tid; c < W; c += row_threads()) L.sb[cix(c)] = 0;
    __syncthreads();

    // phase 5: records, local edges, partial spans (in row entry order)
    const uint64_t rec_base_r = A.alloc ? s_base[0] : A.rec_base[r];
    const uint64_t loc_base_r = A.alloc ? s_base[1] : A.loc_base[r];
    const uint64_t part_base_r = A.alloc ? s_base[2] : A.part_base[r];
    {
        uint64_t dummy = 0;
        all_column_records<true>(A, D, L, rec_base_r, loc_base_r, part_base_r, dummy);
        if (rmulti) for_each_run(D, [&](int i, int je) { claimant_walk<true>(A, D, L, i, je, rec_base_r, W); });
        else
            for (int c = tid; c < W; c += row_threads()) {
                const uint32_t w = L.sx_get(cix(c));
                if ((w & L.sx_flag()) && (w & ~L.sx_flag())) {
                    uint32_t last;
                    const uint64_t slot = rec_slot(L, c, rec_base_r, last);
                    Cand cd{};
                    cd.poly = (w & ~L.sx_flag()) - 1u;
                    cd.meta = CAND_S | last;
                    cd.eoff = 0;
                    cd.poff = 0;
                    A.cands[slot] = cd;
                }
            }
        for (int q = tid; q < D.n; q += row_threads())
            if (is_partial(D.f[q])) {
                const Edge e = A.edges[D.edge[q]];
                A.pspan[part_base_r + (pre_excl(D, q) & 0x7fffffffu)] = make_double2(e.ylo, e.yhi);
            }
    }
    __syncthreads();

    // phase 6: write the canvas row (tile-major); a boundary pixel points
    //          at its first record (the last one carries CAND_LAST)
    for (int c = tid; c < W; c += row_threads()) {
        uint32_t word = L.sx_get(cix(c));
        if (word & L.sx_flag()) {
            const int32_t b = c ? L.sa[cix(c - 1)] : 0;
            const int32_t e = L.sa[cix(c)];
            if (e - b <= 0 || L.sb[cix(c)] != e - b) { atomicOr(A.errflags, 8u); word = 0; }
            else word = BFLAG | (uint32_t)(rec_base_r + (uint64_t)b);
        }
        cells_q[tile_index(Wt, c, r_local)] = word;
    }
}

template <bool EMIT>
__global__ __launch_bounds__(ROW_THREADS_MAX) void k_rows(RowArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t wtoti[ROW_THREADS_MAX / 64];
    __shared__ uint32_t wtotu[5 * (ROW_THREADS_MAX / 64)];
    __shared__ uint32_t s_locfill, s_nint, s_nbp, s_multi, s_nlong;
    __shared__ uint32_t s_longq[LONGQ];
    __shared__ unsigned long long s_nloc, s_nrec, s_base[4];
    const int cap = A.cap;
    const int cwmax = col_words(A.maxW);
    RowShared L;
    L.sa = (int32_t *)smem;
    L.sb = L.sa + cwmax;
    L.sx = (void *)(L.sb + cwmax);
    L.cls16 = A.cls16 != 0;
    L.locfill = &s_locfill;
    L.nint = &s_nint;
    L.nlong = &s_nlong;
    L.longq = s_longq;
    L.nrec = &s_nrec;
    uint32_t *lpoly = (uint32_t *)(L.sb + cwmax) + sx_words(cwmax, L.cls16);
    uint32_t *lc = lpoly + cap;
    uint32_t *ledge = lc + cap;
    uint32_t *lpm = ledge + cap;
    uint32_t *lpre = lpm + cap;
    uint32_t *lih = lpre + cap;
    uint32_t *lie = lih + cap;
    uint32_t *lic = lie + cap;
    uint32_t *lil = lic + cap;
    uint8_t *lf = (uint8_t *)(lil + cap);
    const int tid = threadIdx.x;

    const int64_t nr = A.rows ? A.nlist : A.nfirst + A.Htot;
    for (int64_t k = blockIdx.x; k < nr; k += gridDim.x) {
        const int64_t r = A.rows ? (int64_t)A.rows[k] : k < A.nfirst ? (int64_t)A.first[k] : k - A.nfirst;
        const int s = (int)A.row_off[r], e = (int)A.row_off[r + 1];
        const int n = e - s;
        if (n < A.min_n || n > A.max_n) continue;
        if (!A.rows && k >= A.nfirst && n > cap) continue;   // taken first
        const CanvasDesc &cd = A.cds[canvas_of_row(A.cds, A.nc, r)];
        const int W = cd.W, Wt = cd.Wt;
        L.W = W;
        uint32_t *cells_q = A.cells + cd.cell_off;
        const int r_local = (int)(r - cd.row_base);
        const int cw = col_words(W);
        if (n <= cap) {
            for (int q = tid; q < n; q += row_threads()) {
                lpoly[q] = A.spoly[s + q];
                lc[q] = A.sc[s + q];
                ledge[q] = A.sedge[s + q];
                lf[q] = A.sf[s + q];
            }
        }
        for (int c = tid; c < cw; c += row_threads()) { L.sa[c] = 0; L.sb[c] = 0; L.sx_set(c, 0u); }
        if (tid == 0) { s_locfill = 0; s_nint = 0; s_nbp = 0; s_multi = 0; s_nloc = 0; s_nrec = 0; s_nlong = 0; }
        __syncthreads();
        if (n <= cap) {
            const RowData D{lpoly, lc, lf, ledge, lpm, lpre, lih, lie, lic, lil, n};
            process_row<EMIT>(A, D, L, r, W, Wt, cells_q, r_local, wtoti, wtotu, &s_nbp, &s_multi, &s_nloc,
                              &s_nrec, s_base);
        } else {
            uint32_t *g = A.gaux + (size_t)6 * s;
            const RowData D{A.spoly + s, A.sc + s, A.sf + s, A.sedge + s, g, g + n, g + 2 * n, g + 3 * n,
                            g + 4 * n, g + 5 * n, n};
            process_row<EMIT>(A, D, L, r, W, Wt, cells_q, r_local, wtoti, wtotu, &s_nbp, &s_multi, &s_nloc,
                              &s_nrec, s_base);
        }
        __syncthreads();
    }
}

// Canvas holding global coarse word g.
__device__ __forceinline__ int canvas_of_coarse(const CanvasDesc *cds, int nc, int64_t g)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cds[mid].coarse_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Coarse level, one wave per coarse block (lane l handles pixels l, l + 64,
// ...): a block whose pixels all carry the same non-boundary word that the
// coarse word can hold stores it, any other block COARSE_FULL.  No
// allocation and no global atomic.
__global__ __launch_bounds__(256) void k_compact(const CanvasDesc *cds, int nc, int64_t ncoarse_tot,
                                                 const uint32_t *cells_all, uint16_t *coarse_all)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t gcell = wave; gcell < ncoarse_tot; gcell += nw) {
        const int q = canvas_of_coarse(cds, nc, gcell);
        const CanvasDesc &cd = cds[q];
        const int W = cd.W, H = cd.H, Wt = cd.Wt, blog = cd.blog, Wc = cd.Wc;
        const uint32_t *cells = cells_all + cd.cell_off;
        uint16_t *coarse = coarse_all + cd.coarse_off;
        const int B = 1 << blog, J = (B * B) / 64;
        if (cd.blog <= 4) continue;   // k_compact_tiles covers these canvases
        const int64_t cell = gcell - cd.coarse_off;
        const uint32_t fullw = cd.cbyte ? COARSE_BYTE_FULL : (uint32_t)COARSE_FULL;
        uint32_t v = 0u;
        if (!cd.empty) {
            const int cy = (int)(cell / Wc), cx = (int)(cell % Wc);
            const int c0 = cx << blog, r0 = cy << blog;
            const uint32_t first = cells[tile_index(Wt, c0, r0)];
            bool same = true;
            for (int j = 0; j < J; ++j) {
                const int p = lane + 64 * j;
                const int c = c0 + (p & (B - 1)), r = r0 + (p >> blog);
                same &= !(c < W && r < H) || cells[tile_index(Wt, c, r)] == first;
            }
            v = (__all(same) && !(first & BFLAG) && first < fullw) ? first : fullw;
        }
        if (lane == 0) {
            if (cd.cbyte) ((uint8_t *)coarse)[cell] = (uint8_t)v;
            else coarse[cell] = (uint16_t)v;
        }
    }
}

// Canvas holding global tile g (canvas words are 256-word tiles).
__device__ __forceinline__ int canvas_of_tile(const CanvasDesc *cds, int nc, int64_t g)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((cds[mid].cell_off >> 8) <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Coarse level of the canvases with 8 x 8 or 16 x 16 blocks, one wavefront
// per 16 x 16 tile, read with one 16-byte load per lane (lane l holds tile
// row l / 4, columns 4 (l % 4) .. 4 (l % 4) + 3): a block is uniform when
// every in-canvas pixel equals its top-left one, found with one ballot.
__global__ __launch_bounds__(256) void k_compact_tiles(const CanvasDesc *cds, int nc, int64_t ntiles,
                                                       const uint32_t *cells_all, uint16_t *coarse_all)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t gt = wave; gt < ntiles; gt += nw) {
        const CanvasDesc &cd = cds[canvas_of_tile(cds, nc, gt)];
        if (cd.blog > 4) continue;
        const int64_t t = gt - (cd.cell_off >> 8);
        const int ty = (int)(t / cd.Wt), tx = (int)(t % cd.Wt);
        const uint4 w = ((const uint4 *)(cells_all + cd.cell_off + t * 256))[lane];
        const int r = ty * 16 + (lane >> 2), c0 = tx * 16 + (lane & 3) * 4;
        const bool b8 = cd.blog == 3;
        const int by = b8 ? (lane >> 5) : 0, bx = b8 ? ((lane & 3) >> 1) : 0;
        const int ref_lane = by * 32 + bx * 2;
        const uint32_t ref = (uint32_t)__shfl((int)w.x, ref_lane, 64);
        const uint32_t wk[4] = {w.x, w.y, w.z, w.w};
        bool same = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) same &= !(c0 + k < cd.W && r < cd.H) || wk[k] == ref;
        const unsigned long long bad = __ballot(!same);
        const unsigned long long mask = b8 ? ((bx ? 0xCCCCCCCCull : 0x33333333ull) << (by * 32)) : ~0ull;
        if (lane == ref_lane) {
            const int cx = b8 ? tx * 2 + bx : tx, cy = b8 ? ty * 2 + by : ty;
            if (cx < cd.Wc && cy < cd.Hc) {
                const uint32_t fullw = cd.cbyte ? COARSE_BYTE_FULL : (uint32_t)COARSE_FULL;
                const uint32_t v = cd.empty ? 0u : ((bad & mask) == 0 && !(ref & BFLAG) && ref < fullw) ? ref : fullw;
                const int64_t cell = (int64_t)cy * cd.Wc + cx;
                uint16_t *coarse = coarse_all + cd.coarse_off;
                if (cd.cbyte) ((uint8_t *)coarse)[cell] = (uint8_t)v;
                else coarse[cell] = (uint16_t)v;
            }
        }
    }
}

// ------------------------------------------------------------ host driver

static int bits_for(uint64_t v)   // bits needed to store values 0..v
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

void drop_graph(spade_canvas *cv)
{
    if (cv->gexec) (void)hipGraphExecDestroy(cv->gexec);
    cv->gexec = nullptr;
    cv->gkey.clear();
}

// Runs `enqueue` (a fixed sequence of launches on ctx's stream) for a canvas
// build whose launch parameters are `key`.  The first build with a key runs
// eagerly and remembers it; the second captures the launches into a graph;
// later builds with the same key replay the graph.  Any capture failure falls
// back to eager launches.  The graph holds no memory-set nodes (buffers are
// cleared by kernels), so replays match eager runs.
// The capture runs on an internal stream (the caller's may be the null
// stream, which cannot be captured): `qs`, the stream the launches go to,
// points there during the capture; the graph is then launched on ctx's stream.
template <typename F>
static hipError_t run_captured(spade_ctx *ctx, spade_canvas *cv, const std::vector<uint64_t> &key,
                               hipStream_t &qs, F &&enqueue)
{
    hipStream_t st = ctx->stream;
    qs = st;
    if (!ctx->graphs) return enqueue();
    if (cv->gexec && cv->gkey == key) {
        ++ctx->graph_replays;
        return hipGraphLaunch(cv->gexec, st);
    }
    if (cv->gkey != key) {
        drop_graph(cv);
        cv->gkey = key;
        return enqueue();
    }
    if (!ctx->capture && hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ctx->capture = nullptr;
        return enqueue();
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return enqueue();
    }
    qs = ctx->capture;
    const hipError_t e1 = enqueue();
    const hipError_t e2 = hipStreamEndCapture(ctx->capture, &g);
    qs = st;
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipErrorUnknown;
    if (e1 == hipSuccess && e2 == hipSuccess && g) e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        (void)hipGetLastError();
        cv->gkey.clear();
        return enqueue();
    }
    cv->gexec = ex;
    ++ctx->graph_captures;
    return hipGraphLaunch(ex, st);
}

static int grid_for(int64_t n, int64_t cap = 65536)
{
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Probe view of canvas q of a set (shared arrays + that canvas's map).
CanvasView view_of(const spade_canvas *cv, int q)
{
    const CanvasDesc &d = cv->descs[(size_t)q];
    CanvasView v{};
    v.X0 = d.X0; v.Y0 = d.Y0; v.sx = d.sx; v.sy = d.sy;
    v.bx0 = d.bx0; v.by0 = d.by0; v.bx1 = d.bx1; v.by1 = d.by1;
    v.W = d.W; v.H = d.H; v.Wt = d.Wt; v.Wc = d.Wc; v.Hc = d.Hc; v.blog = d.blog;
    v.cbyte = d.cbyte;
    v.M = d.M;
    v.cells = (const uint32_t *)cv->cells.p + d.cell_off;
    v.coarse = (const uint16_t *)cv->coarse.p + d.coarse_off;
    v.cands = (const Cand *)cv->cands.p;
    v.ledges = (const Edge *)cv->ledges.p;
    v.pspan = (const double2 *)cv->pspan.p;
    return v;
}

static void finish_views(spade_canvas *cv)
{
    cv->view = view_of(cv, 0);
}

// Sizes canvas q of a set: the context's fixed size, else about ctx->ppv
// pixels per vertex (at most 4096 x 4096 pixels, at least 64 x 64) with
// square world pixels.
static void choose_size(const spade_ctx *ctx, double w, double h, int64_t nverts, int &W, int &H)
{
    if (ctx->canvas_w > 0 && ctx->canvas_h > 0) { W = ctx->canvas_w; H = ctx->canvas_h; return; }
    const double target = std::min(4096.0 * 4096.0, std::max(64.0 * 64.0, ctx->ppv * (double)nverts));
    const double aspect = w / h;
    W = (int)std::max(1.0, std::min((double)MAXW, std::round(std::sqrt(target * aspect))));
    H = (int)std::max(1.0, std::min(16384.0, std::round(target / W)));
}

// First error among the build's device flags (0 if none).
static int flag_error(spade_ctx *ctx, unsigned ef)
{
    if (ef & 1u) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off must start at 0 and be non-decreasing");
    if (ef & 2u) return set_error(ctx, SPADE_E_INVALID, "poly_ring_off must start at 0, be non-decreasing and end at n_rings");
    if (ef & 4u) return set_error(ctx, SPADE_E_INVALID, "non-finite polygon vertex coordinate");
    if (ef & 64u) return set_error(ctx, SPADE_E_INVALID, "n_vertices does not match ring_vtx_off[n_rings]");
    if (ef & 128u) return set_error(ctx, SPADE_E_INVALID, "a polygon vertex lies outside the given bounding box");
    if (ef & 8u) return set_error(ctx, SPADE_E_HIP, "internal: boundary pixel without candidates");
    if (ef & 16u)
        return set_error(ctx, SPADE_E_UNSUPPORTED, "a boundary pixel has more than 32767 edges of one polygon; raise the canvas resolution");
    return SPADE_OK;
}

// The flags word and the row pass's counters sit in one device block (the
// flags at its start, the NGCTR counter words from byte CTR_HEAD), copied
// to the host in one piece.
constexpr size_t CTR_HEAD = 128;
constexpr size_t COUNTER_COPY = CTR_HEAD + sizeof(uint64_t) * NGCTR;

static hipError_t copy_counters(void *hc, const unsigned *d_ctr, hipStream_t st)
{
    return hipMemcpyAsync(hc, d_ctr, COUNTER_COPY, hipMemcpyDeviceToHost, st);
}

static unsigned counter_flags(const void *hc)
{
    unsigned ef;
    std::memcpy(&ef, hc, sizeof(unsigned));
    return ef;
}

// Totals over the shards of counter c, and the largest shard's.
static uint64_t counter_total(const void *hcb, int c, uint64_t *largest = nullptr)
{
    const uint64_t *hc = (const uint64_t *)((const char *)hcb + CTR_HEAD);
    uint64_t t = 0, m = 0;
    for (int k = 0; k < NSHARD; ++k) {
        t += hc[gctr_at(k, c)];
        m = std::max<uint64_t>(m, hc[gctr_at(k, c)]);
    }
    if (largest) *largest = m;
    return t;
}

// Leaves the build's counters and flags on the device; build_flush queues
// their copy to pinned memory (after the caller's probe, so the copy does
// not delay it) and build_finish reads them after the caller's next
// synchronisation.
static int defer_counters(spade_ctx *ctx, spade_canvas *cv, const unsigned *d_ctr)
{
    if (!ctx->pend && hipHostMalloc(&ctx->pend, COUNTER_COPY, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->pend = nullptr;
        return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    }
    cv->pend_src = d_ctr;
    cv->pending = true;
    return SPADE_OK;
}

int build_flush(spade_ctx *ctx, spade_canvas *cv)
{
    if (!cv->pending || !cv->pend_src) return SPADE_OK;
    const unsigned *src = (const unsigned *)cv->pend_src;
    cv->pend_src = nullptr;
    SPADE_HIP(ctx, copy_counters(ctx->pend, src, ctx->stream));
    return SPADE_OK;
}

int build_finish(spade_ctx *ctx, spade_canvas *cv)
{
    if (!cv->pending) return SPADE_OK;
    cv->pending = false;
    if (cv->pend_src) return set_error(ctx, SPADE_E_HIP, "internal: deferred build counters never copied");
    const void *hc = ctx->pend;
    const unsigned ef = counter_flags(hc);
    if (ef & (1u | 2u | 4u | 64u | 128u)) return flag_error(ctx, ef);
    uint64_t mrec, mloc, mpart;
    const uint64_t nrec = counter_total(hc, 0, &mrec), nloc = counter_total(hc, 1, &mloc);
    const uint64_t npart = counter_total(hc, 2, &mpart);
    if (ef & 32u) {
        // the row pass counted every row: with room for every shard's
        // count the next single pass fits
        if (ensure(ctx, cv->cands, sizeof(Cand) * (size_t)(NSHARD * (mrec + 64))) ||
            ensure(ctx, cv->ledges, sizeof(Edge) * (size_t)(NSHARD * (mloc + 64))) ||
            ensure(ctx, cv->pspan, sizeof(double2) * (size_t)(NSHARD * (mpart + 1))))
            return SPADE_E_NOMEM;
        return BUILD_AGAIN;
    }
    if (int rc = flag_error(ctx, ef)) return rc;
    cv->n_boundary = (int64_t)counter_total(hc, 3);
    cv->n_cands = (int64_t)nrec;
    cv->n_elist = (int64_t)(nloc + npart);
    return SPADE_OK;
}

int build_set(spade_ctx *ctx, const spade_polys *polys, int nc, const int64_t *pbound, spade_canvas *cv,
              bool defer)
{
    hipStream_t st = ctx->stream;
    cv->pending = false;
    cv->pend_src = nullptr;
    const int64_t M = polys->n_polys, R = polys->n_rings;
    if (nc < 1) return set_error(ctx, SPADE_E_INVALID, "a canvas set needs at least one canvas");
    cv->nc = nc;

    // vertex count: the caller's (checked on the device), else read back
    int64_t V = 0;
    if (R == 0 && polys->n_vertices > 0)
        return set_error(ctx, SPADE_E_INVALID, "n_vertices does not match ring_vtx_off[n_rings]");
    if (R > 0 && polys->n_vertices > 0) {
        V = polys->n_vertices;
        if (V >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "more than 2^32-1 vertices");
    } else if (R > 0) {
        int64_t *h = (int64_t *)ensure_pinned(ctx, 64);
        if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
        SPADE_HIP(ctx, hipMemcpyAsync(h, polys->ring_vtx_off + R, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        V = h[0];
        if (V < 0) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off[n_rings] is negative");
        if (V >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "more than 2^32-1 vertices");
    }

    // With the caller's box (one canvas, vertex count known) the canvas is
    // sized without waiting for the validation: the edge kernel checks the
    // flags and the box before anything reads the polygon arrays.
    const bool hinted = polys->bbox != nullptr && nc == 1 && (R == 0 || polys->n_vertices > 0);

    // validation + ring->polygon map
    DevBuf &rp = ctx->scratch[S_RINGPOLY];
    DevBuf &br = ctx->scratch[S_BLOCKRED];
    const size_t bbbytes = sizeof(unsigned long long) * 4 * (size_t)nc;
    if (ensure(ctx, rp, sizeof(int32_t) * (size_t)std::max<int64_t>(R, 1)) ||
        ensure(ctx, br, sizeof(double) * 4 * RED_BLOCKS + bbbytes + 128 + COUNTER_COPY))
        return SPADE_E_NOMEM;
    unsigned long long *d_bb = (unsigned long long *)((char *)br.p + sizeof(double) * 4 * RED_BLOCKS);
    // the flags word, then the allocation counters of the row pass (one
    // cache-line-aligned block)
    unsigned *d_err = (unsigned *)(((uintptr_t)(d_bb + 4 * (size_t)nc) + 127) & ~(uintptr_t)127);
    unsigned long long *gctr = (unsigned long long *)((char *)d_err + CTR_HEAD);
    hipLaunchKernelGGL(k_init, dim3((unsigned)std::min<int64_t>((4 * (int64_t)nc + 255) / 256 + 1, 1024)), dim3(256), 0,
                       st, d_err, d_bb, 4 * (int64_t)nc, gctr);
    SPADE_HIP(ctx, hipGetLastError());
    if (M > 0 || R > 0 || V > 0) {
        hipLaunchKernelGGL(k_validate, dim3(RED_BLOCKS), dim3(256), 0, st, M, R, polys->poly_ring_off,
                           polys->ring_vtx_off, V, polys->vx, polys->vy, (int32_t *)rp.p,
                           (double *)br.p, d_err, nc == 1 ? d_bb : nullptr);
        SPADE_HIP(ctx, hipGetLastError());
    }
    // Pinned staging: error flags, canvas descriptors, bounding-box keys.
    // The bounding boxes are computed before the validation verdict is read
    // (one synchronisation for both): the box kernel only reads within the
    // offsets' range even when they are malformed.
    const size_t desc_stage = sizeof(CanvasDesc) * (size_t)nc;
    char *pin = (char *)ensure_pinned(ctx, 64 + desc_stage + 64 + bbbytes);
    if (!pin) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    unsigned *herr = (unsigned *)pin;
    CanvasDesc *hcd = (CanvasDesc *)(pin + 64);
    unsigned long long *hbb = (unsigned long long *)(pin + 64 + ((desc_stage + 63) & ~(size_t)63));

    // per-canvas polygon ranges and vertex counts (host), bounding boxes (device)
    std::vector<CanvasDesc> &cds = cv->descs;
    cds.assign((size_t)nc, CanvasDesc{});
    for (int q = 0; q < nc; ++q) {
        cds[q].poly_base = pbound[q];
        cds[q].M = pbound[q + 1] - pbound[q];
    }
    DevBuf &dcd = cv->dcds;
    if (ensure(ctx, dcd, sizeof(CanvasDesc) * (size_t)nc)) return SPADE_E_NOMEM;
    if (!hinted) {
        std::memcpy(hcd, cds.data(), sizeof(CanvasDesc) * (size_t)nc);
        SPADE_HIP(ctx, hipMemcpyAsync(dcd.p, hcd, sizeof(CanvasDesc) * (size_t)nc, hipMemcpyHostToDevice, st));
    }
    std::vector<int64_t> nverts((size_t)nc, 0);
    std::vector<int64_t> pro, rvo;
    if (V > 0 && nc > 1) {
        hipLaunchKernelGGL(k_canvas_bbox, dim3(grid_for((V + BB_SPAN - 1) / BB_SPAN)), dim3(256), 0, st, R, polys->ring_vtx_off, V,
                           polys->vx, polys->vy, (const int32_t *)rp.p, (const CanvasDesc *)dcd.p, nc, d_bb);
        SPADE_HIP(ctx, hipGetLastError());
        if (nc > 1) {
            // offsets for the vertices per canvas (used once they are validated)
            pro.resize((size_t)M + 1);
            rvo.resize((size_t)R + 1);
            if (polys->poly_ring_off)
                SPADE_HIP(ctx, hipMemcpyAsync(pro.data(), polys->poly_ring_off, sizeof(int64_t) * (M + 1),
                                              hipMemcpyDeviceToHost, st));
            else
                for (int64_t k = 0; k <= M; ++k) pro[k] = k;
            SPADE_HIP(ctx, hipMemcpyAsync(rvo.data(), polys->ring_vtx_off, sizeof(int64_t) * (R + 1),
                                          hipMemcpyDeviceToHost, st));
        }
    }
    if (!hinted) {
        SPADE_HIP(ctx, hipMemcpyAsync(herr, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipMemcpyAsync(hbb, d_bb, bbbytes, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        if (int rc = flag_error(ctx, herr[0])) return rc;
    }
    if (V > 0) {
        if (nc > 1)
            for (int q = 0; q < nc; ++q) nverts[q] = rvo[pro[pbound[q + 1]]] - rvo[pro[pbound[q]]];
        else
            nverts[0] = V;
    }
    auto undkey = [](unsigned long long k) {
        const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
        double d;
        std::memcpy(&d, &b, sizeof d);
        return d;
    };

    // canvas maps, sizes and offsets
    int maxW = 1;
    int64_t Htot = 0, cells_tot = 0, coarse_tot = 0;
    bool any = false;
    for (int q = 0; q < nc; ++q) {
        CanvasDesc &d = cds[q];
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        if (hinted && V > 0) {
            x0 = polys->bbox[0]; x1 = polys->bbox[1];
            y0 = polys->bbox[2]; y1 = polys->bbox[3];
            if (!(x0 <= x1 && y0 <= y1)) return set_error(ctx, SPADE_E_INVALID, "bounding box is not ordered");
        } else if (nverts[q] > 0 || (nc == 1 && V > 0)) {
            x0 = undkey(hbb[4 * q + 0]); x1 = -undkey(hbb[4 * q + 1]);
            y0 = undkey(hbb[4 * q + 2]); y1 = -undkey(hbb[4 * q + 3]);
        }
        d.empty = !(x0 < x1 && y0 < y1);
        int W = 1, H = 1;
        if (!d.empty) choose_size(ctx, x1 - x0, y1 - y0, nverts[q], W, H);
        if (W > MAXW || H > 16384) return set_error(ctx, SPADE_E_UNSUPPORTED, "canvas larger than 8192 x 16384");
        d.W = W; d.H = H;
        if (!d.empty) {
            d.X0 = x0; d.Y0 = y0;
            d.sx = (double)W / (x1 - x0);
            d.sy = (double)H / (y1 - y0);
            d.hy = (y1 - y0) / (double)H;
            d.bx0 = x0; d.bx1 = x1; d.by0 = y0; d.by1 = y1;
            any = true;
        } else {
            d.X0 = d.Y0 = d.sx = d.sy = d.hy = 0.0;
            d.bx0 = d.by0 = INFINITY; d.bx1 = d.by1 = -INFINITY;
        }
        d.Wt = (W + 15) / 16;
        const int Ht = (H + 15) / 16;
        // coarse grid: blocks of 2^blog pixels, as fine as the probe's LDS
        // allows; a single canvas of few polygons has byte-sized words
        d.cbyte = (nc == 1 && d.M <= COARSE_BYTE_MAXM) ? 1 : 0;
        const size_t cw_bytes = d.cbyte ? 1 : 2;
        int blog = 3;
        const size_t cbudget = coarse_lds_budget(d.M);
        while (blog < 6 && (size_t)((W + (1 << blog) - 1) >> blog) * ((H + (1 << blog) - 1) >> blog) * cw_bytes > cbudget)
            ++blog;
        if ((size_t)((W + (1 << blog) - 1) >> blog) * ((H + (1 << blog) - 1) >> blog) * cw_bytes > cbudget)
            return set_error(ctx, SPADE_E_UNSUPPORTED, "coarse canvas exceeds the probe's LDS; lower the canvas resolution");
        d.blog = blog;
        d.Wc = (W + (1 << blog) - 1) >> blog;
        d.Hc = (H + (1 << blog) - 1) >> blog;
        d.row_base = Htot;
        d.cell_off = cells_tot;
        d.coarse_off = coarse_tot;
        Htot += H;
        cells_tot += (int64_t)d.Wt * Ht * 256;
        coarse_tot += (int64_t)d.Wc * d.Hc;
        maxW = std::max(maxW, W);
    }
    if (Htot > 0x7fffffffLL) return set_error(ctx, SPADE_E_UNSUPPORTED, "canvas set has too many rows");
    std::memcpy(hcd, cds.data(), sizeof(CanvasDesc) * (size_t)nc);
    SPADE_HIP(ctx, hipMemcpyAsync(dcd.p, hcd, sizeof(CanvasDesc) * (size_t)nc, hipMemcpyHostToDevice, st));
    const CanvasDesc *d_cds = (const CanvasDesc *)dcd.p;

    if (ensure(ctx, cv->cells, sizeof(uint32_t) * (size_t)cells_tot) ||
        ensure(ctx, cv->coarse, sizeof(uint16_t) * ((size_t)coarse_tot + 2)) ||
        ensure(ctx, cv->edges, sizeof(Edge) * (size_t)std::max<int64_t>(V, 1)))
        return SPADE_E_NOMEM;
    cv->n_edges = V;
    if (!any) {
        SPADE_HIP(ctx, hipMemsetAsync(cv->cells.p, 0, sizeof(uint32_t) * (size_t)cells_tot, st));
        SPADE_HIP(ctx, hipMemsetAsync(cv->coarse.p, 0, sizeof(uint16_t) * ((size_t)coarse_tot + 2), st));
        if (ensure(ctx, cv->cands, 2 * sizeof(Cand)) || ensure(ctx, cv->ledges, sizeof(Edge)) ||
            ensure(ctx, cv->pspan, sizeof(double2)))
            return SPADE_E_NOMEM;
        cv->n_boundary = cv->n_cands = cv->n_elist = 0;
        finish_views(cv);
        if (hinted) {
            // the validation verdict is still to be read
            if (defer) return defer_counters(ctx, cv, d_err);
            unsigned *hf = (unsigned *)ensure_pinned(ctx, 64);
            SPADE_HIP(ctx, hipMemcpyAsync(hf, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            SPADE_HIP(ctx, hipStreamSynchronize(st));
            return flag_error(ctx, hf[0]);
        }
        return SPADE_OK;
    }
    const int W = maxW;
    const int64_t H = Htot;

    // edges, per-edge row spans and the row histogram
    DevBuf &dn = ctx->scratch[S_NROWS];
    DevBuf &dmisc = ctx->scratch[S_MISC];
    DevBuf &drs = ctx->scratch[S_ROWSCAN];
    DevBuf &drow = ctx->scratch[S_ROWOFF];
    const size_t Vs = (size_t)V;
    // misc: epoly[V] u32 | erow0[V] i32 | off[V+1] u64
    // rowscan: rcount[(H+1)*rs] u32 | cursor[H*rs] u32 | longrows[2H] u32 | info[4] u64,
    // with one counter per cache line (rs words apart) unless the set has
    // very many rows
    const int rstride = (H <= 65536) ? 32 : 1;
    const size_t rs = (size_t)rstride;
    if (ensure(ctx, dn, sizeof(uint64_t) * (Vs + 1)) ||
        ensure(ctx, dmisc, sizeof(uint32_t) * Vs * 2 + sizeof(uint64_t) * (Vs + 2)) ||
        ensure(ctx, drs, 4 * rs * (2 * (size_t)H + 1) + 8 * (size_t)H + 96) ||
        ensure(ctx, drow, 8 * ((size_t)H + 1)))
        return SPADE_E_NOMEM;
    uint64_t *nrows = (uint64_t *)dn.p;
    uint32_t *epoly = (uint32_t *)dmisc.p;
    int32_t *erow0 = (int32_t *)(epoly + Vs);
    uint64_t *eoff = (uint64_t *)(((uintptr_t)(erow0 + Vs) + 7) & ~(uintptr_t)7);
    uint32_t *rcount = (uint32_t *)drs.p;
    uint32_t *cursor = rcount + (H + 1) * rs;
    uint32_t *longrows = cursor + H * rs;
    unsigned long long *rinfo = (unsigned long long *)(((uintptr_t)(longrows + 2 * H) + 7) & ~(uintptr_t)7);
    uint32_t *row_off = (uint32_t *)drow.p;
    // per-row counters of the exact path (8 arrays of H + 1)
    DevBuf &drc = ctx->scratch[S_ROWCNT];
    if (ensure(ctx, drc, 8 * 8 * ((size_t)H + 1))) return SPADE_E_NOMEM;

    // LDS stage of the row kernel: up to `cap` entries of a row; narrow
    // canvases aim for three or four workgroups per CU, wider ones for two
    // (measured best).  Pixel classes take 16 bits when every label + 1 fits
    // in 15.
    int64_t maxM_all = 1;
    for (int q = 0; q < nc; ++q) maxM_all = std::max<int64_t>(maxM_all, cds[q].M);
    const bool cls16 = maxM_all < 0x8000;
    const size_t col_bytes = row_lds_bytes(W, 0, cls16);
    const size_t target = (col_bytes <= 40 * 1024) ? 38 * 1024 : (col_bytes <= 60 * 1024) ? 78 * 1024 : 150 * 1024;
    const int cap = (int)std::max<size_t>(256, (target - std::min(target - 256 * 37, col_bytes)) / 37);
    // rows up to capB entries run in the launch over all rows, taken first,
    // their entries and auxiliary words in global memory; longer ones get a
    // launch of their own with a stage for the longest
    const int capB = std::max(cap, 640);

    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for((H + 1) * rstride, 1024)), dim3(256), 0, st, (H + 1) * rstride, rcount);
    hipLaunchKernelGGL(k_edges, dim3(grid_for(2 * V)), dim3(256), 0, st, R, polys->ring_vtx_off, V,
                       polys->vx, polys->vy, (const int32_t *)rp.p, d_cds, nc, (Edge *)cv->edges.p, epoly,
                       erow0, nrows, rcount, rstride, hinted ? 1 : 0, d_err, (const unsigned long long *)d_bb,
                       hinted ? polys->bbox[0] : 0.0, hinted ? polys->bbox[1] : 0.0,
                       hinted ? polys->bbox[2] : 0.0, hinted ? polys->bbox[3] : 0.0);
    SPADE_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_rowscan, dim3(1), dim3(SCAN_THREADS), 0, st, H, (const uint32_t *)rcount, rstride, cap, capB,
                       row_off, cursor, longrows, rinfo);
    SPADE_HIP(ctx, hipGetLastError());
    uint64_t *hT = (uint64_t *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(hT, rinfo, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    if (!ctx->evinfo) SPADE_HIP(ctx, hipEventCreateWithFlags(&ctx->evinfo, hipEventDisableTiming));
    SPADE_HIP(ctx, hipEventRecord(ctx->evinfo, st));

    const int cbits = std::max(1, bits_for((uint64_t)W - 1));
    int64_t maxM = 1;
    for (int q = 0; q < nc; ++q) maxM = std::max<int64_t>(maxM, cds[q].M);
    const int pbits = std::max(1, bits_for((uint64_t)(maxM - 1)));
    const int rbits = std::max(1, bits_for((uint64_t)H - 1));
    const int ebits = std::max(1, bits_for((uint64_t)V - 1));
    DevBuf &dk = ctx->scratch[S_KEYS], &dk2 = ctx->scratch[S_KEYS2];
    DevBuf &dv = ctx->scratch[S_VALS], &dv2 = ctx->scratch[S_VALS2];
    DevBuf &dc = ctx->scratch[S_ENTC], &df = ctx->scratch[S_ENTF];
    // While the host waits for the totals, the entries go into the buffers
    // of earlier builds when the total fits them (the kernel checks); the
    // room is counted so that no buffer below grows under it.
    const uint64_t tcap = std::min(std::min(dk.cap / 8, dc.cap / 20), df.cap >= 16 ? (df.cap - 16) / 2 : 0);
    const bool spec = tcap > 0 && pbits + cbits + ebits <= 63;
    if (spec) {
        hipLaunchKernelGGL(k_entries_rows, dim3(grid_for(4 * V)), dim3(256), 0, st, V, (const Edge *)cv->edges.p,
                           epoly, erow0, nrows, d_cds, nc, ebits, cbits + ebits, cursor, rstride,
                           (uint64_t *)dk.p, (uint32_t *)dc.p, (uint8_t *)df.p,
                           (const unsigned long long *)rinfo, tcap);
        SPADE_HIP(ctx, hipGetLastError());
    }
    SPADE_HIP(ctx, hipEventSynchronize(ctx->evinfo));
    const uint64_t T = hT[0], maxrow = hT[1], nlistB = hT[2], nlistC = hT[3];
    if (T >= 0x7fffffffULL) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many (edge,row) entries; lower the canvas height");
    // Entries go straight into row buckets and each row is sorted in LDS by
    // (polygon, first column, edge); rows longer than the LDS sort, or keys
    // wider than 63 bits (the top bit stays clear so that real keys sort
    // before the padding), take one device-wide sort of (row, polygon, first
    // column) instead.  Both give the same order.
    const bool bucketed = maxrow <= (uint64_t)ROWSORT_MAX && pbits + cbits + ebits <= 63;
    // stage of the longest rows' launch: the longest row, up to 150 KB
    const int cap_stage = (int)std::max<size_t>((size_t)capB, (150 * 1024 - std::min<size_t>(150 * 1024 - 256 * 37, col_bytes)) / 37);
    const int cap_big = (int)std::max<uint64_t>((uint64_t)capB, std::min<uint64_t>((uint64_t)cap_stage, maxrow));

    if (!bucketed && cbits + pbits + rbits > 64) return set_error(ctx, SPADE_E_UNSUPPORTED, "sort key exceeds 64 bits");

    // the speculative entries stand when the rows are sorted per row
    const bool entries_done = spec && bucketed && T <= tcap;
    const size_t Ts = (size_t)std::max<uint64_t>(T, 1);
    // dc: ent_c[T] | sorted c[T] | perm[T] | perm2[T] | sorted poly[T]; df: ent_f[T] | sorted f[T]
    if (ensure(ctx, dk, 8 * Ts) || ensure(ctx, dv2, 4 * Ts) || ensure(ctx, dc, 20 * Ts) ||
        ensure(ctx, df, 2 * Ts + 16))
        return SPADE_E_NOMEM;
    if (!bucketed && (ensure(ctx, dk2, 8 * Ts) || ensure(ctx, dv, 4 * Ts))) return SPADE_E_NOMEM;
    uint32_t *ent_c = (uint32_t *)dc.p, *s_c = ent_c + Ts, *perm = s_c + Ts, *perm2 = perm + Ts;
    uint32_t *s_poly = perm2 + Ts;
    uint8_t *ent_f = (uint8_t *)df.p, *s_f = ent_f + Ts;
    uint32_t *s_edge = (uint32_t *)dv2.p;
    const int kbits = cbits + pbits + rbits;
    hipStream_t qs = st;   // stream of the build's launches (see run_captured)
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tbytes = 0, tscan = 0;
    const int pmax = (int)std::max<uint64_t>(1, maxrow);
    const size_t sort_lds = (size_t)pmax * 16 + 16;
    if (bucketed)
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_rowsort, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sort_lds));
    if (!bucketed) {
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tscan, nrows, eoff, (int)(V + 1), st));
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, (const uint64_t *)dk.p,
                                                          (uint64_t *)dk2.p, (const uint32_t *)perm,
                                                          perm2, (int)T, 0, kbits, st));
        if (ensure(ctx, cub, std::max(tbytes, tscan))) return SPADE_E_NOMEM;
    }
    auto enqueue_entries = [&]() -> hipError_t {
        hipError_t e;
        if (bucketed) {
            if (!entries_done) {
                hipLaunchKernelGGL(k_entries_rows, dim3(grid_for(4 * V)), dim3(256), 0, qs, V,
                                   (const Edge *)cv->edges.p, epoly, erow0, nrows, d_cds, nc, ebits, cbits + ebits,
                                   cursor, rstride, (uint64_t *)dk.p, ent_c, ent_f,
                                   (const unsigned long long *)nullptr, (uint64_t)0);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            const int64_t sort_items = H + (int64_t)nlistB + (int64_t)nlistC;
            hipLaunchKernelGGL(k_rowsort, dim3((unsigned)std::min<int64_t>(sort_items, 65535)), dim3(SORT_THREADS), sort_lds,
                               qs, H, (const uint32_t *)row_off, (const uint64_t *)dk.p, (const uint32_t *)ent_c,
                               (const uint8_t *)ent_f, cbits + ebits, (1ULL << ebits) - 1, s_poly, s_edge, s_c,
                               s_f, pmax, (const uint32_t *)longrows, (int64_t)nlistB, (int64_t)nlistC, cap);
            return hipGetLastError();
        }
        size_t tb1 = tscan;
        e = hipcub::DeviceScan::ExclusiveSum(cub.p, tb1, nrows, eoff, (int)(V + 1), qs);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_entries, dim3(grid_for(V)), dim3(256), 0, qs, V, (const Edge *)cv->edges.p,
                           epoly, erow0, nrows, eoff, d_cds, nc, cbits, pbits, (uint64_t *)dk.p, (uint32_t *)dv.p,
                           ent_c, ent_f, perm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        size_t tb2 = tbytes;
        e = hipcub::DeviceRadixSort::SortPairs(cub.p, tb2, (const uint64_t *)dk.p, (uint64_t *)dk2.p,
                                               (const uint32_t *)perm, perm2, (int)T, 0, kbits, qs);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gather, dim3(grid_for((int64_t)T + 1)), dim3(256), 0, qs, (int64_t)T, perm2, ent_c,
                           ent_f, (const uint32_t *)dv.p, (const uint64_t *)dk2.p, cbits,
                           (pbits >= 64) ? ~0ULL : ((1ULL << pbits) - 1), cbits + pbits, H, s_c, s_f, s_poly,
                           s_edge, row_off);
        return hipGetLastError();
    };

    uint64_t *row_nrec = (uint64_t *)drc.p;
    uint64_t *row_nloc = row_nrec + (H + 1);
    uint64_t *row_npart = row_nloc + (H + 1);
    uint64_t *row_nbp = row_npart + (H + 1);
    uint64_t *rec_base = row_nbp + (H + 1);
    uint64_t *loc_base = rec_base + (H + 1);
    uint64_t *part_base = loc_base + (H + 1);
    uint64_t *bp_scan = part_base + (H + 1);

    RowArgs ra{};
    ra.cds = d_cds;
    ra.nc = nc;
    ra.maxW = W;
    ra.Htot = H;
    ra.row_off = row_off;
    ra.spoly = s_poly;
    ra.sedge = s_edge;
    ra.sc = s_c;
    ra.sf = s_f;
    ra.edges = (const Edge *)cv->edges.p;
    ra.row_nrec = row_nrec; ra.row_nloc = row_nloc; ra.row_npart = row_npart; ra.row_nbp = row_nbp;
    ra.rec_base = rec_base; ra.loc_base = loc_base; ra.part_base = part_base;
    ra.errflags = d_err;
    ra.cap = cap;
    ra.cls16 = cls16 ? 1 : 0;
    const size_t rlds = row_lds_bytes(W, ra.cap, cls16);
    // the longest rows: a stage for the longest of them, up to 150 KB
    const size_t rlds_big = row_lds_bytes(W, cap_big, cls16);
    if (maxrow > (uint64_t)cap_big || nlistB > 0) {
        // rows without a stage: global auxiliary words for them
        if (ensure(ctx, ctx->scratch[S_NEXTP], sizeof(uint32_t) * 6 * Ts)) return SPADE_E_NOMEM;
        ra.gaux = (uint32_t *)ctx->scratch[S_NEXTP].p;
    }
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_rows<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::max(rlds, rlds_big)));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_rows<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::max(rlds, rlds_big)));
    // The longest rows run in a launch of their own, one workgroup per row
    // with a stage for the longest, on an internal stream beside the launch
    // over all rows (a few long border rows would otherwise add their whole
    // latency).  That launch takes the mid-length rows first, so that their
    // slower global-memory passes start at once.
    const bool bigrows = nlistC > 0;
    if (bigrows && !ctx->side2) {
        if (!ctx->side) SPADE_HIP(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        SPADE_HIP(ctx, hipStreamCreateWithFlags(&ctx->side2, hipStreamNonBlocking));
        if (!ctx->fork) SPADE_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
        if (!ctx->join) SPADE_HIP(ctx, hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
        SPADE_HIP(ctx, hipEventCreateWithFlags(&ctx->join2, hipEventDisableTiming));
    }
    // a stage that leaves room for at most two workgroups per CU gets 512
    // threads per row instead of 256, so the CU still runs 16 waves
    auto row_threads_for = [](size_t lds) {
        return (ROW_LDS_PER_CU / std::max<size_t>(lds, 1) <= 2) ? ROW_THREADS_MAX : ROW_THREADS;
    };
    auto launch_list = [&](bool emit, hipStream_t s2, hipEvent_t done, const uint32_t *list, uint64_t n,
                           int stage, size_t lds, int min_n, int max_n) -> hipError_t {
        RowArgs a2 = ra;
        a2.cap = stage;
        a2.min_n = min_n;
        a2.max_n = max_n;
        a2.rows = list;
        a2.nlist = (int64_t)n;
        const int bgrid = (int)std::min<uint64_t>(n, 8192);
        hipError_t e = hipStreamWaitEvent(s2, ctx->fork, 0);
        if (e != hipSuccess) return e;
        const int rt = row_threads_for(lds);
        if (emit) hipLaunchKernelGGL(k_rows<true>, dim3(bgrid), dim3(rt), lds, s2, a2);
        else hipLaunchKernelGGL(k_rows<false>, dim3(bgrid), dim3(rt), lds, s2, a2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return hipEventRecord(done, s2);
    };
    auto launch_rows = [&](bool emit) -> hipError_t {
        hipError_t e;
        if (bigrows && (e = hipEventRecord(ctx->fork, qs)) != hipSuccess) return e;
        if (bigrows && (e = launch_list(emit, ctx->side2, ctx->join2, longrows + H, nlistC, cap_big, rlds_big,
                                        capB + 1, 0x7fffffff)) != hipSuccess)
            return e;
        RowArgs a1 = ra;
        a1.min_n = 0;
        a1.max_n = capB;
        a1.first = longrows;
        a1.nfirst = (int64_t)nlistB;
        const int g1 = (int)std::min<int64_t>(H + (int64_t)nlistB, 8192);
        const int rt = row_threads_for(rlds);
        if (emit) hipLaunchKernelGGL(k_rows<true>, dim3(g1), dim3(rt), rlds, qs, a1);
        else hipLaunchKernelGGL(k_rows<false>, dim3(g1), dim3(rt), rlds, qs, a1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (bigrows && (e = hipStreamWaitEvent(qs, ctx->join2, 0)) != hipSuccess) return e;
        return hipSuccess;
    };
    ra.cells = (uint32_t *)cv->cells.p;

    // Coarse level from the canvas words: tile by tile for 8 x 8 and 16 x 16
    // blocks, block by block for larger ones.
    bool small_blocks = false, large_blocks = false;
    for (int q = 0; q < nc; ++q) (cds[q].blog <= 4 ? small_blocks : large_blocks) = true;
    const int compact_mode = (small_blocks ? 1 : 0) | (large_blocks ? 2 : 0);
    auto launch_compact = [&]() -> hipError_t {
        if (small_blocks) {
            const int64_t ntiles = cells_tot / 256;
            const int tgrid = (int)std::max<int64_t>(1, std::min<int64_t>((ntiles + 3) / 4, 65536));
            hipLaunchKernelGGL(k_compact_tiles, dim3(tgrid), dim3(256), 0, qs, d_cds, nc, ntiles,
                               (const uint32_t *)cv->cells.p, (uint16_t *)cv->coarse.p);
        }
        if (large_blocks) {
            const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>((coarse_tot + 3) / 4, 65536));
            hipLaunchKernelGGL(k_compact, dim3(cgrid), dim3(256), 0, qs, d_cds, nc, coarse_tot,
                               (const uint32_t *)cv->cells.p, (uint16_t *)cv->coarse.p);
        }
        return hipGetLastError();
    };

    // One row pass: rows reserve their output ranges with atomics inside the
    // capacity the canvas already holds (at least a guess from the entry
    // count; partial spans <= T exactly).  A row that would overflow is
    // abandoned and the host redoes the canvas with exact sizes (which then
    // stay allocated for the next build).  The coarse level is built right
    // behind the pass, and one synchronisation reads the counters and flags
    // of both.
    bool done_single = false;
    uint64_t nrec = 0, nloc = 0, npart = 0, nbp = 0;
    unsigned ef = 0;
    {
        ra.alloc = 1;
        ra.gctr = gctr;
        if (ensure(ctx, cv->cands, sizeof(Cand) * (size_t)(2 * T + 1024)) ||
            ensure(ctx, cv->ledges, sizeof(Edge) * (size_t)(2 * T + 1024)) ||
            ensure(ctx, cv->pspan, sizeof(double2) * (size_t)(T + 16)))
            return SPADE_E_NOMEM;
        // the slot after the last record stays unused: the count probe reads
        // a pixel's records two at a time
        ra.cap_rec = std::min<uint64_t>(cv->cands.cap / sizeof(Cand) - 1, (uint64_t)BFLAG - 1) / NSHARD;
        ra.cap_loc = std::min<uint64_t>(cv->ledges.cap / sizeof(Edge), 0xffffffffULL) / NSHARD;
        ra.cap_part = std::min<uint64_t>(cv->pspan.cap / sizeof(double2), 0xffffffffULL) / NSHARD;
        ra.cands = (Cand *)cv->cands.p;
        ra.ledges = (Edge *)cv->ledges.p;
        ra.pspan = (double2 *)cv->pspan.p;
        auto enqueue = [&]() -> hipError_t {
            hipError_t e = enqueue_entries();
            if (e == hipSuccess) e = launch_rows(true);
            if (e == hipSuccess) e = launch_compact();
            return e;
        };
        // The launches from the entries to the coarse level depend only on
        // the values below: a canvas rebuilt with the same ones replays them
        // from a captured graph instead of launching some thirty kernels.
        std::vector<uint64_t> key;
        auto put = [&](uint64_t v) { key.push_back(v); };
        auto putp = [&](const void *p) { key.push_back((uint64_t)(uintptr_t)p); };
        put(T); put((uint64_t)V); put((uint64_t)H); put((uint64_t)W); put((uint64_t)nc); put((uint64_t)coarse_tot);
        put((uint64_t)cbits); put((uint64_t)pbits); put((uint64_t)kbits); put(tbytes); put(tscan);
        put(bucketed ? 1 : 0); put(entries_done ? 1 : 0); put((uint64_t)ebits); put(sort_lds); put(nlistB); put(nlistC);
        put((uint64_t)capB); put((uint64_t)rstride);
        put((uint64_t)ra.cap); put((uint64_t)cap_big); put(rlds); put(rlds_big); put((uint64_t)ra.cls16);
        put((uint64_t)compact_mode);
        put(ra.cap_rec); put(ra.cap_loc); put(ra.cap_part);
        putp(cv->edges.p); putp(epoly); putp(erow0); putp(nrows); putp(eoff); putp(d_cds);
        putp(dk.p); putp(dk2.p); putp(dv.p); putp(dv2.p); putp(dc.p); putp(df.p); putp(drow.p); putp(cub.p);
        putp(ra.gaux); putp(gctr); putp(d_err); putp(drc.p); putp(drs.p);
        putp(cv->cells.p); putp(cv->cands.p); putp(cv->ledges.p); putp(cv->pspan.p); putp(cv->coarse.p);
        putp(ctx->side); putp(ctx->side2); putp(ctx->fork); putp(ctx->join); putp(ctx->join2);
        SPADE_HIP(ctx, run_captured(ctx, cv, key, qs, enqueue));
        if (defer) {
            finish_views(cv);
            return defer_counters(ctx, cv, d_err);
        }
        void *hc = ensure_pinned(ctx, COUNTER_COPY);
        if (!hc) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
        SPADE_HIP(ctx, copy_counters(hc, d_err, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        ef = counter_flags(hc);
        if (ef & (1u | 2u | 4u | 64u | 128u)) return flag_error(ctx, ef);   // a hinted build's verdict
        if (!(ef & 32u)) {
            done_single = true;
            nrec = counter_total(hc, 0); nloc = counter_total(hc, 1);
            npart = counter_total(hc, 2); nbp = counter_total(hc, 3);
        } else {
            // overflow: clear the flag and redo with exact sizes
            ef &= ~32u;
            SPADE_HIP(ctx, hipMemcpyAsync(d_err, &ef, sizeof(unsigned), hipMemcpyHostToDevice, st));
        }
    }
    if (!done_single) {
        ra.alloc = 0;
        SPADE_HIP(ctx, hipMemsetAsync(drc.p, 0, 8 * 8 * ((size_t)H + 1), st));
        SPADE_HIP(ctx, launch_rows(false));
        // per-row bases (exclusive scans over H+1 entries with a zero tail)
        size_t tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, row_nrec, rec_base, H + 1, st));
        if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nrec, rec_base, H + 1, st));
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nloc, loc_base, H + 1, st));
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_npart, part_base, H + 1, st));
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nbp, bp_scan, H + 1, st));
        uint64_t *hs = (uint64_t *)ensure_pinned(ctx, 64);
        SPADE_HIP(ctx, hipMemcpyAsync(hs + 0, rec_base + H, 8, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipMemcpyAsync(hs + 1, loc_base + H, 8, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipMemcpyAsync(hs + 2, part_base + H, 8, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipMemcpyAsync(hs + 3, bp_scan + H, 8, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        nrec = hs[0]; nloc = hs[1]; npart = hs[2]; nbp = hs[3];
        if (nrec >= (uint64_t)BFLAG) return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary index exceeds 2^31 records; lower the canvas resolution");
        if (nloc >= 0xffffffffULL || npart >= 0xffffffffULL)
            return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary edge lists exceed 2^32 entries");
        if (ensure(ctx, cv->cands, sizeof(Cand) * (size_t)(nrec + 1)) ||
            ensure(ctx, cv->ledges, sizeof(Edge) * (size_t)std::max<uint64_t>(nloc, 1)) ||
            ensure(ctx, cv->pspan, sizeof(double2) * (size_t)std::max<uint64_t>(npart, 1)))
            return SPADE_E_NOMEM;
        ra.cands = (Cand *)cv->cands.p;
        ra.ledges = (Edge *)cv->ledges.p;
        ra.pspan = (double2 *)cv->pspan.p;
        SPADE_HIP(ctx, launch_rows(true));
        SPADE_HIP(ctx, launch_compact());
        unsigned *herr2 = (unsigned *)ensure_pinned(ctx, 64);
        SPADE_HIP(ctx, hipMemcpyAsync(herr2, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        ef = herr2[0];
    }
    if (int rc = flag_error(ctx, ef)) return rc;
    cv->n_boundary = (int64_t)nbp;
    cv->n_cands = (int64_t)nrec;
    cv->n_elist = (int64_t)(nloc + npart);
    finish_views(cv);
    return SPADE_OK;
}

int build_canvas(spade_ctx *ctx, const spade_polys *polys, spade_canvas *cv, bool defer)
{
    const int64_t b[2] = {0, polys->n_polys};
    return build_set(ctx, polys, 1, b, cv, defer);
}

}  // namespace spade
