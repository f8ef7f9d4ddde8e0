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
//   k_edges      one thread per vertex: edge record, pixel row range
//   scan         edge -> first (edge,row) entry
//   k_entries    one (edge,row) entry per row an edge touches: footprint
//                columns [c0,c1], spanning flag, parity weight at the row centre
//   radix sort   entries by (row, polygon, c0)
//   k_row_off    row -> first entry
//   k_rows<0>    per row, in LDS: count boundary pixels / records / edge ids
//   scans        per-row bases
//   k_rows<1>    per row, in LDS: write canvas words, records, edge ids
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
constexpr int RED_BLOCKS = 256;

constexpr uint8_t F_SPAN = 1;    // edge spans the whole dilated row band
constexpr uint8_t F_W = 2;       // edge straddles the row-centre line
constexpr uint8_t F_HORIZ = 4;   // horizontal edge (never crosses)

struct Map {
    double X0, Y0, sx, sy, hy;
    int32_t W, H;
};

// ------------------------------------------------------------ validation

__global__ __launch_bounds__(256) void k_validate(int64_t M, int64_t R, const int64_t *pro,
                                                  const int64_t *rvo, int64_t V, const double *vx,
                                                  const double *vy, int32_t *ring_poly,
                                                  double *blockred, unsigned *errflags)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
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
}

// ------------------------------------------------------------ edges

__global__ __launch_bounds__(256) void k_edges(int64_t R, const int64_t *rvo, int64_t V,
                                               const double *vx, const double *vy,
                                               const int32_t *ring_poly, Map m, Edge *edges,
                                               uint32_t *epoly, int32_t *erow0, uint64_t *nrows)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < V; j += nth) {
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
        Edge e;
        if (ay <= by) { e.xlo = ax; e.ylo = ay; e.xhi = bx; e.yhi = by; }
        else          { e.xlo = bx; e.ylo = by; e.xhi = ax; e.yhi = ay; }
        edges[j] = e;
        if (ax == bx && ay == by) { nrows[j] = 0; erow0[j] = 0; continue; }   // zero length
        double vlo = __dmul_rn(__dsub_rn(e.ylo, m.Y0), m.sy);
        double vhi = __dmul_rn(__dsub_rn(e.yhi, m.Y0), m.sy);
        double f0 = floor(vlo - MARGIN), f1 = floor(vhi + MARGIN);
        int32_t r0 = (int32_t)fmax(0.0, fmin(f0, (double)(m.H - 1)));
        int32_t r1 = (int32_t)fmax(0.0, fmin(f1, (double)(m.H - 1)));
        erow0[j] = r0;
        nrows[j] = (uint64_t)(r1 - r0 + 1);
    }
}

// ------------------------------------------------------------ (edge,row) entries

__global__ __launch_bounds__(256) void k_entries(int64_t V, const Edge *edges, const uint32_t *epoly,
                                                 const int32_t *erow0, const uint64_t *nrows,
                                                 const uint64_t *off, Map m, int cbits, int pbits,
                                                 uint64_t *keys, uint32_t *vals, uint32_t *ent_c,
                                                 uint8_t *ent_f)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < V; j += nth) {
        const uint64_t nr = nrows[j];
        if (nr == 0) continue;
        const Edge e = edges[j];
        const bool horiz = (e.ylo == e.yhi);
        const double ulo = __dmul_rn(__dsub_rn(e.xlo, m.X0), m.sx);
        const double uhi = __dmul_rn(__dsub_rn(e.xhi, m.X0), m.sx);
        const double vlo = __dmul_rn(__dsub_rn(e.ylo, m.Y0), m.sy);
        const double vhi = __dmul_rn(__dsub_rn(e.yhi, m.Y0), m.sy);
        const uint64_t poly = epoly[j];
        const uint64_t base = off[j];
        for (uint64_t t = 0; t < nr; ++t) {
            const int32_t r = erow0[j] + (int32_t)t;
            const double b0 = (double)r - MARGIN, b1 = (double)r + 1.0 + MARGIN;
            double xa, xb;
            if (vlo == vhi) {
                xa = ulo; xb = uhi;
            } else {
                double dv = vhi - vlo;
                double ta = fmin(1.0, fmax(0.0, (b0 - vlo) / dv));
                double tb = fmin(1.0, fmax(0.0, (b1 - vlo) / dv));
                xa = ulo + ta * (uhi - ulo);
                xb = ulo + tb * (uhi - ulo);
            }
            double xmn = fmin(xa, xb) - SLOP, xmx = fmax(xa, xb) + SLOP;
            int32_t c0 = (int32_t)fmax(0.0, fmin(floor(xmn - MARGIN), (double)(m.W - 1)));
            int32_t c1 = (int32_t)fmax(0.0, fmin(floor(xmx + MARGIN), (double)(m.W - 1)));
            const bool span = !horiz && vlo <= b0 && vhi >= b1;
            const double yc = m.Y0 + ((double)r + 0.5) * m.hy;
            const bool w = !horiz && straddles(e.ylo, e.yhi, yc);
            const uint64_t idx = base + t;
            keys[idx] = ((uint64_t)r << (pbits + cbits)) | (poly << cbits) | (uint64_t)c0;
            vals[idx] = (uint32_t)j;
            ent_c[idx] = (uint32_t)c0 | ((uint32_t)c1 << 16);
            ent_f[idx] = (span ? F_SPAN : 0) | (w ? F_W : 0) | (horiz ? F_HORIZ : 0);
        }
    }
}

// After the sort, vals holds the edge id and a second array the permutation;
// gather the per-entry payload into sorted order.
__global__ void k_gather_entries(int64_t T, const uint32_t *perm, const uint32_t *ent_c,
                                 const uint8_t *ent_f, const uint64_t *skeys, int cbits, uint64_t pmask,
                                 uint32_t *s_c, uint8_t *s_f, uint32_t *s_poly)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += nth) {
        uint32_t p = perm[i];
        s_c[i] = ent_c[p];
        s_f[i] = ent_f[p];
        s_poly[i] = (uint32_t)((skeys[i] >> cbits) & pmask);
    }
}

__global__ void k_gather_u32(int64_t T, const uint32_t *perm, const uint32_t *src, uint32_t *dst)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += nth) dst[i] = src[perm[i]];
}

__global__ void k_iota(int64_t T, uint32_t *v)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += nth) v[i] = (uint32_t)i;
}

__global__ void k_row_off(int64_t T, const uint64_t *skeys, int shift, int32_t H, uint32_t *row_off)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= T; i += nth) {
        int64_t ri = (i < T) ? (int64_t)(skeys[i] >> shift) : (int64_t)H;
        int64_t rp = (i == 0) ? -1 : (int64_t)(skeys[i - 1] >> shift);
        for (int64_t rr = rp + 1; rr <= ri; ++rr) row_off[rr] = (uint32_t)i;
    }
}

// ------------------------------------------------------------ per-row scanline

// Column arrays of a row live in LDS with one pad word per 32 so that the
// contiguous per-thread chunks of the scans do not collide in LDS banks.
__device__ __forceinline__ int cix(int c) { return c + (c >> 5); }
__host__ __device__ inline int col_words(int W) { return W + 1 + (W + 1) / 32 + 1; }

// Block-wide in-place inclusive scan of a[cix(0..n)) with ROW_THREADS
// threads: contiguous per-thread chunks, wave-level shuffle scan of the
// chunk totals, one LDS word per wave.  `op` must be associative and
// commutative.
template <typename T, typename Op>
__device__ void block_scan(T *a, int n, T *wtot, Op op, T ident)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + ROW_THREADS - 1) / ROW_THREADS;
    const int b = min(n, tid * per), e = min(n, b + per);
    T acc = ident;
    for (int i = b; i < e; ++i) { acc = op(acc, a[cix(i)]); a[cix(i)] = acc; }
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
    for (int i = b; i < e; ++i) a[cix(i)] = op(pre, a[cix(i)]);
    __syncthreads();
}

struct RowArgs {
    Map m;
    int Wt;                  // canvas tiles per row (tile = 16 x 16 pixels)
    int cap;                 // entries of one row staged in LDS
    const uint32_t *row_off;
    const uint32_t *spoly;   // polygon per sorted entry
    const uint32_t *sedge;   // edge id per sorted entry
    const uint32_t *sc;      // c0 | c1 << 16
    const uint8_t *sf;
    const Edge *edges;
    uint32_t *gaux;          // 5 words per entry for rows too long to stage
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
    uint32_t *rhead;  // run list: first entry, end, inclusive prefix of column spans
    uint32_t *rend;
    uint32_t *rspan;
    int n;
};

// Row-level LDS state shared by the run workers.
struct RowShared {
    int32_t *sa;        // footprint counts -> per-column record counts / bases
    int32_t *sb;        // claim counts -> per-column fill counters
    uint32_t *sx;       // claimant xor -> pixel class
    uint32_t *locfill;  // row-local fill counter of the local-edge array
    uint32_t *nruns;
};

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
    for (int q = sp - 1; q >= i && (int)(D.pm[q] >> 16) > col; --q)
        if ((int)(D.c[q] >> 16) >= col && !(D.f[q] & F_HORIZ)) ++nloc;
    if (nloc > 0x7fffu || npart > 0x7fffu) atomicOr(A.errflags, 16u);
    if (!EMIT) {
        atomicAdd(&L.sa[cix(col)], 1);
        nloc_tot += nloc;
        return;
    }
    const uint64_t slot = rec_base_r + (uint64_t)L.sa[cix(col)] + (uint64_t)atomicAdd(&L.sb[cix(col)], 1);
    uint64_t eoff = 0;
    if (nloc) {
        eoff = loc_base_r + atomicAdd(L.locfill, nloc);
        uint64_t o = eoff;
        for (int q = sp - 1; q >= i && (int)(D.pm[q] >> 16) > col; --q)
            if ((int)(D.c[q] >> 16) >= col && !(D.f[q] & F_HORIZ)) A.ledges[o++] = A.edges[D.edge[q]];
    }
    Cand cd;
    cd.poly = D.poly[i];
    cd.meta = S | ((nloc & 0x7fffu) << 2) | ((npart & 0x7fffu) << 17);
    cd.eoff = (uint32_t)eoff;
    cd.poff = (uint32_t)(part_base_r + (ps & 0x7fffffffu));
    A.cands[slot] = cd;
}

// Claimant records of a run in rows where interiors overlap: every boundary
// column inside the run's interior spans gets (S = 1, no edges).
template <bool EMIT>
__device__ void claimant_walk(const RowArgs &A, const RowData &D, const RowShared &L, int i, int je,
                              uint64_t rec_base_r)
{
    const int W = A.m.W;
    uint32_t par = 0;
    for (int q = i; q < je; ++q) par ^= (D.f[q] & F_W) ? 1u : 0u;
    auto emit = [&](int col) {
        if (!EMIT) { atomicAdd(&L.sa[cix(col)], 1); return; }
        const uint64_t slot = rec_base_r + (uint64_t)L.sa[cix(col)] + (uint64_t)atomicAdd(&L.sb[cix(col)], 1);
        Cand cd;
        cd.poly = D.poly[i];
        cd.meta = CAND_S;
        cd.eoff = 0;
        cd.poff = 0;
        A.cands[slot] = cd;
    };
    int mx = -1;
    const int c0first = (int)(D.c[i] & 0xffff);
    if (par)
        for (int col = 0; col < c0first; ++col)
            if (L.sx[cix(col)] & BFLAG) emit(col);
    for (int q = i; q < je; ++q) {
        const uint32_t c = D.c[q];
        mx = max(mx, (int)(c >> 16));
        if (D.f[q] & F_W) par ^= 1u;
        const int nc0 = (q + 1 < je) ? (int)(D.c[q + 1] & 0xffff) : W;
        const int lo = max((int)(c & 0xffff), mx + 1), hi = nc0 - 1;
        if (par)
            for (int col = lo; col <= hi; ++col)
                if (L.sx[cix(col)] & BFLAG) emit(col);
    }
}

// Calls fn(i, je) for every run (maximal block of entries of one polygon)
// whose first entry this thread owns.
template <typename Fn>
__device__ __forceinline__ void for_each_run(const RowData &D, Fn fn)
{
    for (int i = threadIdx.x; i < D.n; i += ROW_THREADS) {
        const uint32_t k = D.poly[i];
        if (i != 0 && D.poly[i - 1] == k) continue;
        int je = i + 1;
        while (je < D.n && D.poly[je] == k) ++je;
        fn(i, je);
    }
}

// Block-wide in-place inclusive scan of a[0..n) under an associative,
// commutative operator.
template <typename Op>
__device__ void block_plain_scan(uint32_t *a, int n, uint32_t *wtot, Op op)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + ROW_THREADS - 1) / ROW_THREADS;
    const int b = min(n, tid * per), e = min(n, b + per);
    uint32_t acc = 0;
    for (int q = b; q < e; ++q) { acc = op(acc, a[q]); a[q] = acc; }
    uint32_t inc = acc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc = op(inc, t);
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int q = 0; q < wv; ++q) pre = op(pre, wtot[q]);
    uint32_t prev = __shfl_up(inc, 1, 64);
    if (lane > 0) pre = op(pre, prev);
    for (int q = b; q < e; ++q) a[q] = op(pre, a[q]);
    __syncthreads();
}

// Runs every (run, column) item of the row through column_record.
template <bool EMIT>
__device__ void all_column_records(const RowArgs &A, const RowData &D, const RowShared &L,
                                   uint64_t rec_base_r, uint64_t loc_base_r, uint64_t part_base_r,
                                   uint64_t &nloc_tot)
{
    const int nr = (int)*L.nruns;
    if (nr == 0) return;
    const uint32_t total = D.rspan[nr - 1];
    for (uint32_t t = threadIdx.x; t < total; t += ROW_THREADS) {
        int lo = 0, hi = nr - 1;            // first run with rspan > t
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (D.rspan[mid] > t) hi = mid; else lo = mid + 1;
        }
        const int i = (int)D.rhead[lo], je = (int)D.rend[lo];
        const uint32_t before = lo ? D.rspan[lo - 1] : 0u;
        const int col = (int)(D.c[i] & 0xffff) + (int)(t - before);
        column_record<EMIT>(A, D, L, i, je, col, rec_base_r, loc_base_r, part_base_r, nloc_tot);
    }
}

// Dynamic LDS: three padded column arrays, then `cap` staged entries with
// their auxiliary words, then the run list (at most cap / 2 runs).
__host__ __device__ inline size_t row_lds_bytes(int W, int cap)
{
    return (size_t)3 * col_words(W) * 4 + (size_t)cap * 21 + (size_t)(cap / 2 + 1) * 12 + 32;
}

template <bool EMIT>
__device__ void process_row(const RowArgs &A, const RowData &D, const RowShared &L, int r,
                            int32_t *wtoti, uint32_t *wtotu, uint32_t *s_nbp, uint32_t *s_multi,
                            unsigned long long *s_nloc, unsigned long long *s_nrec)
{
    const int W = A.m.W;
    const int tid = threadIdx.x;

    // phase 1: per run, footprints (boundary counts), interior claims, the
    //          running footprint maxima and the run list; per entry, the
    //          partial / spanning indicators to be scanned
    for (int q = tid; q < D.n; q += ROW_THREADS) D.pre[q] = pre_own(D.f[q]);
    for_each_run(D, [&](int i, int je) {
        const uint32_t lab = D.poly[i] + 1;
        uint32_t wtot = 0;
        for (int q = i; q < je; ++q) wtot ^= (D.f[q] & F_W) ? 1u : 0u;
        uint32_t par = wtot;
        int mx = -1;
        uint32_t mall = 0, mnh = 0;
        const int c0first = (int)(D.c[i] & 0xffff);
        if (par && c0first > 0) {
            atomicAdd(&L.sb[cix(0)], 1); atomicSub(&L.sb[cix(c0first)], 1);
            atomicXor(&L.sx[cix(0)], lab); atomicXor(&L.sx[cix(c0first)], lab);
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
                atomicXor(&L.sx[cix(lo)], lab); atomicXor(&L.sx[cix(hi + 1)], lab);
            }
        }
        const uint32_t j = atomicAdd(L.nruns, 1u);
        D.rhead[j] = (uint32_t)i;
        D.rend[j] = (uint32_t)je;
        D.rspan[j] = (uint32_t)((int)mall - c0first);   // columns c0first .. max c1
    });
    __syncthreads();

    // phase 2: prefix scans -> per-pixel boundary count, claim count,
    //          claimant; per-entry partial/spanning prefixes; run spans
    block_scan(L.sa, W, wtoti, [](int32_t a, int32_t b) { return a + b; }, 0);
    block_scan(L.sb, W, wtoti, [](int32_t a, int32_t b) { return a + b; }, 0);
    block_scan(L.sx, W, wtotu, [](uint32_t a, uint32_t b) { return a ^ b; }, 0u);
    block_plain_scan(D.pre, D.n, wtotu, [](uint32_t a, uint32_t b) { return pre_op(a, b); });
    block_plain_scan(D.rspan, (int)*L.nruns, wtotu, [](uint32_t a, uint32_t b) { return a + b; });

    // phase 3: classify pixels.  sx := 0 (no polygon), label + 1, or for a
    // boundary pixel BFLAG | (label + 1 of its single interior claimant, or 0);
    // sa := per-column record counters, starting with the claimant record.
    uint32_t nb = 0, multi = 0;
    for (int c = tid; c < W; c += ROW_THREADS) {
        const int32_t bc = L.sa[cix(c)], cc = L.sb[cix(c)];
        const uint32_t xc = L.sx[cix(c)];
        const bool bnd = bc > 0 || cc >= 2;
        L.sx[cix(c)] = bnd ? (BFLAG | (cc == 1 ? xc : 0u)) : (cc == 1 ? xc : 0u);
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
        for (int c = tid; c < W; c += ROW_THREADS) L.sa[cix(c)] = 0;
        __syncthreads();
    }

    // phase 4: count records per column (and local-edge totals)
    uint64_t nloc = 0;
    all_column_records<false>(A, D, L, 0, 0, 0, nloc);
    if (rmulti) for_each_run(D, [&](int i, int je) { claimant_walk<false>(A, D, L, i, je, 0); });
    atomicAdd(s_nloc, (unsigned long long)nloc);
    __syncthreads();

    if (!EMIT) {
        uint32_t nrec = 0;
        for (int c = tid; c < W; c += ROW_THREADS) nrec += (uint32_t)L.sa[cix(c)];
        atomicAdd(s_nrec, (unsigned long long)nrec);
        __syncthreads();
        if (tid == 0) {
            A.row_nrec[r] = *s_nrec;
            A.row_nloc[r] = *s_nloc;
            A.row_npart[r] = D.n ? (D.pre[D.n - 1] & 0x7fffffffu) : 0u;
            A.row_nbp[r] = *s_nbp;
        }
        return;
    }

    // exclusive column bases for the records of this row
    block_scan(L.sa, W, wtoti, [](int32_t a, int32_t b) { return a + b; }, 0);
    {
        int32_t mine[MAXW / ROW_THREADS];
        int cnt = 0;
        for (int c = tid; c < W; c += ROW_THREADS) mine[cnt++] = (c == 0) ? 0 : L.sa[cix(c - 1)];
        __syncthreads();
        cnt = 0;
        for (int c = tid; c < W; c += ROW_THREADS) { L.sa[cix(c)] = mine[cnt++]; L.sb[cix(c)] = 0; }
        __syncthreads();
    }

    // phase 5: records, local edges, partial spans (in row entry order)
    const uint64_t rec_base_r = A.rec_base[r], loc_base_r = A.loc_base[r], part_base_r = A.part_base[r];
    {
        uint64_t dummy = 0;
        all_column_records<true>(A, D, L, rec_base_r, loc_base_r, part_base_r, dummy);
        if (rmulti) for_each_run(D, [&](int i, int je) { claimant_walk<true>(A, D, L, i, je, rec_base_r); });
        else
            for (int c = tid; c < W; c += ROW_THREADS) {
                const uint32_t w = L.sx[cix(c)];
                if ((w & BFLAG) && (w & ~BFLAG)) {
                    const uint64_t slot = rec_base_r + (uint64_t)L.sa[cix(c)] + (uint64_t)atomicAdd(&L.sb[cix(c)], 1);
                    Cand cd;
                    cd.poly = (w & ~BFLAG) - 1u;
                    cd.meta = CAND_S;
                    cd.eoff = 0;
                    cd.poff = 0;
                    A.cands[slot] = cd;
                }
            }
        for (int q = tid; q < D.n; q += ROW_THREADS)
            if (is_partial(D.f[q])) {
                const Edge e = A.edges[D.edge[q]];
                A.pspan[part_base_r + (pre_excl(D, q) & 0x7fffffffu)] = make_double2(e.ylo, e.yhi);
            }
    }
    __syncthreads();

    // phase 6: order each pixel's records by polygon, flag the last one,
    //          write the canvas row (tile-major)
    for (int c = tid; c < W; c += ROW_THREADS) {
        uint32_t word = L.sx[cix(c)];
        if (word & BFLAG) {
            const uint64_t base = rec_base_r + (uint64_t)L.sa[cix(c)];
            const int n = L.sb[cix(c)];
            if (n <= 0) { atomicOr(A.errflags, 8u); word = 0; }
            else {
                Cand *cs = A.cands + base;
                for (int a = 1; a < n; ++a) {
                    Cand key = cs[a];
                    int b = a - 1;
                    while (b >= 0 && cs[b].poly > key.poly) { cs[b + 1] = cs[b]; --b; }
                    cs[b + 1] = key;
                }
                cs[n - 1].meta |= CAND_LAST;
                word = BFLAG | (uint32_t)base;
            }
        }
        A.cells[tile_index(A.Wt, c, r)] = word;
    }
}

template <bool EMIT>
__global__ __launch_bounds__(ROW_THREADS) void k_rows(RowArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t wtoti[ROW_THREADS / 64];
    __shared__ uint32_t wtotu[ROW_THREADS / 64];
    __shared__ uint32_t s_locfill, s_nruns, s_nbp, s_multi;
    __shared__ unsigned long long s_nloc, s_nrec;
    const int W = A.m.W, H = A.m.H, cap = A.cap;
    const int cw = col_words(W);
    RowShared L;
    L.sa = (int32_t *)smem;
    L.sb = L.sa + cw;
    L.sx = (uint32_t *)(L.sb + cw);
    L.locfill = &s_locfill;
    L.nruns = &s_nruns;
    uint32_t *lpoly = L.sx + cw;
    uint32_t *lc = lpoly + cap;
    uint32_t *ledge = lc + cap;
    uint32_t *lpm = ledge + cap;
    uint32_t *lpre = lpm + cap;
    uint32_t *lrh = lpre + cap;
    uint32_t *lre = lrh + (cap / 2 + 1);
    uint32_t *lrs = lre + (cap / 2 + 1);
    uint8_t *lf = (uint8_t *)(lrs + (cap / 2 + 1));
    const int tid = threadIdx.x;

    for (int r = blockIdx.x; r < H; r += gridDim.x) {
        const int s = (int)A.row_off[r], e = (int)A.row_off[r + 1];
        const int n = e - s;
        if (n <= cap) {
            for (int q = tid; q < n; q += ROW_THREADS) {
                lpoly[q] = A.spoly[s + q];
                lc[q] = A.sc[s + q];
                ledge[q] = A.sedge[s + q];
                lf[q] = A.sf[s + q];
            }
        }
        for (int c = tid; c < cw; c += ROW_THREADS) { L.sa[c] = 0; L.sb[c] = 0; L.sx[c] = 0; }
        if (tid == 0) { s_locfill = 0; s_nruns = 0; s_nbp = 0; s_multi = 0; s_nloc = 0; s_nrec = 0; }
        __syncthreads();
        if (n <= cap) {
            const RowData D{lpoly, lc, lf, ledge, lpm, lpre, lrh, lre, lrs, n};
            process_row<EMIT>(A, D, L, r, wtoti, wtotu, &s_nbp, &s_multi, &s_nloc, &s_nrec);
        } else {
            uint32_t *g = A.gaux + (size_t)5 * s;
            const RowData D{A.spoly + s, A.sc + s, A.sf + s, A.sedge + s, g, g + n, g + 2 * n, g + 3 * n,
                            g + 4 * n, n};
            process_row<EMIT>(A, D, L, r, wtoti, wtotu, &s_nbp, &s_multi, &s_nloc, &s_nrec);
        }
        __syncthreads();
    }
}

// Coarse canvas: one 16-bit word per B x B block of pixels (B = 2^blog >= 16),
// holding the block's common label + 1 (0: in no polygon) when every pixel
// of the block carries that same non-boundary value, else COARSE_MIXED.  One
// wavefront per block.
__global__ __launch_bounds__(256) void k_coarse(int W, int H, int Wt, int blog, int Wc, int Hc,
                                                const uint32_t *cells, uint16_t *coarse)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int B = 1 << blog;
    for (int64_t cell = wave; cell < (int64_t)Wc * Hc; cell += nw) {
        const int cy = (int)(cell / Wc), cx = (int)(cell % Wc);
        const int c0 = cx << blog, r0 = cy << blog;
        const int cw = min(B, W - c0), ch = min(B, H - r0);
        const uint32_t first = cells[tile_index(Wt, c0, r0)];
        bool same = true;
        for (int p = lane; p < cw * ch; p += 64) {
            const int c = c0 + p % cw, r = r0 + p / cw;
            same &= cells[tile_index(Wt, c, r)] == first;
        }
        const bool all = __all(same);
        if (lane == 0)
            coarse[cell] = (all && !(first & BFLAG) && first < COARSE_MIXED) ? (uint16_t)first : COARSE_MIXED;
    }
}

// ------------------------------------------------------------ host driver

static int bits_for(uint64_t v)   // bits needed to store values 0..v
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

static int grid_for(int64_t n, int64_t cap = 65536)
{
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

int build_canvas(spade_ctx *ctx, const spade_polys *polys, spade_canvas *cv)
{
    hipStream_t st = ctx->stream;
    const int64_t M = polys->n_polys, R = polys->n_rings;
    CanvasView &view = cv->view;
    view = CanvasView{};
    view.M = M;
    view.bx0 = INFINITY; view.by0 = INFINITY; view.bx1 = -INFINITY; view.by1 = -INFINITY;

    // vertex count
    int64_t V = 0;
    if (R > 0) {
        int64_t *h = (int64_t *)ensure_pinned(ctx, 64);
        if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
        SPADE_HIP(ctx, hipMemcpyAsync(h, polys->ring_vtx_off + R, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        V = h[0];
        if (V < 0) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off[n_rings] is negative");
        if (V >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "more than 2^32-1 vertices");
    }

    // validation + ring->polygon + bbox
    DevBuf &rp = ctx->scratch[S_RINGPOLY];
    DevBuf &br = ctx->scratch[S_BLOCKRED];
    if (ensure(ctx, rp, sizeof(int32_t) * (size_t)std::max<int64_t>(R, 1)) ||
        ensure(ctx, br, sizeof(double) * 4 * RED_BLOCKS + 64))
        return SPADE_E_NOMEM;
    unsigned *d_err = (unsigned *)((char *)br.p + sizeof(double) * 4 * RED_BLOCKS);
    SPADE_HIP(ctx, hipMemsetAsync(d_err, 0, sizeof(unsigned), st));
    if (M > 0 || R > 0 || V > 0) {
        hipLaunchKernelGGL(k_validate, dim3(RED_BLOCKS), dim3(256), 0, st, M, R, polys->poly_ring_off,
                           polys->ring_vtx_off, V, polys->vx, polys->vy, (int32_t *)rp.p,
                           (double *)br.p, d_err);
        SPADE_HIP(ctx, hipGetLastError());
    }
    double *hred = (double *)ensure_pinned(ctx, sizeof(double) * 4 * RED_BLOCKS + 64);
    if (!hred) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(hred, br.p, sizeof(double) * 4 * RED_BLOCKS + sizeof(unsigned),
                                  hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    unsigned herr = 0;
    std::memcpy(&herr, (char *)hred + sizeof(double) * 4 * RED_BLOCKS, sizeof(unsigned));
    if (herr & 1u) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off must start at 0 and be non-decreasing");
    if (herr & 2u) return set_error(ctx, SPADE_E_INVALID, "poly_ring_off must start at 0, be non-decreasing and end at n_rings");
    if (herr & 4u) return set_error(ctx, SPADE_E_INVALID, "non-finite polygon vertex coordinate");
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    if (V > 0) {
        for (int b = 0; b < RED_BLOCKS; ++b) {
            x0 = std::min(x0, hred[b * 4 + 0]); x1 = std::max(x1, -hred[b * 4 + 1]);
            y0 = std::min(y0, hred[b * 4 + 2]); y1 = std::max(y1, -hred[b * 4 + 3]);
        }
    }

    // canvas size and map
    const bool empty = !(V > 0 && x0 < x1 && y0 < y1);
    int W = 1, H = 1;
    if (!empty) {
        if (ctx->canvas_w > 0 && ctx->canvas_h > 0) {
            W = ctx->canvas_w; H = ctx->canvas_h;
        } else {
            const double aspect = (x1 - x0) / (y1 - y0);
            const double target = 4096.0 * 4096.0;
            double w = std::sqrt(target * aspect);
            W = (int)std::max(1.0, std::min((double)MAXW, std::round(w)));
            H = (int)std::max(1.0, std::min(65535.0, std::round(target / W)));
        }
    }
    if (W > MAXW || H > 65535) return set_error(ctx, SPADE_E_UNSUPPORTED, "canvas larger than 8192 x 65535");
    Map m;
    m.W = W; m.H = H;
    if (!empty) {
        m.X0 = x0; m.Y0 = y0;
        m.sx = (double)W / (x1 - x0);
        m.sy = (double)H / (y1 - y0);
        m.hy = (y1 - y0) / (double)H;
        view.bx0 = x0; view.bx1 = x1; view.by0 = y0; view.by1 = y1;
    } else {
        m.X0 = 0; m.Y0 = 0; m.sx = 0; m.sy = 0; m.hy = 0;
    }
    view.X0 = m.X0; view.Y0 = m.Y0; view.sx = m.sx; view.sy = m.sy;
    view.W = W; view.H = H;

    const int Wt = (W + 15) / 16, Ht = (H + 15) / 16;
    view.Wt = Wt;
    const size_t ncells = (size_t)Wt * Ht * 256;
    if (ensure(ctx, cv->cells, sizeof(uint32_t) * ncells)) return SPADE_E_NOMEM;
    view.cells = (const uint32_t *)cv->cells.p;
    // coarse grid: blocks of 2^blog pixels, as fine as the probe's LDS allows
    int blog = 4;
    const size_t cbudget = coarse_lds_budget(M);
    while (blog < 15 && (size_t)((W + (1 << blog) - 1) >> blog) * ((H + (1 << blog) - 1) >> blog) * 2 > cbudget)
        ++blog;
    view.blog = blog;
    view.Wc = (W + (1 << blog) - 1) >> blog;
    view.Hc = (H + (1 << blog) - 1) >> blog;
    if (ensure(ctx, cv->coarse, sizeof(uint16_t) * ((size_t)view.Wc * view.Hc + 2))) return SPADE_E_NOMEM;
    view.coarse = (const uint16_t *)cv->coarse.p;
    if (ensure(ctx, cv->edges, sizeof(Edge) * (size_t)std::max<int64_t>(V, 1))) return SPADE_E_NOMEM;
    cv->n_edges = V;
    if (empty) {
        SPADE_HIP(ctx, hipMemsetAsync(cv->cells.p, 0, sizeof(uint32_t) * ncells, st));
        SPADE_HIP(ctx, hipMemsetAsync(cv->coarse.p, 0, sizeof(uint16_t) * ((size_t)view.Wc * view.Hc + 2), st));
        if (ensure(ctx, cv->cands, sizeof(Cand)) || ensure(ctx, cv->ledges, sizeof(Edge)) ||
            ensure(ctx, cv->pspan, sizeof(double2)))
            return SPADE_E_NOMEM;
        view.cands = (const Cand *)cv->cands.p;
        view.ledges = (const Edge *)cv->ledges.p;
        view.pspan = (const double2 *)cv->pspan.p;
        cv->n_boundary = cv->n_cands = cv->n_elist = 0;
        return SPADE_OK;
    }

    // edges + per-edge row counts
    DevBuf &dn = ctx->scratch[S_NROWS];
    DevBuf &dmisc = ctx->scratch[S_MISC];
    const size_t Vs = (size_t)V;
    // misc: epoly[V] u32 | erow0[V] i32 | off[V+1] u64
    if (ensure(ctx, dn, sizeof(uint64_t) * (Vs + 1)) ||
        ensure(ctx, dmisc, sizeof(uint32_t) * Vs * 2 + sizeof(uint64_t) * (Vs + 2)))
        return SPADE_E_NOMEM;
    uint64_t *nrows = (uint64_t *)dn.p;
    uint32_t *epoly = (uint32_t *)dmisc.p;
    int32_t *erow0 = (int32_t *)(epoly + Vs);
    uint64_t *eoff = (uint64_t *)(((uintptr_t)(erow0 + Vs) + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_edges, dim3(grid_for(V)), dim3(256), 0, st, R, polys->ring_vtx_off, V,
                       polys->vx, polys->vy, (const int32_t *)rp.p, m, (Edge *)cv->edges.p, epoly,
                       erow0, nrows);
    SPADE_HIP(ctx, hipGetLastError());
    SPADE_HIP(ctx, hipMemsetAsync(nrows + V, 0, sizeof(uint64_t), st));

    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, nrows, eoff, (int)(V + 1), st));
    if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, nrows, eoff, (int)(V + 1), st));
    uint64_t *hT = (uint64_t *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(hT, eoff + V, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const uint64_t T = hT[0];
    if (T >= 0x7fffffffULL) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many (edge,row) entries; lower the canvas height");

    const int cbits = std::max(1, bits_for((uint64_t)W - 1));
    const int pbits = std::max(1, bits_for((uint64_t)std::max<int64_t>(M - 1, 0)));
    const int rbits = std::max(1, bits_for((uint64_t)H - 1));
    if (cbits + pbits + rbits > 64) return set_error(ctx, SPADE_E_UNSUPPORTED, "sort key exceeds 64 bits");

    DevBuf &dk = ctx->scratch[S_KEYS], &dk2 = ctx->scratch[S_KEYS2];
    DevBuf &dv = ctx->scratch[S_VALS], &dv2 = ctx->scratch[S_VALS2];
    DevBuf &dc = ctx->scratch[S_ENTC], &df = ctx->scratch[S_ENTF];
    DevBuf &drow = ctx->scratch[S_ROWOFF], &drc = ctx->scratch[S_ROWCNT];
    const size_t Ts = (size_t)std::max<uint64_t>(T, 1);
    // dc: ent_c[T] | sorted c[T] | perm[T] | perm2[T]; df: ent_f[T] | sorted f[T]
    if (ensure(ctx, dk, 8 * Ts) || ensure(ctx, dk2, 8 * Ts) || ensure(ctx, dv, 4 * Ts) ||
        ensure(ctx, dv2, 4 * Ts) || ensure(ctx, dc, 20 * Ts) || ensure(ctx, df, 2 * Ts + 16) ||
        ensure(ctx, drow, 4 * ((size_t)H + 1)) ||
        ensure(ctx, drc, 8 * 8 * ((size_t)H + 1)))
        return SPADE_E_NOMEM;
    uint32_t *ent_c = (uint32_t *)dc.p, *s_c = ent_c + Ts, *perm = s_c + Ts, *perm2 = perm + Ts;
    uint32_t *s_poly = perm2 + Ts;
    uint8_t *ent_f = (uint8_t *)df.p, *s_f = ent_f + Ts;
    hipLaunchKernelGGL(k_entries, dim3(grid_for(V)), dim3(256), 0, st, V, (const Edge *)cv->edges.p,
                       epoly, erow0, nrows, eoff, m, cbits, pbits, (uint64_t *)dk.p, (uint32_t *)dv.p,
                       ent_c, ent_f);
    SPADE_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_iota, dim3(grid_for((int64_t)T)), dim3(256), 0, st, (int64_t)T, perm);
    SPADE_HIP(ctx, hipGetLastError());

    // sort entries by (row, polygon, c0); stable, so ties keep edge order.
    const int kbits = cbits + pbits + rbits;
    {
        // sort (key, perm) to get the permutation, then gather edge ids and payload
        size_t tbytes = 0;
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, (const uint64_t *)dk.p,
                                                          (uint64_t *)dk2.p, (const uint32_t *)perm,
                                                          perm2, (int)T, 0, kbits, st));
        if (ensure(ctx, cub, tbytes)) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub.p, tbytes, (const uint64_t *)dk.p,
                                                          (uint64_t *)dk2.p, (const uint32_t *)perm,
                                                          perm2, (int)T, 0, kbits, st));
    }
    // sorted edge ids: vals[perm2[i]]
    hipLaunchKernelGGL(k_gather_entries, dim3(grid_for((int64_t)T)), dim3(256), 0, st, (int64_t)T,
                       perm2, ent_c, ent_f, (const uint64_t *)dk2.p, cbits,
                       (pbits >= 64) ? ~0ULL : ((1ULL << pbits) - 1), s_c, s_f, s_poly);
    SPADE_HIP(ctx, hipGetLastError());
    uint32_t *s_edge = (uint32_t *)dv2.p;
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_for((int64_t)T)), dim3(256), 0, st, (int64_t)T,
                       (const uint32_t *)perm2, (const uint32_t *)dv.p, s_edge);
    SPADE_HIP(ctx, hipGetLastError());
    const int rshift = cbits + pbits;
    hipLaunchKernelGGL(k_row_off, dim3(grid_for((int64_t)T + 1)), dim3(256), 0, st, (int64_t)T,
                       (const uint64_t *)dk2.p, rshift, H, (uint32_t *)drow.p);
    SPADE_HIP(ctx, hipGetLastError());

    uint64_t *row_nrec = (uint64_t *)drc.p;
    uint64_t *row_nloc = row_nrec + (H + 1);
    uint64_t *row_npart = row_nloc + (H + 1);
    uint64_t *row_nbp = row_npart + (H + 1);
    uint64_t *rec_base = row_nbp + (H + 1);
    uint64_t *loc_base = rec_base + (H + 1);
    uint64_t *part_base = loc_base + (H + 1);
    uint64_t *bp_scan = part_base + (H + 1);
    SPADE_HIP(ctx, hipMemsetAsync(drc.p, 0, 8 * 8 * ((size_t)H + 1), st));

    RowArgs ra{};
    ra.m = m;
    ra.Wt = Wt;
    ra.row_off = (const uint32_t *)drow.p;
    ra.spoly = s_poly;
    ra.sedge = s_edge;
    ra.sc = s_c;
    ra.sf = s_f;
    ra.edges = (const Edge *)cv->edges.p;
    ra.row_nrec = row_nrec; ra.row_nloc = row_nloc; ra.row_npart = row_npart; ra.row_nbp = row_nbp;
    ra.rec_base = rec_base; ra.loc_base = loc_base; ra.part_base = part_base;
    ra.errflags = d_err;
    // stage up to `cap` entries of a row in LDS; aim for two workgroups per CU
    const size_t col_bytes = row_lds_bytes(W, 0);
    const size_t target = (col_bytes <= 60 * 1024) ? 78 * 1024 : 150 * 1024;
    ra.cap = (int)std::max<size_t>(256, (target - std::min(target - 256 * 27, col_bytes)) / 27);
    if (T > (uint64_t)ra.cap) {
        // some row may exceed the LDS stage: global auxiliary words for it
        if (ensure(ctx, ctx->scratch[S_NEXTP], sizeof(uint32_t) * 5 * Ts)) return SPADE_E_NOMEM;
        ra.gaux = (uint32_t *)ctx->scratch[S_NEXTP].p;
    }
    const size_t rlds = row_lds_bytes(W, ra.cap);
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_rows<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_rows<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds));
    const int rgrid = std::min(H, 8192);
    hipLaunchKernelGGL(k_rows<false>, dim3(rgrid), dim3(ROW_THREADS), rlds, st, ra);
    SPADE_HIP(ctx, hipGetLastError());

    // per-row bases (exclusive scans over H+1 entries with a zero tail)
    tb = 0;
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
    const uint64_t nrec = hs[0], nloc = hs[1], npart = hs[2], nbp = hs[3];
    if (nrec >= (uint64_t)BFLAG) return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary index exceeds 2^31 records; lower the canvas resolution");
    if (nloc >= 0xffffffffULL || npart >= 0xffffffffULL)
        return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary edge lists exceed 2^32 entries");
    if (ensure(ctx, cv->cands, sizeof(Cand) * (size_t)std::max<uint64_t>(nrec, 1)) ||
        ensure(ctx, cv->ledges, sizeof(Edge) * (size_t)std::max<uint64_t>(nloc, 1)) ||
        ensure(ctx, cv->pspan, sizeof(double2) * (size_t)std::max<uint64_t>(npart, 1)))
        return SPADE_E_NOMEM;
    ra.cells = (uint32_t *)cv->cells.p;
    ra.cands = (Cand *)cv->cands.p;
    ra.ledges = (Edge *)cv->ledges.p;
    ra.pspan = (double2 *)cv->pspan.p;
    hipLaunchKernelGGL(k_rows<true>, dim3(rgrid), dim3(ROW_THREADS), rlds, st, ra);
    SPADE_HIP(ctx, hipGetLastError());
    {
        const int64_t ncoarse = (int64_t)view.Wc * view.Hc;
        const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>((ncoarse + 3) / 4, 65536));
        hipLaunchKernelGGL(k_coarse, dim3(cgrid), dim3(256), 0, st, W, H, Wt, blog, view.Wc, view.Hc,
                           (const uint32_t *)cv->cells.p, (uint16_t *)cv->coarse.p);
        SPADE_HIP(ctx, hipGetLastError());
    }
    unsigned *herr2 = (unsigned *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(herr2, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (herr2[0] & 8u) return set_error(ctx, SPADE_E_HIP, "internal: boundary pixel without candidates");
    if (herr2[0] & 16u)
        return set_error(ctx, SPADE_E_UNSUPPORTED, "a boundary pixel has more than 32767 edges of one polygon; raise the canvas resolution");
    view.cands = (const Cand *)cv->cands.p;
    view.ledges = (const Edge *)cv->ledges.p;
    view.pspan = (const double2 *)cv->pspan.p;
    cv->n_boundary = (int64_t)nbp;
    cv->n_cands = (int64_t)nrec;
    cv->n_elist = (int64_t)(nloc + npart);
    return SPADE_OK;
}

}  // namespace spade
