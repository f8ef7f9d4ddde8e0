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
                                 const uint8_t *ent_f, uint32_t *s_c, uint8_t *s_f)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += nth) {
        uint32_t p = perm[i];
        s_c[i] = ent_c[p];
        s_f[i] = ent_f[p];
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

// In-place block-wide inclusive scan of a[0..n) (n <= MAXW) with 256 threads.
template <typename T, typename Op>
__device__ void block_scan(T *a, int n, T *tmp, Op op, T ident)
{
    const int per = (n + ROW_THREADS - 1) / ROW_THREADS;
    const int b = threadIdx.x * per;
    const int e = min(n, b + per);
    T acc = ident;
    for (int i = b; i < e; ++i) { acc = op(acc, a[i]); a[i] = acc; }
    tmp[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = ident;
        for (int t = 0; t < ROW_THREADS; ++t) { T v = tmp[t]; tmp[t] = run; run = op(run, v); }
    }
    __syncthreads();
    const T pre = tmp[threadIdx.x];
    for (int i = b; i < e; ++i) a[i] = op(pre, a[i]);
    __syncthreads();
}

struct RowArgs {
    Map m;
    int cbits;
    uint64_t pmask;
    const uint32_t *row_off;
    const uint64_t *skeys;
    const uint32_t *sedge;   // edge id per sorted entry
    const uint32_t *sc;      // c0 | c1 << 16
    const uint8_t *sf;
    uint32_t *nextp;         // next partial entry at or after i within its run
    const Edge *edges;
    // count pass
    uint64_t *row_nrec, *row_nel, *row_nbp;
    // emit pass
    const uint64_t *rec_base, *el_base;
    uint32_t *cells;
    Cand *cands;
    uint32_t *elist;
    unsigned *errflags;
};

// Emits (or counts) the records of one run (entries [i, je) of polygon k in
// row r).  `cls` holds the pixel classes of the row.
template <bool EMIT>
__device__ void run_records(const RowArgs &A, int r, int i, int je, uint32_t k,
                            const uint32_t *cls, int32_t *colcnt, int32_t *colfill,
                            uint32_t *elfill, uint64_t &nel)
{
    const int W = A.m.W;
    // spanning parity over the run and widest footprint
    uint32_t stot = 0, wtot = 0;
    int maxlen = 0;
    for (int q = i; q < je; ++q) {
        uint8_t f = A.sf[q];
        if ((f & F_SPAN) && !(f & F_HORIZ)) stot ^= 1u;
        if (f & F_W) wtot ^= 1u;
        uint32_t c = A.sc[q];
        maxlen = max(maxlen, (int)(c >> 16) - (int)(c & 0xffff));
    }
    auto emit = [&](int col, uint32_t S, int sp, int lp, bool with_edges) {
        // count locals and partials
        uint32_t nloc = 0, npart = 0;
        if (with_edges) {
            for (int q = lp; q < sp; ++q) {
                uint32_t c = A.sc[q];
                if ((int)(c >> 16) >= col && !(A.sf[q] & F_HORIZ)) ++nloc;
            }
            for (int q = (sp < je) ? (int)A.nextp[sp] : je; q < je; q = (q + 1 < je) ? (int)A.nextp[q + 1] : je)
                ++npart;
        }
        if (!EMIT) {
            atomicAdd(&colcnt[col], 1);
            nel += nloc + npart;
            return;
        }
        const uint64_t slot = A.rec_base[r] + (uint64_t)colcnt[col] + (uint64_t)atomicAdd(&colfill[col], 1);
        uint64_t eoff = 0;
        if (nloc + npart) {
            eoff = A.el_base[r] + atomicAdd(elfill, nloc + npart);
            uint64_t o = eoff;
            for (int q = lp; q < sp; ++q) {
                uint32_t c = A.sc[q];
                if ((int)(c >> 16) >= col && !(A.sf[q] & F_HORIZ)) A.elist[o++] = A.sedge[q];
            }
            for (int q = (sp < je) ? (int)A.nextp[sp] : je; q < je; q = (q + 1 < je) ? (int)A.nextp[q + 1] : je)
                A.elist[o++] = A.sedge[q];
        }
        Cand cd;
        cd.poly = k;
        cd.meta = (S & 1u) | (nloc << 2);
        cd.eoff = (uint32_t)eoff;
        cd.npart = npart;
        A.cands[slot] = cd;
    };

    // (a) every column of the union of the run's footprints
    {
        int col = (int)(A.sc[i] & 0xffff);
        int reach = -1, sp = i, lp = i;
        uint32_t sleft = 0;
        while (true) {
            while (sp < je && (int)(A.sc[sp] & 0xffff) <= col) {
                reach = max(reach, (int)(A.sc[sp] >> 16));
                uint8_t f = A.sf[sp];
                if ((f & F_SPAN) && !(f & F_HORIZ)) sleft ^= 1u;
                ++sp;
            }
            if (col > reach) {
                if (sp >= je) break;
                col = (int)(A.sc[sp] & 0xffff);
                continue;
            }
            while (lp < sp && (int)(A.sc[lp] & 0xffff) < col - maxlen) ++lp;
            emit(col, stot ^ sleft, sp, lp, true);
            if (++col >= W) break;
        }
    }
    // (b) interior columns of the run that are boundary pixels because of
    //     other polygons: the polygon covers the whole pixel (S = 1, no edges)
    {
        uint32_t par = wtot;
        int mx = -1;
        int c0first = (int)(A.sc[i] & 0xffff);
        if (par)
            for (int col = 0; col < c0first; ++col)
                if (cls[col] == BFLAG) emit(col, 1u, 0, 0, false);
        for (int q = i; q < je; ++q) {
            uint32_t c = A.sc[q];
            mx = max(mx, (int)(c >> 16));
            if (A.sf[q] & F_W) par ^= 1u;
            int nc0 = (q + 1 < je) ? (int)(A.sc[q + 1] & 0xffff) : W;
            int lo = max((int)(c & 0xffff), mx + 1), hi = nc0 - 1;
            if (par)
                for (int col = lo; col <= hi; ++col)
                    if (cls[col] == BFLAG) emit(col, 1u, 0, 0, false);
        }
    }
}

template <bool EMIT>
__global__ __launch_bounds__(ROW_THREADS) void k_rows(RowArgs A)
{
    __shared__ int32_t sa[MAXW + 1];
    __shared__ int32_t sb[MAXW + 1];
    __shared__ uint32_t sx[MAXW + 1];
    __shared__ int32_t tmpi[ROW_THREADS];
    __shared__ uint32_t tmpu[ROW_THREADS];
    __shared__ uint32_t s_elfill, s_nbp;
    __shared__ unsigned long long s_nel;
    const int W = A.m.W, H = A.m.H;
    const int tid = threadIdx.x;

    for (int r = blockIdx.x; r < H; r += gridDim.x) {
        const int s = (int)A.row_off[r], e = (int)A.row_off[r + 1];
        for (int c = tid; c <= W; c += ROW_THREADS) { sa[c] = 0; sb[c] = 0; sx[c] = 0; }
        if (tid == 0) { s_elfill = 0; s_nbp = 0; s_nel = 0; }
        __syncthreads();

        // phase 1: footprints (boundary counts) and interior claims per run
        for (int i = s + tid; i < e; i += ROW_THREADS) {
            const uint32_t k = (uint32_t)((A.skeys[i] >> A.cbits) & A.pmask);
            if (i != s && (uint32_t)((A.skeys[i - 1] >> A.cbits) & A.pmask) == k) continue;
            int je = i + 1;
            while (je < e && (uint32_t)((A.skeys[je] >> A.cbits) & A.pmask) == k) ++je;
            uint32_t wtot = 0;
            for (int q = i; q < je; ++q) wtot ^= (A.sf[q] & F_W) ? 1u : 0u;
            if (!EMIT) {
                int nxt = je;
                for (int q = je - 1; q >= i; --q) {
                    uint8_t f = A.sf[q];
                    if (!(f & F_SPAN) && !(f & F_HORIZ)) nxt = q;
                    A.nextp[q] = (uint32_t)nxt;
                }
            }
            uint32_t par = wtot;
            int mx = -1;
            const uint32_t lab = k + 1;
            int c0first = (int)(A.sc[i] & 0xffff);
            if (par && c0first > 0) {
                atomicAdd(&sb[0], 1); atomicSub(&sb[c0first], 1);
                atomicXor(&sx[0], lab); atomicXor(&sx[c0first], lab);
            }
            for (int q = i; q < je; ++q) {
                const uint32_t c = A.sc[q];
                const int c0 = (int)(c & 0xffff), c1 = (int)(c >> 16);
                atomicAdd(&sa[c0], 1);
                atomicSub(&sa[c1 + 1], 1);
                mx = max(mx, c1);
                if (A.sf[q] & F_W) par ^= 1u;
                const int nc0 = (q + 1 < je) ? (int)(A.sc[q + 1] & 0xffff) : W;
                const int lo = max(c0, mx + 1), hi = nc0 - 1;
                if (par && lo <= hi) {
                    atomicAdd(&sb[lo], 1); atomicSub(&sb[hi + 1], 1);
                    atomicXor(&sx[lo], lab); atomicXor(&sx[hi + 1], lab);
                }
            }
        }
        __syncthreads();

        // phase 2: prefix scans -> per-pixel boundary count, claim count, claimant
        block_scan(sa, W, tmpi, [](int32_t a, int32_t b) { return a + b; }, 0);
        block_scan(sb, W, tmpi, [](int32_t a, int32_t b) { return a + b; }, 0);
        block_scan(sx, W, tmpu, [](uint32_t a, uint32_t b) { return a ^ b; }, 0u);

        // phase 3: classify pixels; sx := class, sa := per-column record count
        uint32_t nb = 0;
        for (int c = tid; c < W; c += ROW_THREADS) {
            const bool bnd = sa[c] > 0 || sb[c] >= 2;
            sx[c] = bnd ? BFLAG : (sb[c] == 1 ? sx[c] : 0u);
            nb += bnd ? 1u : 0u;
        }
        atomicAdd(&s_nbp, nb);
        __syncthreads();
        for (int c = tid; c < W; c += ROW_THREADS) { sa[c] = 0; sb[c] = 0; }
        __syncthreads();

        // phase 4: count records per column (both passes need the counts)
        uint64_t nel = 0;
        for (int i = s + tid; i < e; i += ROW_THREADS) {
            const uint32_t k = (uint32_t)((A.skeys[i] >> A.cbits) & A.pmask);
            if (i != s && (uint32_t)((A.skeys[i - 1] >> A.cbits) & A.pmask) == k) continue;
            int je = i + 1;
            while (je < e && (uint32_t)((A.skeys[je] >> A.cbits) & A.pmask) == k) ++je;
            run_records<false>(A, r, i, je, k, sx, sa, sb, &s_elfill, nel);
        }
        atomicAdd(&s_nel, (unsigned long long)nel);
        __syncthreads();

        if (!EMIT) {
            uint32_t nrec = 0;
            for (int c = tid; c < W; c += ROW_THREADS) nrec += (uint32_t)sa[c];
            tmpu[tid] = nrec;
            __syncthreads();
            if (tid == 0) {
                uint64_t t = 0;
                for (int q = 0; q < ROW_THREADS; ++q) t += tmpu[q];
                A.row_nrec[r] = t;
                A.row_nel[r] = s_nel;
                A.row_nbp[r] = s_nbp;
            }
            __syncthreads();
            continue;
        }

        // exclusive column bases for the records of this row
        block_scan(sa, W, tmpi, [](int32_t a, int32_t b) { return a + b; }, 0);
        {
            int32_t mine[MAXW / ROW_THREADS];
            int cnt = 0;
            for (int c = tid; c < W; c += ROW_THREADS) mine[cnt++] = (c == 0) ? 0 : sa[c - 1];
            __syncthreads();
            cnt = 0;
            for (int c = tid; c < W; c += ROW_THREADS) { sa[c] = mine[cnt++]; sb[c] = 0; }
            __syncthreads();
        }

        // phase 5: emit records and edge ids
        for (int i = s + tid; i < e; i += ROW_THREADS) {
            const uint32_t k = (uint32_t)((A.skeys[i] >> A.cbits) & A.pmask);
            if (i != s && (uint32_t)((A.skeys[i - 1] >> A.cbits) & A.pmask) == k) continue;
            int je = i + 1;
            while (je < e && (uint32_t)((A.skeys[je] >> A.cbits) & A.pmask) == k) ++je;
            uint64_t dummy = 0;
            run_records<true>(A, r, i, je, k, sx, sa, sb, &s_elfill, dummy);
        }
        __syncthreads();

        // phase 6: order each pixel's records by polygon, flag the last one,
        //          write the canvas row
        for (int c = tid; c < W; c += ROW_THREADS) {
            uint32_t word = sx[c];
            if (word == BFLAG) {
                const uint64_t base = A.rec_base[r] + (uint64_t)sa[c];
                const int n = sb[c];
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
            A.cells[(size_t)r * W + c] = word;
        }
        __syncthreads();
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

    if (ensure(ctx, cv->cells, sizeof(uint32_t) * (size_t)W * H)) return SPADE_E_NOMEM;
    view.cells = (const uint32_t *)cv->cells.p;
    if (ensure(ctx, cv->edges, sizeof(Edge) * (size_t)std::max<int64_t>(V, 1))) return SPADE_E_NOMEM;
    view.edges = (const Edge *)cv->edges.p;
    cv->n_edges = V;
    if (empty) {
        SPADE_HIP(ctx, hipMemsetAsync(cv->cells.p, 0, sizeof(uint32_t) * (size_t)W * H, st));
        if (ensure(ctx, cv->cands, sizeof(Cand)) || ensure(ctx, cv->elist, sizeof(uint32_t))) return SPADE_E_NOMEM;
        view.cands = (const Cand *)cv->cands.p;
        view.elist = (const uint32_t *)cv->elist.p;
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
    DevBuf &dnext = ctx->scratch[S_NEXTP], &drow = ctx->scratch[S_ROWOFF], &drc = ctx->scratch[S_ROWCNT];
    const size_t Ts = (size_t)std::max<uint64_t>(T, 1);
    // dc: ent_c[T] | sorted c[T] | perm[T] | perm2[T]; df: ent_f[T] | sorted f[T]
    if (ensure(ctx, dk, 8 * Ts) || ensure(ctx, dk2, 8 * Ts) || ensure(ctx, dv, 4 * Ts) ||
        ensure(ctx, dv2, 4 * Ts) || ensure(ctx, dc, 16 * Ts) || ensure(ctx, df, 2 * Ts + 16) ||
        ensure(ctx, dnext, 4 * Ts) || ensure(ctx, drow, 4 * ((size_t)H + 1)) ||
        ensure(ctx, drc, 8 * 6 * ((size_t)H + 1)))
        return SPADE_E_NOMEM;
    uint32_t *ent_c = (uint32_t *)dc.p, *s_c = ent_c + Ts, *perm = s_c + Ts, *perm2 = perm + Ts;
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
                       perm2, ent_c, ent_f, s_c, s_f);
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
    uint64_t *row_nel = row_nrec + (H + 1);
    uint64_t *row_nbp = row_nel + (H + 1);
    uint64_t *rec_base = row_nbp + (H + 1);
    uint64_t *el_base = rec_base + (H + 1);
    SPADE_HIP(ctx, hipMemsetAsync(drc.p, 0, 8 * 6 * ((size_t)H + 1), st));

    RowArgs ra{};
    ra.m = m;
    ra.cbits = cbits;
    ra.pmask = (pbits >= 64) ? ~0ULL : ((1ULL << pbits) - 1);
    ra.row_off = (const uint32_t *)drow.p;
    ra.skeys = (const uint64_t *)dk2.p;
    ra.sedge = s_edge;
    ra.sc = s_c;
    ra.sf = s_f;
    ra.nextp = (uint32_t *)dnext.p;
    ra.edges = (const Edge *)cv->edges.p;
    ra.row_nrec = row_nrec; ra.row_nel = row_nel; ra.row_nbp = row_nbp;
    ra.rec_base = rec_base; ra.el_base = el_base;
    ra.errflags = d_err;
    const int rgrid = std::min(H, 4096);
    hipLaunchKernelGGL(k_rows<false>, dim3(rgrid), dim3(ROW_THREADS), 0, st, ra);
    SPADE_HIP(ctx, hipGetLastError());

    // per-row bases (inclusive scan shifted: scan H+1 entries with a zero tail)
    tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, row_nrec, rec_base, H + 1, st));
    if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nrec, rec_base, H + 1, st));
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nel, el_base, H + 1, st));
    // total boundary pixels: scan into the (unused) tail of row_nbp's neighbour
    uint64_t *bp_scan = el_base + (H + 1);
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, row_nbp, bp_scan, H + 1, st));
    uint64_t *hs = (uint64_t *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(hs + 0, rec_base + H, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipMemcpyAsync(hs + 1, el_base + H, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipMemcpyAsync(hs + 2, bp_scan + H, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const uint64_t nrec = hs[0], nel = hs[1], nbp = hs[2];
    if (nrec >= (uint64_t)BFLAG) return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary index exceeds 2^31 records; lower the canvas resolution");
    if (nel >= 0xffffffffULL) return set_error(ctx, SPADE_E_UNSUPPORTED, "boundary edge list exceeds 2^32 entries");
    if (ensure(ctx, cv->cands, sizeof(Cand) * (size_t)std::max<uint64_t>(nrec, 1)) ||
        ensure(ctx, cv->elist, sizeof(uint32_t) * (size_t)std::max<uint64_t>(nel, 1)))
        return SPADE_E_NOMEM;
    ra.cells = (uint32_t *)cv->cells.p;
    ra.cands = (Cand *)cv->cands.p;
    ra.elist = (uint32_t *)cv->elist.p;
    hipLaunchKernelGGL(k_rows<true>, dim3(rgrid), dim3(ROW_THREADS), 0, st, ra);
    SPADE_HIP(ctx, hipGetLastError());
    unsigned *herr2 = (unsigned *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(herr2, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (herr2[0] & 8u) return set_error(ctx, SPADE_E_HIP, "internal: boundary pixel without candidates");
    view.cands = (const Cand *)cv->cands.p;
    view.elist = (const uint32_t *)cv->elist.p;
    cv->n_boundary = (int64_t)nbp;
    cv->n_cands = (int64_t)nrec;
    cv->n_elist = (int64_t)nel;
    return SPADE_OK;
}

}  // namespace spade
