// Resident point tables and query batches.
//
// A table keeps the points in HBM sorted by the cell of a G x G grid over
// their bounding box (row-major cells) and cut into chunks of CHUNK points
// with their exact bounding boxes.  A batch is a canvas set (one canvas per
// query).  Work is organised by (chunk, query) pairs whose boxes overlap:
// one workgroup holds a chunk's points in registers and tests them against
// every query that can contain one of them, so a chunk is read from HBM once
// per pass for the whole batch.  Selection output uses the paper's two-step
// Map (Sec. 5.1): a count pass sizes every (chunk, query) pair, a scan places
// the pairs query by query, a write pass stores the ids, and a radix sort of
// (query, id) keys orders each query's ids.  The join-count needs no pair
// list: its single probe launch finds each chunk's queries itself.
#include "common.h"
#include "exact.h"
#include "lookup.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

namespace spade {

constexpr int CHUNK = 4096;               // table points per chunk
constexpr int BT_THREADS = 256;           // batch probe workgroup
constexpr int BT_PER = CHUNK / BT_THREADS;
constexpr int GRID_MAX = 1024;            // table grid side

}  // namespace spade

struct spade_table {
    int device = 0;
    int64_t n = 0;        // points
    int64_t nfin = 0;     // points with finite coordinates (clustered prefix)
    int G = 1;
    double X0 = 0, Y0 = 0, sx = 0, sy = 0;
    int64_t nchunk = 0;
    spade::DevBuf x, y, ids, cell_off, chunk_bb;
    size_t bytes() const { return x.cap + y.cap + ids.cap + cell_off.cap + chunk_bb.cap; }
};

namespace spade {

__device__ __forceinline__ unsigned long long okey(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

static double from_okey(unsigned long long k)
{
    const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

static int grid_of(int64_t n, int64_t cap = 65536)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

static int bits_of(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// Bounding box of the finite points: keys of (min x, -max x, min y, -max y).
__global__ __launch_bounds__(256) void k_pt_bbox(int64_t n, const double *X, const double *Y,
                                                 unsigned long long *bb)
{
    __shared__ unsigned long long s[4][256];
    unsigned long long k0 = ~0ull, k1 = ~0ull, k2 = ~0ull, k3 = ~0ull;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
        const double x = X[i], y = Y[i];
        if (!isfinite(x) || !isfinite(y)) continue;
        k0 = min(k0, okey(x)); k1 = min(k1, okey(-x));
        k2 = min(k2, okey(y)); k3 = min(k3, okey(-y));
    }
    s[0][threadIdx.x] = k0; s[1][threadIdx.x] = k1; s[2][threadIdx.x] = k2; s[3][threadIdx.x] = k3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = min(s[q][threadIdx.x], s[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 4) atomicMin(&bb[threadIdx.x], s[threadIdx.x][0]);
}

// Grid cell key of every point (non-finite points: G * G, sorted last).
// The bits of v (< 2^16) spread to the even bit positions.
__device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Sort key of each point: the Z-order (Morton) index of its cell of the
// G x G grid, so that runs of consecutive cells, and hence table chunks,
// are compact in space; nonfinite points get nfkey, after every cell.
__global__ void k_pt_key(int64_t n, const double *X, const double *Y, double X0, double Y0, double sx,
                         double sy, int G, uint32_t nfkey, uint32_t *keys, uint32_t *idx)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
        const double x = X[i], y = Y[i];
        uint32_t k = nfkey;
        if (isfinite(x) && isfinite(y)) {
            const int cx = (int)fmin((double)(G - 1), fmax(0.0, floor((x - X0) * sx)));
            const int cy = (int)fmin((double)(G - 1), fmax(0.0, floor((y - Y0) * sy)));
            k = spread_bits((uint32_t)cx) | (spread_bits((uint32_t)cy) << 1);
        }
        keys[i] = k;
        idx[i] = (uint32_t)i;
    }
}

__global__ void k_pt_gather(int64_t n, const uint32_t *perm, const double *X, const double *Y, double *x2,
                            double *y2)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
        const uint32_t p = perm[i];
        x2[i] = X[p];
        y2[i] = Y[p];
    }
}

// cell_off[c] = first sorted point of cell code c (c = 0 .. ncell + 1).
__global__ void k_cell_off(int64_t n, const uint32_t *skeys, int64_t ncell, uint32_t *cell_off)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += nth) {
        const int64_t ki = (i < n) ? (int64_t)skeys[i] : ncell;
        const int64_t kp = (i == 0) ? -1 : (int64_t)skeys[i - 1];
        for (int64_t c = kp + 1; c <= ki; ++c) cell_off[c] = (uint32_t)i;
    }
}

// Exact bounding box of every chunk of the finite prefix (one wave per chunk).
__global__ __launch_bounds__(256) void k_chunk_bb(int64_t nfin, int64_t nchunk, const double *X,
                                                  const double *Y, double4 *bb)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < nchunk; c += nw) {
        const int64_t b = c * CHUNK, e = std::min<int64_t>(nfin, b + CHUNK);
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int64_t i = b + lane; i < e; i += 64) {
            x0 = fmin(x0, X[i]); x1 = fmax(x1, X[i]);
            y0 = fmin(y0, Y[i]); y1 = fmax(y1, Y[i]);
        }
        for (int d = 32; d > 0; d >>= 1) {
            x0 = fmin(x0, __shfl_xor(x0, d, 64)); x1 = fmax(x1, __shfl_xor(x1, d, 64));
            y0 = fmin(y0, __shfl_xor(y0, d, 64)); y1 = fmax(y1, __shfl_xor(y1, d, 64));
        }
        if (lane == 0) bb[c] = make_double4(x0, y0, x1, y1);
    }
}

// ------------------------------------------------------------ pairs

// Chunk c can hold a point of canvas q: its closed point box meets the
// canvas's half-open polygon box.
__device__ __forceinline__ bool overlaps(const double4 &b, const CanvasDesc &d)
{
    return !d.empty && b.z >= d.bx0 && b.x < d.bx1 && b.w >= d.by0 && b.y < d.by1;
}

// Pass 1 counts overlapping chunks per canvas, pass 2 lists them (query-major).
template <bool FILL>
__global__ __launch_bounds__(256) void k_pairs(int nq, int64_t nchunk, const double4 *bb, const CanvasDesc *cds,
                                               unsigned long long *qcount, const unsigned long long *qbase,
                                               unsigned long long *qfill, uint32_t *pq, uint32_t *pc)
{
    for (int q = blockIdx.y; q < nq; q += gridDim.y) {
        const CanvasDesc d = cds[q];
        uint32_t mine = 0;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunk;
             c += (int64_t)gridDim.x * blockDim.x) {
            if (!overlaps(bb[c], d)) continue;
            if (!FILL) { ++mine; continue; }
            const unsigned long long p = qbase[q] + atomicAdd(&qfill[q], 1ull);
            pq[p] = (uint32_t)q;
            pc[p] = (uint32_t)c;
        }
        if (!FILL && mine) atomicAdd(&qcount[q], (unsigned long long)mine);
    }
}

// Chunk-major lists of pair ids (counting sort by chunk).
__global__ void k_pair_chunk_count(int64_t np, const uint32_t *pc, unsigned int *ccount)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += nth) atomicAdd(&ccount[pc[p]], 1u);
}

__global__ void k_pair_chunk_fill(int64_t np, const uint32_t *pc, const unsigned int *cbase, unsigned int *cfill,
                                  uint32_t *plist)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += nth) {
        const uint32_t c = pc[p];
        plist[cbase[c] + atomicAdd(&cfill[c], 1u)] = (uint32_t)p;
    }
}

// Canvas q of a set as a probe view (descriptor in device memory).
__device__ __forceinline__ CanvasView set_view(const CanvasDesc &d, const uint32_t *cells, const uint16_t *coarse,
                                               const Cand *cands,
                                               const Edge *ledges, const double2 *pspan)
{
    CanvasView v;
    v.X0 = d.X0; v.Y0 = d.Y0; v.sx = d.sx; v.sy = d.sy;
    v.bx0 = d.bx0; v.by0 = d.by0; v.bx1 = d.bx1; v.by1 = d.by1;
    v.W = d.W; v.H = d.H; v.Wt = d.Wt; v.Wc = d.Wc; v.Hc = d.Hc; v.blog = d.blog;
    v.cbyte = d.cbyte;
    v.M = d.M;
    v.cells = cells + d.cell_off;
    v.coarse = coarse + d.coarse_off;
    v.cands = cands;
    v.ledges = ledges;
    v.pspan = pspan;
    return v;
}

struct SetArgs {
    const CanvasDesc *cds;
    const uint32_t *cells;
    const uint16_t *coarse;
    const Cand *cands;
    const Edge *ledges;
    const double2 *pspan;
    const uint32_t *pid;          // layered set: caller's id of set polygon g (else g itself)
};

__device__ __forceinline__ uint32_t caller_id(const SetArgs &S, int64_t g)
{
    return S.pid ? S.pid[g] : (uint32_t)g;
}

constexpr uint32_t NO_WORD = 0xffffffffu;

// The canvas word of every point of a table chunk, when one word holds for
// all of them: the chunk's exact box lies inside the canvas's half-open box
// and every coarse block its pixels can fall in is uniform with that word
// (0, or an interior label + 1; the pixel map is monotonic, so the box's
// corner pixels bound every point's pixel).  Else NO_WORD.  Called by the
// whole workgroup (it synchronises).
__device__ uint32_t chunk_word(const CanvasView &v, const double4 cb)
{
    if (!(v.bx0 <= cb.x && cb.z < v.bx1 && v.by0 <= cb.y && cb.w < v.by1)) return NO_WORD;
    auto col = [&](double x) { return min((int)__dmul_rn(__dsub_rn(x, v.X0), v.sx), v.W - 1) >> v.blog; };
    auto row = [&](double y) { return min((int)__dmul_rn(__dsub_rn(y, v.Y0), v.sy), v.H - 1) >> v.blog; };
    const int c0 = col(cb.x), c1 = col(cb.z), r0 = row(cb.y), r1 = row(cb.w);
    const int nbx = c1 - c0 + 1, nb = nbx * (r1 - r0 + 1);
    if (nb > BT_THREADS) return NO_WORD;
    auto word = [&](int bx, int by) -> uint32_t {
        const int i = by * v.Wc + bx;
        return v.cbyte ? (uint32_t)((const uint8_t *)v.coarse)[i] : (uint32_t)v.coarse[i];
    };
    const uint32_t w0 = word(c0, r0);
    const int t = (int)threadIdx.x;
    const int same = (t >= nb) || word(c0 + t % nbx, r0 + t / nbx) == w0;
    const uint32_t full = v.cbyte ? COARSE_BYTE_FULL : (uint32_t)COARSE_FULL;
    return (__syncthreads_and(same) && w0 != full) ? w0 : NO_WORD;
}

// ------------------------------------------------------------ batch select

// Pass 1 (EMIT = false): matches per pair into pcount (64-bit, so that the
// scan of the counts accumulates in 64 bits) and, when hits is given, each
// thread's matches as a bit mask (hits[pair * BT_THREADS + thread], bit u
// for the thread's point u).  Pass 2 (EMIT): for
// the pairs of queries q0 <= q < q1 only, the 32-bit keys
// ((query - qrun0[query]) << idbits | point id) of the matching points at
// out[pbase[pair] - kbase ...]: every query's keys land in its own output
// range, and a sort of each run of queries (qrun0: a query's run's first
// query) orders them.
template <bool EMIT>
__global__ __launch_bounds__(BT_THREADS) void k_batch_select(SetArgs S, int64_t nfin, int64_t nchunk,
                                                             const double *X, const double *Y,
                                                             const uint32_t *ids, const unsigned int *cbase,
                                                             const uint32_t *plist, const uint32_t *pq,
                                                             unsigned long long *pcount, const unsigned long long *pbase,
                                                             uint32_t *out, uint32_t q0, uint32_t q1,
                                                             unsigned long long kbase, const uint32_t *qrun0,
                                                             int idbits, uint16_t *hits, const double4 *chunk_bb)
{
    static_assert(BT_PER <= 16, "a thread's matches are kept as 16 bits");
    __shared__ uint32_t wsum[BT_THREADS / 64];
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int64_t b = c * CHUNK;
        double xs[BT_PER], ys[BT_PER];
#pragma unroll
        for (int u = 0; u < BT_PER; ++u) {
            const int64_t i = b + (int64_t)u * BT_THREADS + threadIdx.x;   // coalesced
            xs[u] = i < nfin ? X[i] : NAN;
            ys[u] = i < nfin ? Y[i] : NAN;
        }
        for (uint32_t t = cbase[c]; t < cbase[c + 1]; ++t) {
            const uint32_t p = plist[t];
            const uint32_t qy = pq[p];
            if (EMIT && (qy < q0 || qy >= q1)) continue;   // uniform over the workgroup
            const CanvasDesc d = S.cds[qy];
            const CanvasView v = set_view(d, S.cells, S.coarse, S.cands, S.ledges, S.pspan);
            uint32_t hit = 0;
            const uint32_t cw = chunk_word(v, chunk_bb[c]);
            if (cw != NO_WORD) {
                // one word for the whole chunk: all of its points or none
                if (cw != 0u) {
#pragma unroll
                    for (int u = 0; u < BT_PER; ++u)
                        if (b + (int64_t)u * BT_THREADS + threadIdx.x < nfin) hit |= 1u << u;
                }
            } else {
#pragma unroll
                for (int u = 0; u < BT_PER; ++u) {
                    const uint32_t w = lookup(v, v.coarse, xs[u], ys[u]);
                    bool in = false;
                    if (w & BFLAG) {
                        uint32_t rec = w & ~BFLAG;
                        while (true) {
                            const Cand cd = v.cands[rec];
                            if (cand_inside(v, cd, xs[u], ys[u])) in = true;
                            if (cd.meta & CAND_LAST) break;
                            ++rec;
                        }
                    } else {
                        in = w != 0u;
                    }
                    hit |= (in ? 1u : 0u) << u;
                }
            }
            // block-wide exclusive scan of the per-thread match counts
            const uint32_t cnt = (uint32_t)__popc(hit);
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            uint32_t inc = cnt;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t tt = __shfl_up(inc, dd, 64);
                if (lane >= dd) inc += tt;
            }
            if (lane == 63) wsum[wv] = inc;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
#pragma unroll
            for (int q = 0; q < BT_THREADS / 64; ++q) {
                if (q < wv) pre += wsum[q];
                tot += wsum[q];
            }
            __syncthreads();
            if (!EMIT) {
                if (threadIdx.x == 0) pcount[p] = tot;
                if (hits) hits[(size_t)p * BT_THREADS + threadIdx.x] = (uint16_t)hit;
            } else if (hit) {
                unsigned long long pos = pbase[p] - kbase + pre + inc - cnt;
                const uint32_t qk = (qy - qrun0[qy]) << idbits;
#pragma unroll
                for (int u = 0; u < BT_PER; ++u)
                    if (hit & (1u << u)) out[pos++] = qk | ids[b + (int64_t)u * BT_THREADS + threadIdx.x];
            }
        }
    }
}

// The write pass from the count pass's match masks: no second probe.  Each
// workgroup takes pairs p0 <= p < p1 (the pairs of a run of queries, which
// are contiguous in query-major order), gathers the keys of its matches
// into LDS and stores them as one contiguous block at out[pbase[p] - kbase].
__global__ __launch_bounds__(BT_THREADS) void k_batch_emit_hits(int64_t p0, int64_t p1, const uint32_t *pq,
                                                                const uint32_t *pc, const uint16_t *hits,
                                                                const unsigned long long *pbase, const uint32_t *ids,
                                                                const uint32_t *qrun0, int idbits, uint32_t *out,
                                                                unsigned long long kbase)
{
    __shared__ uint32_t stage[CHUNK];
    __shared__ uint32_t wsum[BT_THREADS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t p = p0 + blockIdx.x; p < p1; p += gridDim.x) {
        const uint32_t hit = hits[(size_t)p * BT_THREADS + threadIdx.x];
        const uint32_t cnt = (uint32_t)__popc(hit);
        uint32_t inc = cnt;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t tt = __shfl_up(inc, dd, 64);
            if (lane >= dd) inc += tt;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < BT_THREADS / 64; ++q) {
            if (q < wv) pre += wsum[q];
            tot += wsum[q];
        }
        if (tot) {
            const uint32_t qy = pq[p];
            const uint32_t qk = (qy - qrun0[qy]) << idbits;
            const int64_t b = (int64_t)pc[p] * CHUNK;
            uint32_t at = pre + inc - cnt;
#pragma unroll
            for (int u = 0; u < BT_PER; ++u)
                if (hit & (1u << u)) stage[at++] = qk | ids[b + (int64_t)u * BT_THREADS + threadIdx.x];
            __syncthreads();
            uint32_t *dst = out + (pbase[p] - kbase);
            for (uint32_t i = threadIdx.x; i < tot; i += BT_THREADS) dst[i] = stage[i];
        }
        __syncthreads();
    }
}

// Ordering a run's keys without a radix sort.  A key is (query - first
// query of the run) << idbits | id, unique within the run.  Its top bits,
// key >> L with L = min(idbits, 20), name a bucket: a query and a window of
// 2^L consecutive ids.  Buckets are counted, the keys scattered into bucket
// order (when a query has more than one window), and each bucket is then
// ordered with a bitmap of its window in LDS: the set bits, read in order,
// are the bucket's ids ascending.
constexpr int SORT_LBITS = 20;                  // window bits: a 128 KB LDS bitmap
constexpr int BUCKETS_MAX = 4096;               // buckets of a run when a query has several windows
constexpr int BKT_THREADS = 1024;
constexpr int SCAT_PER = 8;                     // keys per thread of the scatter

__global__ __launch_bounds__(BKT_THREADS) void k_bucket_hist(int64_t n, const uint32_t *keys, int L,
                                                             uint32_t *hist)
{
    __shared__ uint32_t h[BUCKETS_MAX];
    for (int b = threadIdx.x; b < BUCKETS_MAX; b += BKT_THREADS) h[b] = 0u;
    __syncthreads();
    const int64_t nth = (int64_t)gridDim.x * BKT_THREADS;
    for (int64_t i0 = (int64_t)blockIdx.x * BKT_THREADS + threadIdx.x; i0 < n; i0 += 8 * nth) {
        uint32_t kk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) kk[u] = i0 + u * nth < n ? keys[i0 + u * nth] : 0u;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u * nth < n) atomicAdd(&h[kk[u] >> L], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BUCKETS_MAX; b += BKT_THREADS)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Exclusive scan of nb <= BUCKETS_MAX counts (one workgroup); boff[nb] = total.
__global__ __launch_bounds__(BKT_THREADS) void k_bucket_scan(int nb, const uint32_t *hist, uint32_t *boff)
{
    constexpr int PER = BUCKETS_MAX / BKT_THREADS;
    __shared__ uint32_t wsum[BKT_THREADS / 64];
    uint32_t v[PER], tot = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int b = threadIdx.x * PER + k;
        v[k] = b < nb ? hist[b] : 0u;
        tot += v[k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = tot;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int w = 0; w < BKT_THREADS / 64; ++w) {
        if (w < wv) pre += wsum[w];
        all += wsum[w];
    }
    uint32_t at = pre + inc - tot;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int b = threadIdx.x * PER + k;
        if (b < nb) boff[b] = at;
        at += v[k];
    }
    if (threadIdx.x == 0) boff[nb] = all;
}

// Keys into bucket order: each workgroup takes a tile of keys, counts its
// buckets in LDS, reserves each bucket's share with one atomic, then places
// its keys (cursor: nb zeros on entry).
__global__ __launch_bounds__(BKT_THREADS) void k_bucket_scatter(int64_t n, const uint32_t *keys, int L,
                                                                const uint32_t *boff, uint32_t *cursor,
                                                                uint32_t *out)
{
    __shared__ uint32_t h[BUCKETS_MAX];
    constexpr int64_t TILE = (int64_t)BKT_THREADS * SCAT_PER;
    for (int64_t t0 = (int64_t)blockIdx.x * TILE; t0 < n; t0 += (int64_t)gridDim.x * TILE) {
        for (int b = threadIdx.x; b < BUCKETS_MAX; b += BKT_THREADS) h[b] = 0u;
        __syncthreads();
        uint32_t k[SCAT_PER];
#pragma unroll
        for (int u = 0; u < SCAT_PER; ++u) {
            const int64_t i = t0 + (int64_t)u * BKT_THREADS + threadIdx.x;
            k[u] = i < n ? keys[i] : 0u;
            if (i < n) atomicAdd(&h[k[u] >> L], 1u);
        }
        __syncthreads();
        for (int b = threadIdx.x; b < BUCKETS_MAX; b += BKT_THREADS)
            if (h[b]) h[b] = boff[b] + atomicAdd(&cursor[b], h[b]);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SCAT_PER; ++u) {
            const int64_t i = t0 + (int64_t)u * BKT_THREADS + threadIdx.x;
            if (i < n) out[atomicAdd(&h[k[u] >> L], 1u)] = k[u];
        }
        __syncthreads();
    }
}

// Bucket b's keys keys[boff[b], boff[b+1]) in ascending id order: the ids
// (window << L | bit) of the set bits of its LDS bitmap, written to
// out[boff[b] ...] below limit.  Reads every key of the bucket before
// writing, so out may be keys (the buckets are disjoint ranges).  The bitmap
// is read in blocks of 64 words; the ids of a block are written 64 at a
// time, lane l taking the block's (r * 64 + l)-th set bit, so that a
// wavefront's stores go to consecutive positions.
constexpr int BM_WORDS_MAX = (1 << SORT_LBITS) >> 5;
constexpr int BM_BLOCKS_MAX = BM_WORDS_MAX / 64;

__global__ __launch_bounds__(BKT_THREADS) void k_bucket_bitmap(int nb, const uint32_t *boff, const uint32_t *keys,
                                                               int L, int H, uint32_t *out, int64_t limit)
{
    extern __shared__ uint32_t bm[];            // 2^L bits, whole blocks of 64 words
    __shared__ uint32_t btot[BM_BLOCKS_MAX];    // set bits per block, then the blocks' offsets
    __shared__ uint32_t wsum[BKT_THREADS / 64];
    const int nw = ((1 << L) >> 5) > 0 ? (1 << L) >> 5 : 1;
    const int nbk = (nw + 63) / 64;
    const uint32_t lmask = (1u << L) - 1u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NWAVE = BKT_THREADS / 64;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint32_t s = boff[b], e = boff[b + 1];
        if (s == e || (int64_t)s >= limit) continue;   // uniform over the workgroup
        for (int w = threadIdx.x; w < nbk * 64; w += BKT_THREADS) bm[w] = 0u;
        __syncthreads();
        // eight keys of each thread in flight at a time
        for (uint32_t i0 = s; i0 < e; i0 += 8 * BKT_THREADS) {
            uint32_t kk[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t i = i0 + (uint32_t)(u * BKT_THREADS) + threadIdx.x;
                kk[u] = i < e ? keys[i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (i0 + (uint32_t)(u * BKT_THREADS) + threadIdx.x >= e) continue;
                const uint32_t lo = kk[u] & lmask;
                atomicOr(&bm[lo >> 5], 1u << (lo & 31));
            }
        }
        __syncthreads();
        // set bits per block of 64 words
        for (int k = wv; k < nbk; k += NWAVE) {
            uint32_t c = (uint32_t)__popc(bm[k * 64 + lane]);
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
            if (lane == 0) btot[k] = c;
        }
        __syncthreads();
        // exclusive scan of the block totals (nbk <= BKT_THREADS)
        {
            const uint32_t v = threadIdx.x < nbk ? btot[threadIdx.x] : 0u;
            uint32_t inc = v;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = __shfl_up(inc, d, 64);
                if (lane >= d) inc += t;
            }
            if (lane == 63) wsum[wv] = inc;
            __syncthreads();
            uint32_t pre = 0;
            for (int w = 0; w < wv; ++w) pre += wsum[w];
            if (threadIdx.x < nbk) btot[threadIdx.x] = pre + inc - v;
        }
        __syncthreads();
        const uint32_t hi = (H > 0) ? ((uint32_t)b & ((1u << H) - 1u)) << L : 0u;
        for (int k = wv; k < nbk; k += NWAVE) {
            const uint32_t word = bm[k * 64 + lane];
            const uint32_t c = (uint32_t)__popc(word);
            uint32_t incl = c;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = __shfl_up(incl, d, 64);
                if (lane >= d) incl += t;
            }
            const uint32_t excl = incl - c;
            const uint32_t T = (uint32_t)__shfl((int)incl, 63, 64);
            const int64_t base = (int64_t)s + btot[k];
            for (uint32_t r0 = 0; r0 < T; r0 += 64) {
                const uint32_t o = r0 + (uint32_t)lane;
                // the word holding set bit o of the block: the last lane whose
                // exclusive count is <= o
                int at = 0;
                for (int step = 32; step >= 1; step >>= 1) {
                    const uint32_t ex = (uint32_t)__shfl((int)excl, at + step < 64 ? at + step : 63, 64);
                    if (at + step < 64 && ex <= o) at += step;
                }
                uint32_t w = (uint32_t)__shfl((int)word, at, 64);
                const uint32_t ex_at = (uint32_t)__shfl((int)excl, at, 64);
                if (o < T) {
                    for (uint32_t skip = o - ex_at; skip; --skip) w &= w - 1u;
                    const int bit = __ffs(w) - 1;
                    const int64_t pos = base + o;
                    if (pos < limit) out[pos] = hi | ((uint32_t)(k * 64 + at) << 5) | (uint32_t)bit;
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ batch join pairs

constexpr int PAIR_RANGES = 64;   // point-id ranges the pairs are counted in

// Pairs (point id, polygon id) of the table with a canvas set.  COUNT:
// matches per range of point ids (id >> rshift) into rcount.  Otherwise the
// keys (id << pbits | polygon) of the matches with id >> rshift in
// [r0, r1) are appended to keys (one reservation per workgroup and pair;
// their order is fixed by the sort that follows).
template <bool COUNT>
__global__ __launch_bounds__(BT_THREADS) void k_batch_pairs(SetArgs S, int64_t nfin, int64_t nchunk,
                                                            const double *X, const double *Y, const uint32_t *ids,
                                                            const unsigned int *cbase, const uint32_t *plist,
                                                            const uint32_t *pq, int rshift, int pbits,
                                                            unsigned long long *rcount, uint32_t r0, uint32_t r1,
                                                            unsigned long long *cursor, unsigned long long *keys,
                                                            const double4 *chunk_bb)
{
    __shared__ unsigned long long s_cnt[PAIR_RANGES];
    __shared__ uint32_t wsum[BT_THREADS / 64];
    __shared__ unsigned long long s_at;
    if (COUNT)
        for (int k = threadIdx.x; k < PAIR_RANGES; k += BT_THREADS) s_cnt[k] = 0ull;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int64_t b = c * CHUNK;
        double xs[BT_PER], ys[BT_PER];
        uint32_t pid[BT_PER];
#pragma unroll
        for (int u = 0; u < BT_PER; ++u) {
            const int64_t i = b + (int64_t)u * BT_THREADS + threadIdx.x;
            xs[u] = i < nfin ? X[i] : NAN;
            ys[u] = i < nfin ? Y[i] : NAN;
            pid[u] = i < nfin ? ids[i] : 0u;
        }
        for (uint32_t t = cbase[c]; t < cbase[c + 1]; ++t) {
            const uint32_t p = plist[t];
            const CanvasDesc d = S.cds[pq[p]];
            const CanvasView v = set_view(d, S.cells, S.coarse, S.cands, S.ledges, S.pspan);
            uint32_t mine = 0;
            const uint32_t cw = chunk_word(v, chunk_bb[c]);   // one word for the whole chunk, or NO_WORD
            // the matches of this thread's points, in two sweeps: count, write
            auto sweep = [&](auto &&emit) {
#pragma unroll
                for (int u = 0; u < BT_PER; ++u) {
                    if (!COUNT) {
                        const uint32_t r = pid[u] >> rshift;
                        if (r < r0 || r >= r1) continue;
                    }
                    if (cw != NO_WORD) {
                        if (cw != 0u && b + (int64_t)u * BT_THREADS + threadIdx.x < nfin) emit(u, cw - 1u);
                        continue;
                    }
                    const uint32_t w = lookup(v, v.coarse, xs[u], ys[u]);
                    if (w == 0u) continue;
                    if (!(w & BFLAG)) { emit(u, w - 1u); continue; }
                    uint32_t rec = w & ~BFLAG;
                    while (true) {
                        const Cand cd = v.cands[rec];
                        if (cand_inside(v, cd, xs[u], ys[u])) emit(u, cd.poly);
                        if (cd.meta & CAND_LAST) break;
                        ++rec;
                    }
                }
            };
            if (COUNT) {
                sweep([&](int u, uint32_t) { atomicAdd(&s_cnt[pid[u] >> rshift], 1ull); });
                continue;
            }
            sweep([&](int, uint32_t) { ++mine; });
            // workgroup-wide exclusive scan of the match counts, one reservation
            uint32_t inc = mine;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t tt = __shfl_up(inc, dd, 64);
                if (lane >= dd) inc += tt;
            }
            if (lane == 63) wsum[wv] = inc;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
#pragma unroll
            for (int q = 0; q < BT_THREADS / 64; ++q) {
                if (q < wv) pre += wsum[q];
                tot += wsum[q];
            }
            if (threadIdx.x == 0) s_at = tot ? atomicAdd(cursor, (unsigned long long)tot) : 0ull;
            __syncthreads();
            unsigned long long pos = s_at + pre + inc - mine;
            sweep([&](int u, uint32_t label) {
                keys[pos++] = ((unsigned long long)pid[u] << pbits) | caller_id(S, d.poly_base + label);
            });
            __syncthreads();
        }
    }
    if (COUNT) {
        __syncthreads();
        for (int k = threadIdx.x; k < PAIR_RANGES; k += BT_THREADS)
            if (s_cnt[k]) atomicAdd(&rcount[k], s_cnt[k]);
    }
}

__global__ void k_split_pairs(int64_t n, const unsigned long long *keys, int pbits, uint32_t *pt, uint32_t *pg)
{
    const unsigned long long m = (1ull << pbits) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = keys[i];
        pt[i] = (uint32_t)(k >> pbits);
        pg[i] = (uint32_t)(k & m);
    }
}

// Query starts from pair bases: qoff[q] = pbase[first pair of q], qoff[nq] =
// pbase[np] = the total.
__global__ void k_query_off(int nq, const unsigned long long *qbase, const unsigned long long *pbase, int64_t np,
                            unsigned long long *qoff)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > nq) return;
    const unsigned long long total = pbase[np];
    if (q == nq) { qoff[nq] = total; return; }
    const unsigned long long p = qbase[q];
    qoff[q] = (p < (unsigned long long)np) ? pbase[p] : total;
}

// ------------------------------------------------------------ batch join-count

constexpr int HSLOTS = 512;   // LDS hash slots per workgroup

// Whole-batch join-count in one launch, with no pair list: every workgroup
// takes table chunks (grid-stride), lists in LDS the canvases whose box meets
// the chunk's box (from qbox, a window of QL_MAX canvases at a time) and
// probes its points against them, counting per polygon in an LDS hash
// flushed with atomics per chunk.  Nothing is read back on the host between
// launches, so the call's
// launches are captured into a graph and replayed batch after batch, each
// replay reading the canvas set's descriptors as rebuilt for that batch.
constexpr int QL_MAX = 1024;
constexpr int64_t HIST_MAX_BATCH = 8192;   // polygons the count probe histograms in LDS

// Per-canvas boxes for the direct probe; a canvas with skip[q] set (counted
// by another launch) gets an empty box.
__global__ void k_qbox(int nq, const CanvasDesc *cds, const uint8_t *skip, double4 *qbox)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const CanvasDesc d = cds[q];
        qbox[q] = (d.empty || (skip && skip[q])) ? make_double4(INFINITY, INFINITY, -INFINITY, -INFINITY)
                                                 : make_double4(d.bx0, d.by0, d.bx1, d.by1);
    }
}

__global__ __launch_bounds__(BT_THREADS) void k_batch_count_direct(SetArgs S, int nq, int64_t nfin, int64_t nchunk,
                                                                   const double *X, const double *Y,
                                                                   const double4 *chunk_bb, const double4 *qbox,
                                                                   unsigned long long *counts)
{
    __shared__ unsigned long long hkey[HSLOTS];   // polygon id + 1 (0: empty)
    __shared__ uint32_t hval[HSLOTS];
    __shared__ uint32_t qlist[QL_MAX];
    __shared__ uint32_t s_nq;
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int64_t b = c * CHUNK;
        const double4 cb = chunk_bb[c];
        double xs[BT_PER], ys[BT_PER];
#pragma unroll
        for (int u = 0; u < BT_PER; ++u) {
            const int64_t i = b + (int64_t)u * BT_THREADS + threadIdx.x;
            xs[u] = i < nfin ? X[i] : NAN;
            ys[u] = i < nfin ? Y[i] : NAN;
        }
        for (int s = threadIdx.x; s < HSLOTS; s += BT_THREADS) { hkey[s] = 0ull; hval[s] = 0u; }
        for (int q0 = 0; q0 < nq; q0 += QL_MAX) {
            if (threadIdx.x == 0) s_nq = 0u;
            __syncthreads();
            for (int q = q0 + threadIdx.x; q < min(nq, q0 + QL_MAX); q += BT_THREADS) {
                const double4 qb = qbox[q];
                // the chunk's closed point box meets the canvas's half-open box
                if (cb.z >= qb.x && cb.x < qb.z && cb.w >= qb.y && cb.y < qb.w) qlist[atomicAdd(&s_nq, 1u)] = (uint32_t)q;
            }
            __syncthreads();
            const uint32_t nl = s_nq;
            for (uint32_t t = 0; t < nl; ++t) {
                const CanvasDesc d = S.cds[qlist[t]];
                const CanvasView v = set_view(d, S.cells, S.coarse, S.cands, S.ledges, S.pspan);
                auto add_n = [&](uint32_t label, uint32_t k) {
                    const unsigned long long key = (unsigned long long)caller_id(S, d.poly_base + label) + 1ull;
                    uint32_t h = (uint32_t)(key * 0x9E3779B97F4A7C15ull >> 55) & (HSLOTS - 1);
                    for (int probe = 0; probe < 8; ++probe, h = (h + 1) & (HSLOTS - 1)) {
                        unsigned long long cur = hkey[h];
                        if (cur == 0ull) {
                            cur = atomicCAS(&hkey[h], 0ull, key);
                            if (cur == 0ull) cur = key;
                        }
                        if (cur == key) { atomicAdd(&hval[h], k); return; }
                    }
                    atomicAdd(&counts[key - 1ull], (unsigned long long)k);
                };
                auto add = [&](uint32_t label) { add_n(label, 1u); };
                const uint32_t cw = chunk_word(v, cb);
                if (cw != NO_WORD) {
                    // one word for the whole chunk: its points all count for one polygon, or none
                    if (cw != 0u && threadIdx.x == 0) add_n(cw - 1u, (uint32_t)min<int64_t>(CHUNK, nfin - b));
                    continue;
                }
#pragma unroll
                for (int u = 0; u < BT_PER; ++u) {
                    const uint32_t w = lookup(v, v.coarse, xs[u], ys[u]);
                    if (w == 0u) continue;
                    if (!(w & BFLAG)) { add(w - 1u); continue; }
                    uint32_t rec = w & ~BFLAG;
                    while (true) {
                        const Cand cd = v.cands[rec];
                        if (cand_inside(v, cd, xs[u], ys[u])) add(cd.poly);
                        if (cd.meta & CAND_LAST) break;
                        ++rec;
                    }
                }
            }
            __syncthreads();
        }
        for (int s = threadIdx.x; s < HSLOTS; s += BT_THREADS)
            if (hkey[s]) atomicAdd(&counts[hkey[s] - 1ull], (unsigned long long)hval[s]);
        __syncthreads();
    }
}

__global__ void k_zero64(int64_t n, unsigned long long *p)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) p[i] = 0ull;
}

__global__ void k_zero32(int64_t n, unsigned int *p)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) p[i] = 0u;
}

static int num_cus_of(int device)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0) v = 256;
    return v;
}

// Batch scratch: pairs in query-major order, their chunk-major lists.
struct Pairs {
    int64_t np = 0;
    uint32_t *pq = nullptr, *pc = nullptr, *plist = nullptr;
    unsigned int *cbase = nullptr;
    unsigned long long *qbase = nullptr;
};

static int make_pairs(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, Pairs &P)
{
    hipStream_t st = ctx->stream;
    const int nq = set->nc;
    const int64_t nchunk = t->nchunk;
    DevBuf &bq = ctx->scratch[S_KEYS];
    if (ensure(ctx, bq, sizeof(unsigned long long) * (3 * (size_t)nq + 3) + sizeof(unsigned int) * 2 * ((size_t)nchunk + 2)))
        return SPADE_E_NOMEM;
    unsigned long long *qcount = (unsigned long long *)bq.p;
    unsigned long long *qbase = qcount + (nq + 1);
    unsigned long long *qfill = qbase + (nq + 1);
    unsigned int *ccount = (unsigned int *)(qfill + (nq + 1));
    unsigned int *cbase = ccount + (nchunk + 1);
    hipLaunchKernelGGL(k_zero64, dim3(grid_of(3 * nq + 3, 1024)), dim3(256), 0, st, (int64_t)(3 * nq + 3), qcount);
    hipLaunchKernelGGL(k_zero32, dim3(grid_of(2 * nchunk + 2, 4096)), dim3(256), 0, st, (int64_t)(2 * nchunk + 2), ccount);
    SPADE_HIP(ctx, hipGetLastError());
    const CanvasDesc *cds = (const CanvasDesc *)set->dcds.p;
    const double4 *bb = (const double4 *)t->chunk_bb.p;
    dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((nchunk + 255) / 256, 64)), (unsigned)std::min(nq, 32768));
    if (nchunk > 0) {
        hipLaunchKernelGGL(k_pairs<false>, g, dim3(256), 0, st, nq, nchunk, bb, cds, qcount, nullptr, nullptr, nullptr, nullptr);
        SPADE_HIP(ctx, hipGetLastError());
    }
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, qcount, qbase, nq + 1, st));
    if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, qcount, qbase, nq + 1, st));
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(h, qbase + nq, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const int64_t np = (int64_t)h[0];
    if (np >= (int64_t)INT32_MAX) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many (chunk, query) pairs in one batch");
    DevBuf &bp = ctx->scratch[S_VALS];
    if (ensure(ctx, bp, sizeof(uint32_t) * 3 * (size_t)std::max<int64_t>(np, 1))) return SPADE_E_NOMEM;
    P.np = np;
    ctx->batch_overlaps = np;
    P.pq = (uint32_t *)bp.p;
    P.pc = P.pq + std::max<int64_t>(np, 1);
    P.plist = P.pc + std::max<int64_t>(np, 1);
    P.cbase = cbase;
    P.qbase = qbase;
    if (np > 0) {
        hipLaunchKernelGGL(k_pairs<true>, g, dim3(256), 0, st, nq, nchunk, bb, cds, nullptr, qbase, qfill, P.pq, P.pc);
        hipLaunchKernelGGL(k_pair_chunk_count, dim3(grid_of(np)), dim3(256), 0, st, np, P.pc, ccount);
        SPADE_HIP(ctx, hipGetLastError());
    }
    tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, ccount, cbase, (int)(nchunk + 1), st));
    if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, ccount, cbase, (int)(nchunk + 1), st));
    if (np > 0) {
        hipLaunchKernelGGL(k_zero32, dim3(grid_of(nchunk + 1, 4096)), dim3(256), 0, st, nchunk + 1, ccount);
        hipLaunchKernelGGL(k_pair_chunk_fill, dim3(grid_of(np)), dim3(256), 0, st, np, P.pc, cbase, ccount, P.plist);
        SPADE_HIP(ctx, hipGetLastError());
    }
    return SPADE_OK;
}

static SetArgs set_args(const spade_canvas *set)
{
    SetArgs S;
    S.cds = (const CanvasDesc *)set->dcds.p;
    S.cells = (const uint32_t *)set->cells.p;
    S.coarse = (const uint16_t *)set->coarse.p;
    S.cands = (const Cand *)set->cands.p;
    S.ledges = (const Edge *)set->ledges.p;
    S.pspan = (const double2 *)set->pspan.p;
    S.pid = set->layered ? (const uint32_t *)set->pid.p : nullptr;
    return S;
}

}  // namespace spade

using namespace spade;

extern "C" {

int spade_ctx_set_pixels_per_vertex(spade_ctx *ctx, double ppv)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!(ppv >= 1.0 && ppv <= 1e7)) return set_error(ctx, SPADE_E_INVALID, "pixels per vertex must be in [1, 1e7]");
    ctx->ppv = ppv;
    return SPADE_OK;
}

int spade_table_create(spade_ctx *ctx, const spade_points *pts, spade_table **out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !out) return SPADE_E_INVALID;
    *out = nullptr;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    if (!pts || pts->n < 0 || (pts->n > 0 && (!pts->x || !pts->y)))
        return set_error(ctx, SPADE_E_INVALID, "invalid point arrays");
    if (pts->n > (int64_t)INT32_MAX) return set_error(ctx, SPADE_E_TOO_LARGE, "a table holds at most 2^31 - 1 points");
    hipStream_t st = ctx->stream;
    spade_table *t = new (std::nothrow) spade_table();
    if (!t) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    t->device = ctx->device;
    const int64_t n = pts->n;
    t->n = n;
    auto fail = [&](int rc) { spade_table_destroy(t); return rc; };
    const size_t ns = (size_t)std::max<int64_t>(n, 1);
    if (ensure(ctx, t->x, 8 * ns) || ensure(ctx, t->y, 8 * ns) || ensure(ctx, t->ids, 4 * ns)) return fail(SPADE_E_NOMEM);
    // bounding box and grid
    DevBuf &bb = ctx->scratch[S_BLOCKRED];
    if (ensure(ctx, bb, 64)) return fail(SPADE_E_NOMEM);
    SPADE_HIP(ctx, hipMemsetAsync(bb.p, 0xff, 32, st));
    if (n > 0) hipLaunchKernelGGL(k_pt_bbox, dim3(grid_of(n, 1024)), dim3(256), 0, st, n, pts->x, pts->y, (unsigned long long *)bb.p);
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    SPADE_HIP(ctx, hipMemcpyAsync(h, bb.p, 32, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    double x0 = from_okey(h[0]), x1 = -from_okey(h[1]), y0 = from_okey(h[2]), y1 = -from_okey(h[3]);
    if (!(x0 <= x1)) { x0 = 0; x1 = 1; y0 = 0; y1 = 1; }
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(GRID_MAX, (int64_t)std::sqrt((double)n / 64.0)));
    t->G = G;
    t->X0 = x0; t->Y0 = y0;
    t->sx = (x1 > x0) ? G / (x1 - x0) : 0.0;
    t->sy = (y1 > y0) ? G / (y1 - y0) : 0.0;
    // cells in Z order: codes below P * P, P the power of two >= G
    int64_t P = 1;
    while (P < G) P <<= 1;
    const int64_t ncell = P * P;
    // sort by cell
    DevBuf &dk = ctx->scratch[S_KEYS], &dk2 = ctx->scratch[S_KEYS2], &dv = ctx->scratch[S_VALS];
    if (ensure(ctx, dk, 4 * ns) || ensure(ctx, dk2, 4 * ns) || ensure(ctx, dv, 4 * ns) ||
        ensure(ctx, t->cell_off, 4 * ((size_t)ncell + 2)))
        return fail(SPADE_E_NOMEM);
    if (n > 0) {
        hipLaunchKernelGGL(k_pt_key, dim3(grid_of(n)), dim3(256), 0, st, n, pts->x, pts->y, t->X0, t->Y0, t->sx, t->sy,
                           G, (uint32_t)ncell, (uint32_t *)dk.p, (uint32_t *)dv.p);
        SPADE_HIP(ctx, hipGetLastError());
        DevBuf &cub = ctx->scratch[S_CUBTMP];
        size_t tb = 0;
        const int kb = std::max(1, bits_of((uint64_t)ncell));
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const uint32_t *)dk.p, (uint32_t *)dk2.p,
                                                          (const uint32_t *)dv.p, (uint32_t *)t->ids.p, (int)n, 0, kb, st));
        if (ensure(ctx, cub, tb)) return fail(SPADE_E_NOMEM);
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub.p, tb, (const uint32_t *)dk.p, (uint32_t *)dk2.p,
                                                          (const uint32_t *)dv.p, (uint32_t *)t->ids.p, (int)n, 0, kb, st));
        hipLaunchKernelGGL(k_pt_gather, dim3(grid_of(n)), dim3(256), 0, st, n, (const uint32_t *)t->ids.p, pts->x, pts->y,
                           (double *)t->x.p, (double *)t->y.p);
        hipLaunchKernelGGL(k_cell_off, dim3(grid_of(n + 1)), dim3(256), 0, st, n, (const uint32_t *)dk2.p, ncell,
                           (uint32_t *)t->cell_off.p);
        SPADE_HIP(ctx, hipGetLastError());
        uint32_t *hf = (uint32_t *)ensure_pinned(ctx, 64);
        SPADE_HIP(ctx, hipMemcpyAsync(hf, (uint32_t *)t->cell_off.p + ncell, 4, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        t->nfin = hf[0];
    }
    t->nchunk = (t->nfin + CHUNK - 1) / CHUNK;
    if (ensure(ctx, t->chunk_bb, sizeof(double4) * (size_t)std::max<int64_t>(t->nchunk, 1))) return fail(SPADE_E_NOMEM);
    if (t->nchunk > 0) {
        hipLaunchKernelGGL(k_chunk_bb, dim3(grid_of(t->nchunk * 64, 8192)), dim3(256), 0, st, t->nfin, t->nchunk,
                           (const double *)t->x.p, (const double *)t->y.p, (double4 *)t->chunk_bb.p);
        SPADE_HIP(ctx, hipGetLastError());
    }
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *out = t;
    return SPADE_OK;
}

void spade_table_destroy(spade_table *t)
{
    if (!t) return;
    (void)hipSetDevice(t->device);
    free_buf(t->x);
    free_buf(t->y);
    free_buf(t->ids);
    free_buf(t->cell_off);
    free_buf(t->chunk_bb);
    delete t;
}

int spade_table_info(const spade_table *t, int64_t *n, int32_t *grid, int64_t *chunks, int64_t *device_bytes)
{
    if (!t) return SPADE_E_INVALID;
    if (n) *n = t->n;
    if (grid) *grid = t->G;
    if (chunks) *chunks = t->nchunk;
    if (device_bytes) *device_bytes = (int64_t)t->bytes();
    return SPADE_OK;
}

static int check_batch_args(spade_ctx *ctx, const spade_polys *polys, int32_t nq, const int64_t *qbound)
{
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    if (!polys || nq < 1 || !qbound) return set_error(ctx, SPADE_E_INVALID, "a batch needs polygons and nq >= 1 queries");
    if (polys->n_polys < 0 || polys->n_rings < 0 || (!polys->poly_ring_off && polys->n_rings != polys->n_polys))
        return set_error(ctx, SPADE_E_INVALID, "malformed polygon set");
    if (polys->n_rings > 0 && (!polys->ring_vtx_off || !polys->vx || !polys->vy))
        return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off / vx / vy is NULL");
    if (qbound[0] != 0 || qbound[nq] != polys->n_polys) return set_error(ctx, SPADE_E_INVALID, "qbound must run from 0 to n_polys");
    for (int q = 0; q < nq; ++q)
        if (qbound[q + 1] < qbound[q]) return set_error(ctx, SPADE_E_INVALID, "qbound must be non-decreasing");
    return SPADE_OK;
}

int spade_batch_build(spade_ctx *ctx, const spade_polys *polys, int32_t nq, const int64_t *qbound,
                      spade_canvas **out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !out) return SPADE_E_INVALID;
    *out = nullptr;
    int rc0 = check_batch_args(ctx, polys, nq, qbound);
    if (rc0) return rc0;
    spade_canvas *cv = new (std::nothrow) spade_canvas();
    if (!cv) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    cv->device = ctx->device;
    const int rc = build_set(ctx, polys, nq, qbound, cv);
    if (rc) {
        spade_canvas_destroy(cv);
        return rc;
    }
    *out = cv;
    return SPADE_OK;
}

int spade_batch_rebuild(spade_ctx *ctx, const spade_polys *polys, int32_t nq, const int64_t *qbound,
                        spade_canvas *set)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !set) return ctx ? set_error(ctx, SPADE_E_INVALID, "NULL argument") : SPADE_E_INVALID;
    int rc = check_batch_args(ctx, polys, nq, qbound);
    if (rc) return rc;
    if (set->device != ctx->device) return set_error(ctx, SPADE_E_INVALID, "the canvas set lives on another device");
    if (set == ctx->plain) return set_error(ctx, SPADE_E_INVALID, "not a caller-owned canvas set");
    set->layered = false;
    set->n_layers = 0;
    return build_set(ctx, polys, nq, qbound, set);
}

int spade_batch_select(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, uint32_t *out_ids, int64_t cap,
                       int64_t *out_off)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !set || !t || !out_off) return ctx ? set_error(ctx, SPADE_E_INVALID, "NULL argument") : SPADE_E_INVALID;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    const int nq = set->nc;
    if (set->layered) return set_error(ctx, SPADE_E_INVALID, "a layered set is queried with join calls");
    for (int q = 0; q < nq; ++q)
        if (set->descs[q].M != 1) return set_error(ctx, SPADE_E_INVALID, "batch selection needs exactly one polygon per query");
    if (cap < 0 || (cap > 0 && !out_ids)) return set_error(ctx, SPADE_E_INVALID, "bad output buffer");
    hipStream_t st = ctx->stream;
    ctx->timed_raster = false;
    Pairs P;
    int rc = make_pairs(ctx, set, t, P);
    if (rc) return rc;
    const int64_t np = P.np;
    DevBuf &bc = ctx->scratch[S_VALS2];
    DevBuf &bo = ctx->scratch[S_ENTC];
    if (ensure(ctx, bc, sizeof(unsigned long long) * (size_t)(np + 1) + sizeof(unsigned long long) * (size_t)(np + 1) +
                            sizeof(unsigned long long) * (size_t)(nq + 2) + 64))
        return SPADE_E_NOMEM;
    // 64-bit counts: hipCUB's scan accumulates in the input's type, and a
    // batch may select more than 2^32 ids in total
    unsigned long long *pcount = (unsigned long long *)bc.p;
    unsigned long long *pbase = pcount + (np + 1);
    unsigned long long *qoff = pbase + (np + 1);
    const SetArgs S = set_args(set);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(t->nchunk, (int64_t)num_cus_of(ctx->device) * 8));
    // the count pass keeps every pair's match masks (2 bytes per point slot)
    // when they fit the limit (SPADE_HIT_MASK_LIMIT bytes, default 16 GiB);
    // the write pass then reads them instead of probing again
    size_t hits_max = (size_t)16 << 30;
    if (const char *e = getenv("SPADE_HIT_MASK_LIMIT")) hits_max = (size_t)strtoull(e, nullptr, 10);
    DevBuf &bh = ctx->scratch[S_KEYS2];
    const size_t hbytes = sizeof(uint16_t) * BT_THREADS * (size_t)std::max<int64_t>(np, 1);
    uint16_t *hits = nullptr;
    if (cap > 0 && hbytes <= hits_max) {
        if (ensure(ctx, bh, hbytes) == SPADE_OK) hits = (uint16_t *)bh.p;
        else ctx->err.clear();   // probe twice instead
    }
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, st, (int64_t)1, pcount + np);
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (np > 0) {
        hipLaunchKernelGGL(k_batch_select<false>, dim3(grid), dim3(BT_THREADS), 0, st, S, t->nfin, t->nchunk,
                           (const double *)t->x.p, (const double *)t->y.p, (const uint32_t *)t->ids.p, P.cbase,
                           P.plist, P.pq, pcount, nullptr, nullptr, 0u, (uint32_t)nq, 0ull, nullptr, 0, hits,
                           (const double4 *)t->chunk_bb.p);
        SPADE_HIP(ctx, hipGetLastError());
    }
    // the timed probe of a batch selection is its count pass
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, pcount, pbase, (int)(np + 1), st));
    if (ensure(ctx, cub, tb)) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, pcount, pbase, (int)(np + 1), st));
    // one readback: the queries' output offsets and their first pairs
    unsigned long long *h =
        (unsigned long long *)ensure_pinned(ctx, sizeof(unsigned long long) * 2 * (size_t)(nq + 1) + 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    hipLaunchKernelGGL(k_query_off, dim3((nq + 1 + 255) / 256), dim3(256), 0, st, nq, P.qbase, pbase, np, qoff);
    SPADE_HIP(ctx, hipGetLastError());
    SPADE_HIP(ctx, hipMemcpyAsync(h, qoff, sizeof(unsigned long long) * (size_t)(nq + 1), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipMemcpyAsync(h + nq + 1, P.qbase, sizeof(unsigned long long) * (size_t)(nq + 1),
                                  hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    for (int q = 0; q <= nq; ++q) out_off[q] = (int64_t)h[q];
    const unsigned long long total = h[nq];
    const std::vector<unsigned long long> hq(h + nq + 1, h + 2 * (nq + 1));
    // a buffer that is too small still receives the first cap ids in the
    // canonical order (two-step Map); the call then reports the shortfall
    const bool short_cap = (int64_t)total > cap;
    if (total == 0 || cap == 0) {
        if (short_cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
        return SPADE_OK;
    }
    // Each query's ids are ordered per run of consecutive queries (at most
    // 2^(32 - idbits) queries and 2^30 keys a run; a larger query alone),
    // keyed by the 32-bit key (query - first query of its run) << idbits |
    // id.  One write pass puts every key of the runs that end within cap at
    // its final position in out_ids; each such run is then put in bucket
    // order (query, window of 2^L ids) through scratch when a query spans
    // several windows, and every bucket ordered with an LDS bitmap of its
    // window, which writes the ids themselves.  The run that crosses cap, if
    // any, is written to scratch by a pass of its own and only its first ids
    // are written out; runs from cap on are not evaluated.
    const int idbits = std::max(1, bits_of((uint64_t)std::max<int64_t>(t->n - 1, 1)));
    const int LB = std::min(idbits, SORT_LBITS);
    const int HB = idbits - LB;
    const int64_t QMAX = (int64_t)1 << (32 - idbits);
    const int64_t GROUP = (int64_t)1 << 30;
    struct Run { int q0, q1; int64_t k0, k1; };
    std::vector<Run> runs;
    {
        int qb = 0;
        for (int q = 0; q < nq; ++q)
            if (q > qb && (q - qb >= QMAX || out_off[q + 1] - out_off[qb] > GROUP)) {
                runs.push_back({qb, q, out_off[qb], out_off[q]});
                qb = q;
            }
        runs.push_back({qb, nq, out_off[qb], out_off[nq]});
    }
    std::vector<uint32_t> hrun0((size_t)nq);
    int qdone = 0;                       // queries of the runs that end within cap
    int64_t gmax = 0, cross = -1;        // largest run ordered; index of the run crossing cap
    size_t nbmax = 1;                    // most buckets of a run
    for (size_t r = 0; r < runs.size(); ++r) {
        const Run &R = runs[r];
        for (int q = R.q0; q < R.q1; ++q) hrun0[(size_t)q] = (uint32_t)R.q0;
        if (R.k1 <= cap) qdone = R.q1;
        else if (R.k0 < cap && cross < 0) cross = (int64_t)r;
        if (R.k0 < cap) {
            gmax = std::max(gmax, R.k1 - R.k0);
            nbmax = std::max(nbmax, (size_t)(R.q1 - R.q0) << HB);
        }
    }
    DevBuf &br = ctx->scratch[S_LOOKBACK];
    DevBuf &bo2 = ctx->scratch[S_ENTF];
    const int64_t nbo = cross >= 0 ? runs[(size_t)cross].k1 - runs[(size_t)cross].k0 : 0;
    // br: qrun0 [nq] | bucket counts [nbmax] | bucket offsets [nbmax + 1] | cursors [nbmax]
    if (ensure(ctx, br, sizeof(uint32_t) * ((size_t)nq + 3 * nbmax + 1)) ||
        ensure(ctx, bo2, 4 * (size_t)std::max<int64_t>(HB > 0 ? gmax : 1, 1)) ||
        ensure(ctx, bo, 4 * (size_t)std::max<int64_t>(nbo, 1)))
        return SPADE_E_NOMEM;
    uint32_t *qrun0 = (uint32_t *)br.p;
    uint32_t *bhist = qrun0 + nq, *boff = bhist + nbmax, *bcur = boff + nbmax + 1;
    SPADE_HIP(ctx, hipMemcpyAsync(qrun0, hrun0.data(), sizeof(uint32_t) * (size_t)nq, hipMemcpyHostToDevice, st));
    // the bitmap in whole blocks of 64 words
    const size_t bm_lds = sizeof(uint32_t) * 64 * (size_t)((std::max(1, (1 << LB) >> 5) + 63) / 64);
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_bucket_bitmap, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bm_lds));
    // with one window per query, a run's buckets are its queries: their
    // offsets come from out_off (one host array for all runs, so that no
    // copy reads a slice that is being rewritten)
    std::vector<uint32_t> hoff;
    if (HB == 0)
        for (const auto &R : runs)
            for (int q = R.q0; q <= R.q1; ++q) hoff.push_back((uint32_t)(out_off[q] - R.k0));
    size_t hoff_at = 0;
    // orders the keys keys[0, k1 - k0) of run R; the ids end in dst[0, nwrite)
    auto sort_run = [&](const Run &R, uint32_t *keys, uint32_t *dst, int64_t nwrite) -> int {
        const int64_t n = R.k1 - R.k0;
        const int nb = (R.q1 - R.q0) << HB;
        const int cus = num_cus_of(ctx->device);
        const uint32_t *src = keys;
        if (HB == 0) {
            // one bucket per query: the keys are in bucket order already
            size_t at = 0;
            for (const auto &Q : runs) {
                if (Q.q0 == R.q0) break;
                at += (size_t)(Q.q1 - Q.q0) + 1;
            }
            SPADE_HIP(ctx, hipMemcpyAsync(boff, hoff.data() + at, sizeof(uint32_t) * ((size_t)nb + 1),
                                          hipMemcpyHostToDevice, st));
        } else {
            hipLaunchKernelGGL(k_zero32, dim3(grid_of(nb, 1024)), dim3(256), 0, st, (int64_t)nb, bhist);
            hipLaunchKernelGGL(k_zero32, dim3(grid_of(nb, 1024)), dim3(256), 0, st, (int64_t)nb, bcur);
            const int hg = (int)std::max<int64_t>(1, std::min<int64_t>((n + BKT_THREADS * 16 - 1) / (BKT_THREADS * 16),
                                                                       (int64_t)cus * 2));
            hipLaunchKernelGGL(k_bucket_hist, dim3(hg), dim3(BKT_THREADS), 0, st, n, keys, LB, bhist);
            hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(BKT_THREADS), 0, st, nb, bhist, boff);
            const int sg = (int)std::max<int64_t>(1, std::min<int64_t>((n + BKT_THREADS * SCAT_PER - 1) /
                                                                           (BKT_THREADS * SCAT_PER),
                                                                       (int64_t)cus * 4));
            hipLaunchKernelGGL(k_bucket_scatter, dim3(sg), dim3(BKT_THREADS), 0, st, n, keys, LB, boff, bcur,
                               (uint32_t *)bo2.p);
            src = (const uint32_t *)bo2.p;
        }
        SPADE_HIP(ctx, hipGetLastError());
        hipLaunchKernelGGL(k_bucket_bitmap, dim3((unsigned)std::min<int64_t>(nb, (int64_t)cus * 4)),
                           dim3(BKT_THREADS), bm_lds, st, nb, boff, src, LB, HB, dst, nwrite);
        SPADE_HIP(ctx, hipGetLastError());
        return SPADE_OK;
    };
    // the keys of queries [q0, q1) at out[pbase[pair] - kbase ...]
    auto write_keys = [&](int q0, int q1, uint32_t *out, int64_t kbase) -> int {
        if (hits) {
            const int64_t p0 = (int64_t)hq[q0], p1 = (int64_t)hq[q1];
            if (p1 > p0) {
                const int eg = (int)std::min<int64_t>(p1 - p0, (int64_t)num_cus_of(ctx->device) * 8);
                hipLaunchKernelGGL(k_batch_emit_hits, dim3(eg), dim3(BT_THREADS), 0, st, p0, p1, P.pq, P.pc, hits,
                                   (const unsigned long long *)pbase, (const uint32_t *)t->ids.p, qrun0, idbits,
                                   out, (unsigned long long)kbase);
            }
        } else {
            hipLaunchKernelGGL(k_batch_select<true>, dim3(grid), dim3(BT_THREADS), 0, st, S, t->nfin, t->nchunk,
                               (const double *)t->x.p, (const double *)t->y.p, (const uint32_t *)t->ids.p, P.cbase,
                               P.plist, P.pq, nullptr, (const unsigned long long *)pbase, out, (uint32_t)q0,
                               (uint32_t)q1, (unsigned long long)kbase, qrun0, idbits, nullptr,
                               (const double4 *)t->chunk_bb.p);
        }
        SPADE_HIP(ctx, hipGetLastError());
        return SPADE_OK;
    };
    if (qdone > 0) {
        if ((rc = write_keys(0, qdone, out_ids, 0))) return rc;
        for (const auto &R : runs) {
            if (R.q1 > qdone) break;
            if (R.k1 > R.k0 && (rc = sort_run(R, out_ids + R.k0, out_ids + R.k0, R.k1 - R.k0))) return rc;
        }
    }
    if (cross >= 0) {
        const Run &R = runs[(size_t)cross];
        if ((rc = write_keys(R.q0, R.q1, (uint32_t *)bo.p, R.k0))) return rc;
        if ((rc = sort_run(R, (uint32_t *)bo.p, out_ids + R.k0, cap - R.k0))) return rc;
    }
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (short_cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // extern "C"

namespace spade {

void drop_batch_graph(spade_canvas *cv)
{
    if (cv->bexec) (void)hipGraphExecDestroy(cv->bexec);
    cv->bexec = nullptr;
    cv->bkey.clear();
}

// The batch join-count's launches (clear the counts, the canvas boxes, the
// one-pass probe) for the current buffers; all parameters are in `key`.
static hipError_t batch_count_launches(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, int64_t M,
                                       uint64_t *out_counts, hipStream_t s, const uint8_t *skip = nullptr)
{
    const int nq = set->nc;
    if (M > 0) hipLaunchKernelGGL(k_zero64, dim3(grid_of(M, 4096)), dim3(256), 0, s, M, (unsigned long long *)out_counts);
    hipLaunchKernelGGL(k_qbox, dim3((nq + 255) / 256), dim3(256), 0, s, nq, (const CanvasDesc *)set->dcds.p, skip,
                       (double4 *)set->qbox.p);
    const SetArgs S = set_args(set);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(t->nchunk, (int64_t)num_cus_of(ctx->device) * 8));
    if (t->nchunk > 0 && M > 0)
        hipLaunchKernelGGL(k_batch_count_direct, dim3(grid), dim3(BT_THREADS), 0, s, S, nq, t->nfin, t->nchunk,
                           (const double *)t->x.p, (const double *)t->y.p, (const double4 *)t->chunk_bb.p,
                           (const double4 *)set->qbox.p, (unsigned long long *)out_counts);
    return hipGetLastError();
}

}  // namespace spade

extern "C" {

int spade_batch_join_count(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, uint64_t *out_counts)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !set || !t) return ctx ? set_error(ctx, SPADE_E_INVALID, "NULL argument") : SPADE_E_INVALID;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    int64_t M = 0;
    for (const auto &d : set->descs) M += d.M;
    if (M > 0 && !out_counts) return set_error(ctx, SPADE_E_INVALID, "out_counts is NULL");
    hipStream_t st = ctx->stream;
    ctx->timed_raster = false;
    spade_canvas *cv = const_cast<spade_canvas *>(set);
    if (ensure(ctx, cv->qbox, sizeof(double4) * (size_t)std::max(set->nc, 1))) return SPADE_E_NOMEM;
    // The launches depend only on these values (every pointer and size they
    // take): a call with the same ones (the same set and table memory,
    // typically a rebuilt batch) replays the graph captured on the second
    // such call.
    const std::vector<uint64_t> key = {
        (uint64_t)(uintptr_t)set->dcds.p, (uint64_t)(uintptr_t)set->cells.p, (uint64_t)(uintptr_t)set->coarse.p,
        (uint64_t)(uintptr_t)set->cands.p, (uint64_t)(uintptr_t)set->ledges.p, (uint64_t)(uintptr_t)set->pspan.p,
        (uint64_t)(uintptr_t)set->qbox.p, (uint64_t)(uintptr_t)(set->layered ? set->pid.p : nullptr),
        (uint64_t)set->nc, (uint64_t)M, (uint64_t)(uintptr_t)t->x.p, (uint64_t)(uintptr_t)t->y.p,
        (uint64_t)(uintptr_t)t->chunk_bb.p, (uint64_t)t->nfin, (uint64_t)t->nchunk, (uint64_t)(uintptr_t)out_counts};
    // A canvas over at least a quarter of the table's box whose polygons fit
    // the count probe's LDS histogram is counted by that probe over all the
    // table's points (a canvas of a tessellation over the extent, say): it
    // streams them several times faster than the per-chunk probe looks them
    // up, which outweighs the per-chunk probe's one read of a chunk for all
    // the canvases that meet it.  Not for a layered set, whose counts go
    // through its polygon-id map.
    std::vector<int> routed;
    std::vector<uint8_t> hskip;   // read by an asynchronous copy: lives to the final synchronisation
    if (!set->layered) {
        const double tw = t->sx > 0 ? t->G / t->sx : 0.0, th = t->sy > 0 ? t->G / t->sy : 0.0;
        const double tx1 = t->X0 + tw, ty1 = t->Y0 + th;
        for (int q = 0; q < set->nc && t->nfin > 0; ++q) {
            const CanvasDesc &d = set->descs[(size_t)q];
            if (d.empty || d.M <= 0 || d.M > HIST_MAX_BATCH) continue;
            const double ox = std::min(d.bx1, tx1) - std::max(d.bx0, t->X0);
            const double oy = std::min(d.by1, ty1) - std::max(d.by0, t->Y0);
            if (ox > 0 && oy > 0 && ox * oy >= 0.25 * tw * th) routed.push_back(q);
        }
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    hipError_t e;
    if (!routed.empty()) {
        e = hipSuccess;
        const uint8_t *skip = nullptr;
        int64_t Mrest = 0;
        if ((int)routed.size() < set->nc) {
            hskip.assign((size_t)set->nc, 0);
            for (int q : routed) hskip[(size_t)q] = 1;
            for (int q = 0; q < set->nc; ++q)
                if (!hskip[(size_t)q]) Mrest += set->descs[(size_t)q].M;
            DevBuf &bs = ctx->scratch[S_MISC];
            if (ensure(ctx, bs, (size_t)set->nc)) return SPADE_E_NOMEM;
            SPADE_HIP(ctx, hipMemcpyAsync(bs.p, hskip.data(), (size_t)set->nc, hipMemcpyHostToDevice, st));
            skip = (const uint8_t *)bs.p;
        }
        if (Mrest > 0) e = batch_count_launches(ctx, set, t, M, out_counts, st, skip);
        const bool timing = ctx->timing;
        ctx->timing = false;   // the batch call's events frame every launch
        spade_points tp{};
        tp.n = t->nfin;
        tp.x = (const double *)t->x.p;
        tp.y = (const double *)t->y.p;
        for (int q : routed) {
            if (e != hipSuccess) break;
            const CanvasDesc &d = set->descs[(size_t)q];
            spade_canvas one;
            one.view = view_of(set, q);
            const int rc2 = probe_count(ctx, &one, &tp, out_counts + d.poly_base);
            if (rc2) {
                ctx->timing = timing;
                return rc2;
            }
        }
        ctx->timing = timing;
    } else if (!ctx->graphs) {
        e = batch_count_launches(ctx, set, t, M, out_counts, st);
    } else if (cv->bexec && cv->bkey == key) {
        ++ctx->graph_replays;
        e = hipGraphLaunch(cv->bexec, st);
    } else if (cv->bkey != key) {
        drop_batch_graph(cv);
        cv->bkey = key;
        e = batch_count_launches(ctx, set, t, M, out_counts, st);
    } else {
        // second call with these parameters: capture (on an internal stream,
        // the caller's may be the null stream), then launch the graph
        e = hipSuccess;
        if (!ctx->capture && (e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->capture = nullptr;
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        if (ctx->capture && hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const hipError_t e1 = batch_count_launches(ctx, set, t, M, out_counts, ctx->capture);
            const hipError_t e2 = hipStreamEndCapture(ctx->capture, &g);
            if (e1 == hipSuccess && e2 == hipSuccess && g &&
                hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
                cv->bexec = ex;
                ++ctx->graph_captures;
            }
            if (g) (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
        if (cv->bexec) e = hipGraphLaunch(cv->bexec, st);
        else {
            cv->bkey.clear();
            e = batch_count_launches(ctx, set, t, M, out_counts, st);
        }
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "batch join-count launches");
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    return SPADE_OK;
}

int spade_batch_join_pairs(spade_ctx *ctx, const spade_canvas *set, const spade_table *t, uint32_t *out_pt,
                           uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    if (!ctx) return SPADE_E_INVALID;
    SPADE_CTX_LOCK(ctx);
    if (!ctx || !set || !t || !n_out) return ctx ? set_error(ctx, SPADE_E_INVALID, "NULL argument") : SPADE_E_INVALID;
    ctx->err.clear();
    *n_out = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, SPADE_E_HIP, "hipSetDevice failed");
    if (cap < 0 || (cap > 0 && (!out_pt || !out_poly))) return set_error(ctx, SPADE_E_INVALID, "bad output buffers");
    int64_t M = 0;
    for (const auto &d : set->descs) M += d.M;
    hipStream_t st = ctx->stream;
    ctx->timed_raster = false;
    if (M == 0 || t->nchunk == 0) return SPADE_OK;
    Pairs P;
    int rc = make_pairs(ctx, set, t, P);
    if (rc) return rc;
    const SetArgs S = set_args(set);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(t->nchunk, (int64_t)num_cus_of(ctx->device) * 8));
    const int pbits = std::max(1, bits_of((uint64_t)(M - 1)));
    const int idbits = std::max(1, bits_of((uint64_t)(t->n - 1)));
    if (pbits + idbits > 64) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many polygons and points for 64-bit keys");
    int rshift = 0;
    while (((uint64_t)(t->n - 1) >> rshift) >= (uint64_t)PAIR_RANGES) ++rshift;
    DevBuf &bc = ctx->scratch[S_VALS2];
    if (ensure(ctx, bc, sizeof(unsigned long long) * (PAIR_RANGES + 8))) return SPADE_E_NOMEM;
    unsigned long long *rcount = (unsigned long long *)bc.p;
    unsigned long long *cursor = rcount + PAIR_RANGES;
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, st, (int64_t)(PAIR_RANGES + 1), rcount);
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (P.np > 0) {
        hipLaunchKernelGGL(k_batch_pairs<true>, dim3(grid), dim3(BT_THREADS), 0, st, S, t->nfin, t->nchunk,
                           (const double *)t->x.p, (const double *)t->y.p, (const uint32_t *)t->ids.p, P.cbase,
                           P.plist, P.pq, rshift, pbits, rcount, 0u, 0u, nullptr, nullptr,
                           (const double4 *)t->chunk_bb.p);
        SPADE_HIP(ctx, hipGetLastError());
    }
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, sizeof(unsigned long long) * PAIR_RANGES);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, rcount, sizeof(unsigned long long) * PAIR_RANGES, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    std::vector<unsigned long long> rc_h(h, h + PAIR_RANGES);
    unsigned long long total = 0;
    for (auto v : rc_h) total += v;
    *n_out = (int64_t)total;
    // runs of consecutive id ranges with at most 2^30 pairs each are written,
    // sorted and split one at a time (output order is by point id first)
    const int64_t GROUP = (int64_t)1 << 30;
    struct Run { uint32_t r0, r1; int64_t k0, k1; };
    std::vector<Run> runs;
    {
        uint32_t rb = 0;
        int64_t kb = 0, acc = 0;
        for (uint32_t r = 0; r < PAIR_RANGES; ++r) {
            if (acc + (int64_t)rc_h[r] > GROUP && r > rb) {
                runs.push_back({rb, r, kb, kb + acc});
                kb += acc;
                acc = 0;
                rb = r;
            }
            acc += (int64_t)rc_h[r];
        }
        if (acc > 0) runs.push_back({rb, (uint32_t)PAIR_RANGES, kb, kb + acc});
    }
    int64_t gmax = 0;
    for (const auto &r : runs)
        if (r.k0 < cap) gmax = std::max(gmax, r.k1 - r.k0);
    if (gmax >= (int64_t)INT32_MAX) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many pairs for one point-id range");
    if (gmax > 0) {
        DevBuf &bo = ctx->scratch[S_ENTC], &bo2 = ctx->scratch[S_ENTF];
        if (ensure(ctx, bo, 8 * (size_t)gmax) || ensure(ctx, bo2, 8 * (size_t)gmax)) return SPADE_E_NOMEM;
        DevBuf &cub = ctx->scratch[S_CUBTMP];
        size_t tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(nullptr, tb, (const unsigned long long *)bo.p,
                                                         (unsigned long long *)bo2.p, (int)gmax, 0, pbits + idbits, st));
        if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
        for (const auto &r : runs) {
            if (r.k0 >= cap) break;
            hipLaunchKernelGGL(k_zero64, dim3(1), dim3(64), 0, st, (int64_t)1, cursor);
            hipLaunchKernelGGL(k_batch_pairs<false>, dim3(grid), dim3(BT_THREADS), 0, st, S, t->nfin, t->nchunk,
                               (const double *)t->x.p, (const double *)t->y.p, (const uint32_t *)t->ids.p, P.cbase,
                               P.plist, P.pq, rshift, pbits, nullptr, r.r0, r.r1, cursor,
                               (unsigned long long *)bo.p, (const double4 *)t->chunk_bb.p);
            SPADE_HIP(ctx, hipGetLastError());
            SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(cub.p, tb, (const unsigned long long *)bo.p,
                                                             (unsigned long long *)bo2.p, (int)(r.k1 - r.k0), 0,
                                                             pbits + idbits, st));
            const int64_t nw = std::min<int64_t>(r.k1, cap) - r.k0;
            hipLaunchKernelGGL(k_split_pairs, dim3(grid_of(nw)), dim3(256), 0, st, nw,
                               (const unsigned long long *)bo2.p, pbits, out_pt + r.k0, out_poly + r.k0);
            SPADE_HIP(ctx, hipGetLastError());
        }
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if ((int64_t)total > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // extern "C"
