// Layer index (Sec. 4.3, "Layer Index"; creation in Sec. 5.5): the polygons
// of a set are split into layers such that no two polygons of one layer
// overlap on the index's pixel grid, so that each layer can be drawn as one
// canvas whose pixels each belong to at most one polygon (Sec. 5.2, spatial
// joins, case (1): one selection per layer).
//
// Coverage: a polygon covers the pixels whose centres it contains, by the
// crossing rule of the whole library evaluated on the grid's row-centre
// lines (edge crossings are bucketed to the first column centre at or right
// of them).  Neighbours of a tessellation share edges but no pixel centre,
// so a tessellation is one layer.  Overlaps smaller than the grid's pixels
// may remain inside a layer: the canvases resolve them exactly (a pixel
// claimed by two polygons becomes a boundary pixel), so layers only change
// speed, never results.
//
// Creation follows the paper's iteration.  With the polygons not yet in a
// layer:
//   pass 1 (multiway blend): every pixel keeps the highest id among the
//          remaining polygons covering it (atomic max of (iteration, id));
//   pass 2 (blend + mask): a remaining polygon any of whose pixels holds
//          another id was cropped and waits for a later iteration; the
//          others form this iteration's layer.
// The highest remaining id is never cropped, so every iteration makes a
// layer and the loop ends.  Polygons covering no pixel centre join the
// first layer.
//
// Layered canvas sets (spade_layered_build) rasterise each layer into its
// own canvas of a canvas set and keep the map from the set's polygon order
// (layer by layer) back to the caller's polygon ids; the batch calls over a
// resident table then report counts and pairs by the caller's ids.
#include "common.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace spade {

constexpr int LAYER_RES_DEFAULT = 1024;   // index grid: pixels on the long side
constexpr int LAYER_RES_MAX = 4096;
constexpr int KEY_COL_BITS = 13;           // column 0 .. 4096
constexpr int KEY_ROW_BITS = 12;           // row 0 .. 4095

struct LayerGrid {
    double X0, Y0, sx, sy;
    int W, H;
};

__device__ __forceinline__ int64_t find_seg(const int64_t *off, int64_t n, int64_t v)
{
    // largest i in [0, n) with off[i] <= v
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Rows whose centre line the edge (a, b) straddles (half-open in v).
__device__ __forceinline__ void edge_rows(double va, double vb, int H, int &r0, int &r1)
{
    const double lo = fmin(va, vb), hi = fmax(va, vb);
    // rows r with lo <= r + 0.5 < hi
    r0 = (int)fmax(0.0, ceil(lo - 0.5));
    r1 = (int)fmin((double)H, ceil(hi - 0.5));   // exclusive
    if (!(lo < hi)) r1 = r0;
}

// Pass over the vertices (edge j runs from vertex j to the next vertex of
// its ring): COUNT writes the entries per edge, FILL writes the keys
// (polygon, row, first column centre at or right of the crossing).
template <bool FILL>
__global__ __launch_bounds__(256) void k_layer_entries(int64_t V, int64_t R, const int64_t *rvo, const int64_t *pro,
                                                       int64_t M, const double *vx, const double *vy, LayerGrid g,
                                                       unsigned long long *count, const unsigned long long *off,
                                                       unsigned long long *keys)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < V; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = find_seg(rvo, R + 1, j);
        const int64_t a0 = rvo[r], a1 = rvo[r + 1];
        const int64_t k = j + 1 < a1 ? j + 1 : a0;
        double ua = (vx[j] - g.X0) * g.sx, va = (vy[j] - g.Y0) * g.sy;
        double ub = (vx[k] - g.X0) * g.sx, vb = (vy[k] - g.Y0) * g.sy;
        // endpoints in a fixed order, so that the two polygons sharing an
        // edge compute bit-identical crossings (and claim no centre twice)
        if (vb < va || (vb == va && ub < ua)) {
            double t = ua; ua = ub; ub = t;
            t = va; va = vb; vb = t;
        }
        int r0, r1;
        edge_rows(va, vb, g.H, r0, r1);
        if (!FILL) {
            count[j] = (unsigned long long)max(0, r1 - r0);
            continue;
        }
        if (r1 <= r0) continue;
        const int64_t p = pro ? find_seg(pro, M + 1, r) : r;
        const double du = (ub - ua) / (vb - va);
        unsigned long long at = off[j];
        for (int row = r0; row < r1; ++row) {
            const double u = ua + ((double)row + 0.5 - va) * du;
            const double cf = ceil(u - 0.5);
            const int c = (int)fmin((double)g.W, fmax(0.0, cf));
            keys[at++] = ((unsigned long long)p << (KEY_ROW_BITS + KEY_COL_BITS)) |
                         ((unsigned long long)row << KEY_COL_BITS) | (unsigned long long)c;
        }
    }
}

// Spans: sorted keys in consecutive pairs (a ring crosses a row-centre line
// an even number of times, so every (polygon, row) group has even size).
struct Span {
    uint32_t poly, row, c0, c1;
};

__global__ void k_layer_spans(int64_t S, const unsigned long long *keys, Span *spans)
{
    const unsigned long long cm = (1ull << KEY_COL_BITS) - 1, rm = (1ull << KEY_ROW_BITS) - 1;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long a = keys[2 * s], b = keys[2 * s + 1];
        Span sp;
        sp.poly = (uint32_t)(a >> (KEY_ROW_BITS + KEY_COL_BITS));
        sp.row = (uint32_t)((a >> KEY_COL_BITS) & rm);
        sp.c0 = (uint32_t)(a & cm);
        sp.c1 = (uint32_t)(b & cm);
        spans[s] = sp;
    }
}

// Pass 1: multiway blend keeping the highest id (tagged by iteration so the
// previous iterations' values lose without clearing the grid).
__global__ void k_layer_blend(int64_t S, const Span *spans, const int32_t *layer, int W, unsigned long long tag,
                              unsigned long long *cmax)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const Span sp = spans[s];
        if (layer[sp.poly] >= 0) continue;
        const unsigned long long v = (tag << 32) | (unsigned long long)(sp.poly + 1u);
        unsigned long long *rowp = cmax + (size_t)sp.row * W;
        for (uint32_t c = sp.c0; c < sp.c1; ++c) atomicMax(rowp + c, v);
    }
}

// Pass 2: a remaining polygon with a pixel holding another id is cropped.
__global__ void k_layer_mask(int64_t S, const Span *spans, const int32_t *layer, int W, unsigned long long tag,
                             const unsigned long long *cmax, int32_t *cropped)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        const Span sp = spans[s];
        if (layer[sp.poly] >= 0) continue;
        const unsigned long long v = (tag << 32) | (unsigned long long)(sp.poly + 1u);
        const unsigned long long *rowp = cmax + (size_t)sp.row * W;
        for (uint32_t c = sp.c0; c < sp.c1; ++c)
            if (rowp[c] != v) {
                cropped[sp.poly] = (int32_t)tag;
                break;
            }
    }
}

// Uncropped remaining polygons join layer `it`; *left counts the rest.
__global__ void k_layer_assign(int64_t M, int32_t it, int32_t *layer, const int32_t *cropped,
                               unsigned long long *left)
{
    unsigned long long mine = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        if (layer[p] >= 0) continue;
        if (cropped[p] == it + 1) ++mine;
        else layer[p] = it;
    }
    for (int d = 32; d > 0; d >>= 1) mine += __shfl_xor(mine, d, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(left, mine);
}

__global__ void k_layer_init(int64_t M, int32_t *layer, int32_t *cropped)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        layer[p] = -1;
        cropped[p] = 0;
    }
}

__global__ void k_fill_zero64(int64_t n, unsigned long long *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

static int grid_n(int64_t n, int64_t cap = 65536)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

static int nbits(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// Host copies of a polygon set's offsets, checked; vertex bounding box.
struct HostSet {
    int64_t M = 0, R = 0, V = 0;
    std::vector<int64_t> pro, rvo;
    double x0 = 0, x1 = 0, y0 = 0, y1 = 0;
};

static int host_offsets(spade_ctx *ctx, const spade_polys *polys, HostSet &h)
{
    hipStream_t st = ctx->stream;
    h.M = polys->n_polys;
    h.R = polys->n_rings;
    h.rvo.assign((size_t)h.R + 1, 0);
    if (h.R > 0)
        SPADE_HIP(ctx, hipMemcpyAsync(h.rvo.data(), polys->ring_vtx_off, sizeof(int64_t) * (size_t)(h.R + 1),
                                      hipMemcpyDeviceToHost, st));
    if (polys->poly_ring_off) {
        h.pro.assign((size_t)h.M + 1, 0);
        SPADE_HIP(ctx, hipMemcpyAsync(h.pro.data(), polys->poly_ring_off, sizeof(int64_t) * (size_t)(h.M + 1),
                                      hipMemcpyDeviceToHost, st));
    }
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (h.rvo[0] != 0) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off[0] must be 0");
    for (int64_t r = 0; r < h.R; ++r)
        if (h.rvo[r + 1] < h.rvo[r]) return set_error(ctx, SPADE_E_INVALID, "ring_vtx_off must be non-decreasing");
    if (polys->poly_ring_off) {
        if (h.pro[0] != 0 || h.pro[h.M] != h.R)
            return set_error(ctx, SPADE_E_INVALID, "poly_ring_off must run from 0 to n_rings");
        for (int64_t k = 0; k < h.M; ++k)
            if (h.pro[k + 1] < h.pro[k]) return set_error(ctx, SPADE_E_INVALID, "poly_ring_off must be non-decreasing");
    }
    h.V = h.rvo[h.R];
    if (polys->n_vertices > 0 && polys->n_vertices != h.V)
        return set_error(ctx, SPADE_E_INVALID, "n_vertices does not match ring_vtx_off[n_rings]");
    return SPADE_OK;
}

__global__ __launch_bounds__(256) void k_vbox(int64_t V, const double *vx, const double *vy, double *part,
                                              unsigned *bad)
{
    __shared__ double s[4][256];
    double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
    unsigned nf = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = vx[i], y = vy[i];
        if (!isfinite(x) || !isfinite(y)) { nf = 1; continue; }
        a = fmin(a, x); b = fmax(b, x); c = fmin(c, y); d = fmax(d, y);
    }
    if (nf) atomicOr(bad, 1u);
    s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

int layer_index(spade_ctx *ctx, const spade_polys *polys, int res, int32_t *d_layer, int32_t *n_layers,
                std::vector<int32_t> *host_layer, HostSet *hs_out)
{
    hipStream_t st = ctx->stream;
    HostSet hs;
    int rc = host_offsets(ctx, polys, hs);
    if (rc) return rc;
    const int64_t M = hs.M, R = hs.R, V = hs.V;
    *n_layers = 0;
    if (M == 0) {
        if (hs_out) *hs_out = std::move(hs);
        return SPADE_OK;
    }
    if (M >= ((int64_t)1 << 31) - 1) return set_error(ctx, SPADE_E_TOO_LARGE, "too many polygons");
    // vertex box (and finiteness)
    const int vb = 256;
    DevBuf &wb = ctx->scratch[S_BLOCKRED];
    if (ensure(ctx, wb, sizeof(double) * 4 * vb + 64)) return SPADE_E_NOMEM;
    double *part = (double *)wb.p;
    unsigned *bad = (unsigned *)(part + 4 * vb);
    hipLaunchKernelGGL(k_fill_zero64, dim3(1), dim3(64), 0, st, (int64_t)1, (unsigned long long *)bad);
    hipLaunchKernelGGL(k_vbox, dim3(vb), dim3(256), 0, st, V, polys->vx, polys->vy, part, bad);
    SPADE_HIP(ctx, hipGetLastError());
    std::vector<double> hp(4 * vb + 8);
    SPADE_HIP(ctx, hipMemcpyAsync(hp.data(), part, sizeof(double) * 4 * vb + 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    unsigned hb;
    std::memcpy(&hb, hp.data() + 4 * vb, sizeof hb);
    if (hb) return set_error(ctx, SPADE_E_INVALID, "non-finite polygon vertex");
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int b = 0; b < vb; ++b) {
        x0 = std::min(x0, hp[4 * b]); x1 = std::max(x1, hp[4 * b + 1]);
        y0 = std::min(y0, hp[4 * b + 2]); y1 = std::max(y1, hp[4 * b + 3]);
    }
    hs.x0 = x0; hs.x1 = x1; hs.y0 = y0; hs.y1 = y1;
    // grid over the box, aspect kept, `res` pixels on the long side
    if (res <= 0) res = LAYER_RES_DEFAULT;
    res = std::min(res, LAYER_RES_MAX);
    LayerGrid g{};
    const double w = x1 - x0, h = y1 - y0;
    if (!(w > 0) || !(h > 0)) {
        g.W = g.H = 1;
    } else if (w >= h) {
        g.W = res;
        g.H = std::max(1, std::min(res, (int)std::ceil(res * h / w)));
    } else {
        g.H = res;
        g.W = std::max(1, std::min(res, (int)std::ceil(res * w / h)));
    }
    g.X0 = x0; g.Y0 = y0;
    g.sx = w > 0 ? g.W / w : 0.0;
    g.sy = h > 0 ? g.H / h : 0.0;

    // per-layer state
    DevBuf &bl = ctx->scratch[S_ROWCNT];
    if (ensure(ctx, bl, sizeof(int32_t) * (size_t)M + 64)) return SPADE_E_NOMEM;
    int32_t *cropped = (int32_t *)bl.p;
    unsigned long long *left = (unsigned long long *)(((uintptr_t)(cropped + M) + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_layer_init, dim3(grid_n(M)), dim3(256), 0, st, M, d_layer, cropped);
    SPADE_HIP(ctx, hipGetLastError());

    // entries -> sorted keys -> spans
    int64_t S = 0;
    Span *spans = nullptr;
    if (V > 0 && g.sx > 0 && g.sy > 0) {
        DevBuf &bc = ctx->scratch[S_NROWS], &bo = ctx->scratch[S_ROWOFF];
        if (ensure(ctx, bc, sizeof(unsigned long long) * (size_t)(V + 1)) ||
            ensure(ctx, bo, sizeof(unsigned long long) * (size_t)(V + 1)))
            return SPADE_E_NOMEM;
        // 64-bit counts: the scan accumulates in the input's type
        unsigned long long *cnt = (unsigned long long *)bc.p;
        unsigned long long *off = (unsigned long long *)bo.p;
        const int64_t *pro_d = polys->poly_ring_off;
        hipLaunchKernelGGL(k_layer_entries<false>, dim3(grid_n(V)), dim3(256), 0, st, V, R, polys->ring_vtx_off,
                           pro_d, M, polys->vx, polys->vy, g, cnt, nullptr, nullptr);
        hipLaunchKernelGGL(k_fill_zero64, dim3(1), dim3(64), 0, st, (int64_t)1, cnt + V);   // the scan's total slot
        SPADE_HIP(ctx, hipGetLastError());
        DevBuf &cub = ctx->scratch[S_CUBTMP];
        size_t tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)(V + 1), st));
        if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, cnt, off, (int)(V + 1), st));
        unsigned long long E = 0;
        SPADE_HIP(ctx, hipMemcpyAsync(&E, off + V, sizeof E, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        if (E & 1ull) return set_error(ctx, SPADE_E_HIP, "internal: odd number of layer-grid crossings");
        if (E >= ((unsigned long long)1 << 31)) return set_error(ctx, SPADE_E_UNSUPPORTED, "layer grid too fine");
        S = (int64_t)(E / 2);
        if (E > 0) {
            DevBuf &bk = ctx->scratch[S_KEYS], &bk2 = ctx->scratch[S_KEYS2], &bs = ctx->scratch[S_VALS];
            if (ensure(ctx, bk, 8 * (size_t)E) || ensure(ctx, bk2, 8 * (size_t)E) ||
                ensure(ctx, bs, sizeof(Span) * (size_t)S))
                return SPADE_E_NOMEM;
            hipLaunchKernelGGL(k_layer_entries<true>, dim3(grid_n(V)), dim3(256), 0, st, V, R, polys->ring_vtx_off,
                               pro_d, M, polys->vx, polys->vy, g, nullptr, off, (unsigned long long *)bk.p);
            SPADE_HIP(ctx, hipGetLastError());
            const int kb = KEY_ROW_BITS + KEY_COL_BITS + std::max(1, nbits((uint64_t)(M - 1)));
            tb = 0;
            SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(nullptr, tb, (const unsigned long long *)bk.p,
                                                             (unsigned long long *)bk2.p, (int)E, 0, kb, st));
            if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
            SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(cub.p, tb, (const unsigned long long *)bk.p,
                                                             (unsigned long long *)bk2.p, (int)E, 0, kb, st));
            spans = (Span *)bs.p;
            hipLaunchKernelGGL(k_layer_spans, dim3(grid_n(S)), dim3(256), 0, st, S,
                               (const unsigned long long *)bk2.p, spans);
            SPADE_HIP(ctx, hipGetLastError());
        }
    }

    // iterations
    DevBuf &bg = ctx->scratch[S_ENTC];
    const int64_t npx = (int64_t)g.W * g.H;
    if (S > 0) {
        if (ensure(ctx, bg, 8 * (size_t)npx)) return SPADE_E_NOMEM;
        hipLaunchKernelGGL(k_fill_zero64, dim3(grid_n(npx, 4096)), dim3(256), 0, st, npx,
                           (unsigned long long *)bg.p);
    }
    unsigned long long *hleft = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!hleft) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    int32_t it = 0;
    for (;; ++it) {
        if (it >= (int32_t)M + 1) return set_error(ctx, SPADE_E_HIP, "internal: layer iteration did not end");
        hipLaunchKernelGGL(k_fill_zero64, dim3(1), dim3(64), 0, st, (int64_t)1, left);
        if (S > 0) {
            const unsigned long long tag = (unsigned long long)it + 1;
            hipLaunchKernelGGL(k_layer_blend, dim3(grid_n(S)), dim3(256), 0, st, S, spans, d_layer, g.W, tag,
                               (unsigned long long *)bg.p);
            hipLaunchKernelGGL(k_layer_mask, dim3(grid_n(S)), dim3(256), 0, st, S, spans, d_layer, g.W, tag,
                               (const unsigned long long *)bg.p, cropped);
        }
        hipLaunchKernelGGL(k_layer_assign, dim3(grid_n(M)), dim3(256), 0, st, M, it, d_layer, cropped, left);
        SPADE_HIP(ctx, hipGetLastError());
        SPADE_HIP(ctx, hipMemcpyAsync(hleft, left, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        if (hleft[0] == 0) break;
    }
    *n_layers = it + 1;
    if (host_layer) {
        host_layer->assign((size_t)M, 0);
        SPADE_HIP(ctx, hipMemcpyAsync(host_layer->data(), d_layer, sizeof(int32_t) * (size_t)M,
                                      hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
    }
    if (hs_out) *hs_out = std::move(hs);
    return SPADE_OK;
}

}  // namespace spade

namespace spade {

// Copies polygon perm[k] of the source set to position k of the destination
// (one workgroup per polygon; vertex ranges precomputed on the host).
__global__ __launch_bounds__(256) void k_perm_vertices(int64_t M, const int64_t *src0, const int64_t *dst0,
                                                       const double *vx, const double *vy, double *ox, double *oy)
{
    for (int64_t k = blockIdx.x; k < M; k += gridDim.x) {
        const int64_t s = src0[k], d = dst0[k], n = dst0[k + 1] - dst0[k];
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            ox[d + i] = vx[s + i];
            oy[d + i] = vy[s + i];
        }
    }
}

int layered_build(spade_ctx *ctx, const spade_polys *polys, int res, spade_canvas *cv, int32_t *n_layers_out)
{
    hipStream_t st = ctx->stream;
    const int64_t M = polys->n_polys;
    DevBuf dl;
    auto release = [&]() { free_buf(dl); };
    if (ensure(ctx, dl, sizeof(int32_t) * (size_t)std::max<int64_t>(M, 1))) return SPADE_E_NOMEM;
    std::vector<int32_t> lay;
    HostSet hs;
    int32_t L = 0;
    int rc = layer_index(ctx, polys, res, (int32_t *)dl.p, &L, &lay, &hs);
    release();
    if (rc) return rc;
    if (M == 0) L = 1;
    // stable order by layer: perm[k] = caller's polygon at set position k
    std::vector<int64_t> first((size_t)L + 1, 0);
    for (int64_t p = 0; p < M; ++p) first[(size_t)lay[p] + 1]++;
    for (int32_t l = 0; l < L; ++l) first[l + 1] += first[l];
    std::vector<int64_t> fill(first.begin(), first.end() - 1);
    std::vector<uint32_t> perm((size_t)M);
    for (int64_t p = 0; p < M; ++p) perm[(size_t)fill[(size_t)lay[p]]++] = (uint32_t)p;
    // the permuted CSR: rings and vertices of each polygon moved together
    const int64_t R = hs.R;
    auto rb = [&](int64_t p) { return hs.pro.empty() ? p : hs.pro[p]; };
    std::vector<int64_t> npro((size_t)M + 1, 0), nrvo((size_t)R + 1, 0), src0((size_t)M), dst0((size_t)M + 1, 0);
    int64_t nr = 0, nv = 0;
    for (int64_t k = 0; k < M; ++k) {
        const int64_t p = perm[k];
        src0[k] = hs.rvo[rb(p)];
        dst0[k] = nv;
        for (int64_t r = rb(p); r < rb(p + 1); ++r) {
            nv += hs.rvo[r + 1] - hs.rvo[r];
            nrvo[++nr] = nv;
        }
        npro[k + 1] = nr;
    }
    dst0[M] = nv;
    DevBuf dpro, drvo, dsrc, ddst, dvx, dvy;
    auto fail = [&](int code) {
        free_buf(dpro); free_buf(drvo); free_buf(dsrc); free_buf(ddst); free_buf(dvx); free_buf(dvy);
        return code;
    };
    if (ensure(ctx, dpro, 8 * npro.size()) || ensure(ctx, drvo, 8 * nrvo.size()) ||
        ensure(ctx, dsrc, 8 * std::max<size_t>(src0.size(), 1)) || ensure(ctx, ddst, 8 * dst0.size()) ||
        ensure(ctx, dvx, 8 * (size_t)std::max<int64_t>(nv, 1)) || ensure(ctx, dvy, 8 * (size_t)std::max<int64_t>(nv, 1)) ||
        ensure(ctx, cv->pid, 4 * (size_t)std::max<int64_t>(M, 1)))
        return fail(SPADE_E_NOMEM);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(dpro.p, npro.data(), 8 * npro.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(drvo.p, nrvo.data(), 8 * nrvo.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && M > 0) e = hipMemcpyAsync(dsrc.p, src0.data(), 8 * src0.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ddst.p, dst0.data(), 8 * dst0.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && M > 0) e = hipMemcpyAsync(cv->pid.p, perm.data(), 4 * perm.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)fail(0);
        return hip_fail(ctx, e, "layered set upload");
    }
    if (M > 0) {
        hipLaunchKernelGGL(k_perm_vertices, dim3((unsigned)std::min<int64_t>(M, 65535)), dim3(256), 0, st, M,
                           (const int64_t *)dsrc.p, (const int64_t *)ddst.p, polys->vx, polys->vy, (double *)dvx.p,
                           (double *)dvy.p);
        if ((e = hipGetLastError()) != hipSuccess) {
            (void)fail(0);
            return hip_fail(ctx, e, "k_perm_vertices");
        }
    }
    spade_polys np{};
    np.n_polys = M;
    np.n_rings = R;
    np.poly_ring_off = (const int64_t *)dpro.p;
    np.ring_vtx_off = (const int64_t *)drvo.p;
    np.vx = (const double *)dvx.p;
    np.vy = (const double *)dvy.p;
    np.n_vertices = nv;
    np.bbox = nullptr;
    rc = build_set(ctx, &np, (int)L, first.data(), cv);
    // the build has read the permuted arrays by the time it returns (it
    // synchronises); free them only after the stream has passed them
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    (void)fail(0);
    if (rc) return rc;
    cv->layered = M > 0;
    if (n_layers_out) *n_layers_out = L;
    return SPADE_OK;
}

}  // namespace spade
