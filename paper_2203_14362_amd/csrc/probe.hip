// Point probes against a discrete canvas: the paper's mask + multiway blend
// (aggregation) and mask + Map (selection / join) applied to a stream of
// points (Sec. 5.1, 5.2), as compute kernels.
//
// Every point is read once from HBM (FP64 structure of arrays, coalesced),
// rejected if it lies outside the half-open bounding box of the polygons,
// mapped to its pixel and classified by the canvas word: a label is final,
// a boundary pixel runs the exact test of each candidate polygon.
//
//   k_count  per-polygon counts: workgroup-private histograms in LDS
//            (additive blend), flushed with one 64-bit atomic per polygon and
//            workgroup; polygon sets too large for LDS use global atomics.
//   k_emit   ordered output (point ids, or (point, polygon) pairs ascending):
//            the paper's Map into a null-padded list plus a scan, fused into
//            one pass with a decoupled look-back prefix over chunks of points
//            claimed in order.
#include "common.h"
#include "exact.h"

#include <algorithm>

namespace spade {

constexpr int PROBE_THREADS = 256;
constexpr int HIST_MAX = 16384;           // polygons counted in LDS
constexpr int EMIT_ITEMS = 16;            // points per thread per chunk
constexpr int EMIT_CHUNK = PROBE_THREADS * EMIT_ITEMS;

__device__ __forceinline__ uint32_t canvas_word(const CanvasView &cv, double x, double y)
{
    // exact half-open bbox test; NaN fails every comparison
    if (!(cv.bx0 <= x && x < cv.bx1 && cv.by0 <= y && y < cv.by1)) return 0u;
    const double u = __dmul_rn(__dsub_rn(x, cv.X0), cv.sx);
    const double v = __dmul_rn(__dsub_rn(y, cv.Y0), cv.sy);
    const int c = min((int)u, cv.W - 1);
    const int r = min((int)v, cv.H - 1);
    return cv.cells[(size_t)r * cv.W + c];
}

__device__ __forceinline__ bool cand_inside(const CanvasView &cv, const Cand &cd, double x, double y)
{
    bool in = (cd.meta & CAND_S) != 0;
    const uint32_t nloc = cd.meta >> 2;
    const uint32_t *el = cv.elist + cd.eoff;
    for (uint32_t t = 0; t < nloc; ++t) {
        const Edge e = cv.edges[el[t]];
        in ^= crosses(e.xlo, e.ylo, e.xhi, e.yhi, x, y);
    }
    for (uint32_t t = 0; t < cd.npart; ++t) {
        const Edge e = cv.edges[el[nloc + t]];
        in ^= straddles(e.ylo, e.yhi, y);
    }
    return in;
}

// ------------------------------------------------------------ join-count

template <bool LDS>
__global__ __launch_bounds__(PROBE_THREADS) void k_count(CanvasView cv, int64_t n, const double *X,
                                                         const double *Y,
                                                         unsigned long long *counts)
{
    extern __shared__ uint32_t hist[];
    const int M = (int)cv.M;
    if (LDS) {
        for (int k = threadIdx.x; k < M; k += PROBE_THREADS) hist[k] = 0;
        __syncthreads();
    }
    auto add = [&](uint32_t k) {
        if (LDS) atomicAdd(&hist[k], 1u);
        else atomicAdd(&counts[k], 1ull);
    };
    const int64_t stride = (int64_t)gridDim.x * PROBE_THREADS * 2;
    for (int64_t base = (int64_t)blockIdx.x * PROBE_THREADS * 2 + threadIdx.x; base < n; base += stride) {
        double xs[2], ys[2];
        bool ok[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = base + (int64_t)u * PROBE_THREADS;
            ok[u] = i < n;
            xs[u] = ok[u] ? __builtin_nontemporal_load(X + i) : 0.0;
            ys[u] = ok[u] ? __builtin_nontemporal_load(Y + i) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!ok[u]) continue;
            const uint32_t w = canvas_word(cv, xs[u], ys[u]);
            if (w == 0u) continue;
            if (!(w & BFLAG)) { add(w - 1u); continue; }
            uint32_t rec = w & ~BFLAG;
            while (true) {
                const Cand cd = cv.cands[rec];
                if (cand_inside(cv, cd, xs[u], ys[u])) add(cd.poly);
                if (cd.meta & CAND_LAST) break;
                ++rec;
            }
        }
    }
    if (LDS) {
        __syncthreads();
        for (int k = threadIdx.x; k < M; k += PROBE_THREADS) {
            const uint32_t c = hist[k];
            if (c) atomicAdd(&counts[k], (unsigned long long)c);
        }
    }
}

__global__ void k_zero_u64(int64_t n, unsigned long long *p)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) p[i] = 0ull;
}

static int num_cus(spade_ctx *ctx)
{
    static int cached = 0;
    if (!cached) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || v <= 0)
            v = 256;
        cached = v;
    }
    return cached;
}

int probe_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint64_t *out_counts)
{
    hipStream_t st = ctx->stream;
    const CanvasView &v = cv->view;
    const int64_t M = v.M;
    if (M > 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<int64_t>((M + 255) / 256, 1024)), dim3(256),
                           0, st, M, (unsigned long long *)out_counts);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (pts->n == 0 || M == 0) return SPADE_OK;
    const int cus = num_cus(ctx);
    const int64_t need = (pts->n + 2 * PROBE_THREADS - 1) / (2 * PROBE_THREADS);
    if (M <= HIST_MAX) {
        const size_t lds = sizeof(uint32_t) * (size_t)M;
        const int per_cu = M <= 2048 ? 8 : (M <= 8192 ? 2 : 1);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * per_cu));
        hipLaunchKernelGGL(k_count<true>, dim3(grid), dim3(PROBE_THREADS), lds, st, v, pts->n, pts->x,
                           pts->y, (unsigned long long *)out_counts);
    } else {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * 8));
        hipLaunchKernelGGL(k_count<false>, dim3(grid), dim3(PROBE_THREADS), 0, st, v, pts->n, pts->x,
                           pts->y, (unsigned long long *)out_counts);
    }
    SPADE_HIP(ctx, hipGetLastError());
    return SPADE_OK;
}

// ------------------------------------------------------------ ordered emit

constexpr unsigned long long LB_AGG = 1ull << 62;
constexpr unsigned long long LB_PRE = 2ull << 62;
constexpr unsigned long long LB_VAL = (1ull << 62) - 1;

// Block-wide exclusive scan of one value per thread (256 threads, 4 waves).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t pre = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < PROBE_THREADS / 64; ++q) {
        uint32_t s = wsum[q];
        if (q < wv) pre += s;
        total += s;
    }
    __syncthreads();
    return pre + inc - v;
}

__global__ __launch_bounds__(PROBE_THREADS) void k_emit(CanvasView cv, int64_t n, const double *X,
                                                        const double *Y, uint32_t *out_pt,
                                                        uint32_t *out_poly, int64_t cap,
                                                        unsigned long long *status,
                                                        unsigned int *chunk_ctr, int64_t nchunks,
                                                        unsigned long long *total_out)
{
    __shared__ uint32_t s_chunk;
    __shared__ uint32_t wsum[PROBE_THREADS / 64];
    __shared__ unsigned long long s_prefix;
    while (true) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(chunk_ctr, 1u);
        __syncthreads();
        const int64_t chunk = s_chunk;
        __syncthreads();
        if (chunk >= nchunks) return;
        const int64_t base = chunk * EMIT_CHUNK;

        uint32_t lab[EMIT_ITEMS];   // label of a single match, or first record for several
        uint32_t cnt[EMIT_ITEMS];
#pragma unroll
        for (int it = 0; it < EMIT_ITEMS; ++it) {
            const int64_t i = base + (int64_t)it * PROBE_THREADS + threadIdx.x;
            cnt[it] = 0;
            lab[it] = 0;
            if (i >= n) continue;
            const double x = __builtin_nontemporal_load(X + i), y = __builtin_nontemporal_load(Y + i);
            const uint32_t w = canvas_word(cv, x, y);
            if (w == 0u) continue;
            if (!(w & BFLAG)) { cnt[it] = 1; lab[it] = w - 1u; continue; }
            uint32_t rec = w & ~BFLAG, first = 0, m = 0;
            while (true) {
                const Cand cd = cv.cands[rec];
                if (cand_inside(cv, cd, x, y)) { if (m == 0) first = cd.poly; ++m; }
                if (cd.meta & CAND_LAST) break;
                ++rec;
            }
            if (m == 1) { cnt[it] = 1; lab[it] = first; }
            else if (m > 1) { cnt[it] = m; lab[it] = w & ~BFLAG; }
        }
        // counts in point order: item-major, thread-minor
        uint32_t excl[EMIT_ITEMS];
        uint32_t running = 0;
#pragma unroll
        for (int it = 0; it < EMIT_ITEMS; ++it) {
            uint32_t tot;
            uint32_t e = block_excl_scan(cnt[it], wsum, tot);
            excl[it] = running + e;
            running += tot;
        }
        // decoupled look-back for the chunk prefix
        if (threadIdx.x == 0) {
            unsigned long long prefix = 0;
            if (chunk == 0) {
                __hip_atomic_store(&status[0], LB_PRE | (unsigned long long)running, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(&status[chunk], LB_AGG | (unsigned long long)running, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                int64_t j = chunk - 1;
                while (true) {
                    unsigned long long s;
                    do {
                        s = __hip_atomic_load(&status[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    } while (s == 0ull);
                    prefix += s & LB_VAL;
                    if (s & LB_PRE) break;
                    --j;
                }
                __hip_atomic_store(&status[chunk], LB_PRE | (prefix + running), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            s_prefix = prefix;
            if (chunk == nchunks - 1) *total_out = prefix + running;
        }
        __syncthreads();
        const unsigned long long prefix = s_prefix;
#pragma unroll
        for (int it = 0; it < EMIT_ITEMS; ++it) {
            if (cnt[it] == 0) continue;
            const int64_t i = base + (int64_t)it * PROBE_THREADS + threadIdx.x;
            unsigned long long pos = prefix + excl[it];
            if (cnt[it] == 1) {
                if ((int64_t)pos < cap) {
                    out_pt[pos] = (uint32_t)i;
                    if (out_poly) out_poly[pos] = lab[it];
                }
                continue;
            }
            // several polygons contain the point: re-run its candidates in order
            const double x = X[i], y = Y[i];
            uint32_t rec = lab[it];
            while (true) {
                const Cand cd = cv.cands[rec];
                if (cand_inside(cv, cd, x, y)) {
                    if ((int64_t)pos < cap) {
                        out_pt[pos] = (uint32_t)i;
                        if (out_poly) out_poly[pos] = cd.poly;
                    }
                    ++pos;
                }
                if (cd.meta & CAND_LAST) break;
                ++rec;
            }
        }
        __syncthreads();
    }
}

__global__ void k_zero_u32(int64_t n, unsigned int *p)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) p[i] = 0u;
}

int probe_emit(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint32_t *out_pt,
               uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    hipStream_t st = ctx->stream;
    const int64_t n = pts->n;
    *n_out = 0;
    if (n == 0 || cv->view.M == 0) return SPADE_OK;
    const int64_t nchunks = (n + EMIT_CHUNK - 1) / EMIT_CHUNK;
    DevBuf &lb = ctx->scratch[S_LOOKBACK];
    if (ensure(ctx, lb, sizeof(unsigned long long) * (size_t)(nchunks + 2) + 64)) return SPADE_E_NOMEM;
    unsigned long long *status = (unsigned long long *)lb.p;
    unsigned long long *total = status + nchunks;
    unsigned int *ctr = (unsigned int *)(status + nchunks + 1);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<int64_t>((nchunks + 2 + 255) / 256, 4096)),
                       dim3(256), 0, st, nchunks + 2, status);
    SPADE_HIP(ctx, hipGetLastError());
    const int cus = num_cus(ctx);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, (int64_t)cus * 4));
    hipLaunchKernelGGL(k_emit, dim3(grid), dim3(PROBE_THREADS), 0, st, cv->view, n, pts->x, pts->y,
                       out_pt, out_poly, cap, status, ctr, nchunks, total);
    SPADE_HIP(ctx, hipGetLastError());
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, total, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *n_out = (int64_t)h[0];
    if (*n_out > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // namespace spade
