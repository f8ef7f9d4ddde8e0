// Point probes against a discrete canvas: the paper's mask + multiway blend
// (aggregation) and mask + Map (selection / join) applied to a stream of
// points (Sec. 5.1, 5.2), as compute kernels.
//
// Every point is read once from HBM (FP64 structure of arrays, coalesced,
// non-temporal), rejected if it lies outside the half-open bounding box of
// the polygons and mapped to its pixel.  The pixel is classified in two
// levels: a coarse canvas held in LDS by every workgroup answers directly
// for blocks whose pixels share one label; points in any other block read their
// canvas word from the tile-major canvas in global memory (L2 / MALL).  A
// label is final; a boundary pixel needs the exact test of each candidate
// polygon.  Boundary points are compacted per wavefront (ballot + prefix
// count) into an LDS queue and tested in full wavefronts, so the rare,
// latency-bound exact tests do not stall the stream.
//
//   k_count  per-polygon counts: workgroup-private histograms in LDS
//            (additive blend), flushed into a context accumulator; the last
//            workgroup copies the counts out and clears the accumulator.
//   k_emit   ordered output (point ids, or (point, polygon) pairs ascending):
//            the paper's Map into a null-padded list plus a scan, fused into
//            one pass with a decoupled look-back prefix over chunks of points
//            claimed in order.
#include "common.h"
#include "exact.h"
#include "lookup.h"

#include <algorithm>

namespace spade {

constexpr int CNT_THREADS = 1024;         // count probe workgroup
constexpr int CNT_UNROLL = 5;             // points per thread per iteration (6 spills)
constexpr int QCAP = 64;                  // boundary queue entries per wavefront
constexpr int HIST_MAX = 8192;            // polygons counted in LDS
constexpr int EMIT_THREADS = 512;
constexpr int EMIT_ITEMS = 8;             // points per thread per chunk
constexpr int EMIT_CHUNK = EMIT_THREADS * EMIT_ITEMS;
constexpr size_t LDS_TOTAL = 160 * 1024;
constexpr size_t LDS_RESERVE = 2048;      // static LDS of the kernels
constexpr size_t QUEUE_BYTES = (size_t)(CNT_THREADS / 64) * QCAP * 20;

size_t coarse_lds_budget(int64_t M)
{
    size_t hist = (M <= HIST_MAX) ? sizeof(uint32_t) * (size_t)M : 0;
    size_t used = LDS_RESERVE + QUEUE_BYTES + hist;
    return used < LDS_TOTAL ? LDS_TOTAL - used : 0;
}

// ------------------------------------------------------------ join-count

// Counts accumulate in a context-owned accumulator `acc` that is all zero
// between calls: the last workgroup to finish (found with a counter, after a
// device-scope fence) copies acc into the caller's output and clears acc and
// the counter again, so a query is a single kernel launch with no memset.
template <bool LDSHIST>
__global__ __launch_bounds__(CNT_THREADS) void k_count(CanvasView cv, int64_t n, const double *X,
                                                       const double *Y, unsigned long long *acc,
                                                       unsigned int *done, unsigned long long *out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ bool s_last;
    const int M = (int)cv.M;
    const size_t coarse_bytes = ((size_t)cv.Wc * cv.Hc * (cv.cbyte ? 1 : 2) + 15) & ~(size_t)15;
    uint16_t *coarse = (uint16_t *)smem;
    uint32_t *hist = (uint32_t *)(smem + coarse_bytes);
    const size_t hist_bytes = LDSHIST ? (((size_t)M * 4 + 15) & ~(size_t)15) : 0;
    unsigned char *qbase = smem + coarse_bytes + hist_bytes;
    const int wv = threadIdx.x >> 6;
    double *qx = (double *)(qbase) + wv * QCAP;
    double *qy = (double *)(qbase) + (CNT_THREADS / 64) * QCAP + wv * QCAP;
    uint32_t *qr = (uint32_t *)((double *)(qbase) + 2 * (CNT_THREADS / 64) * QCAP) + wv * QCAP;

    load_coarse(cv, coarse, CNT_THREADS);
    if (LDSHIST)
        for (int k = threadIdx.x; k < M; k += CNT_THREADS) hist[k] = 0;
    __syncthreads();

    auto add = [&](uint32_t k) {
        if (LDSHIST) atomicAdd(&hist[k], 1u);
        else atomicAdd(&acc[k], 1ull);
    };
    const uint32_t lane = lane_id();
    uint32_t qn = 0;   // wave-uniform queue length
    auto drain = [&]() {
        __builtin_amdgcn_wave_barrier();
        if (lane < qn) {
            const double x = qx[lane], y = qy[lane];
            // a pixel's records two at a time (most pixels have two; the
            // slot after the last record exists and is never used)
            uint32_t rec = qr[lane];
            while (true) {
                const Cand c0 = cv.cands[rec];
                const Cand c1 = cv.cands[rec + 1];
                if (cand_inside(cv, c0, x, y)) add(c0.poly);
                if (c0.meta & CAND_LAST) break;
                if (cand_inside(cv, c1, x, y)) add(c1.poly);
                if (c1.meta & CAND_LAST) break;
                rec += 2;
            }
        }
        __builtin_amdgcn_wave_barrier();
        qn = 0;
    };

    // software pipeline: the next iteration's points are in flight while the
    // current ones are classified
    const int64_t step = (int64_t)gridDim.x * CNT_THREADS * CNT_UNROLL;
    double xn[CNT_UNROLL], yn[CNT_UNROLL];
    auto fetch = [&](int64_t b) {
#pragma unroll
        for (int u = 0; u < CNT_UNROLL; ++u) {
            const int64_t i = b + (int64_t)u * CNT_THREADS + threadIdx.x;
            xn[u] = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            yn[u] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
        }
    };
    int64_t base = (int64_t)blockIdx.x * CNT_THREADS * CNT_UNROLL;
    if (base < n) fetch(base);
    for (; base < n; base += step) {
        double xs[CNT_UNROLL], ys[CNT_UNROLL];
#pragma unroll
        for (int u = 0; u < CNT_UNROLL; ++u) { xs[u] = xn[u]; ys[u] = yn[u]; }
        if (base + step < n) fetch(base + step);
        // the coarse words of all points of this iteration first, then
        // their full-canvas reads, all issued before any result is used
        Look lk[CNT_UNROLL];
        uint32_t ws[CNT_UNROLL];
#pragma unroll
        for (int u = 0; u < CNT_UNROLL; ++u) lk[u] = look_coarse(cv, coarse, xs[u], ys[u]);
#pragma unroll
        for (int u = 0; u < CNT_UNROLL; ++u)
            ws[u] = lk[u].full ? ((gu32p)cv.cells)[lk[u].fidx] : lk[u].word;
#pragma unroll
        for (int u = 0; u < CNT_UNROLL; ++u) {
            const uint32_t w = ws[u];
            const bool bnd = (w & BFLAG) != 0;
            if (w != 0u && !bnd) add(w - 1u);
            const unsigned long long mask = __ballot(bnd);
            const uint32_t nnew = (uint32_t)__popcll(mask);
            if (nnew == 0) continue;
            if (qn + nnew > QCAP) drain();
            if (bnd) {
                const uint32_t slot = qn + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                qx[slot] = xs[u];
                qy[slot] = ys[u];
                qr[slot] = w & ~BFLAG;
            }
            qn += nnew;
        }
    }
    if (qn) drain();

    if (LDSHIST) {
        __syncthreads();
        for (int k = threadIdx.x; k < M; k += CNT_THREADS) {
            const uint32_t c = hist[k];
            if (c) atomicAdd(&acc[k], (unsigned long long)c);
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(done, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int k = threadIdx.x; k < M; k += CNT_THREADS) {
        out[k] = __hip_atomic_load(&acc[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc[k] = 0ull;
    }
    if (threadIdx.x == 0) *done = 0u;
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

// The accumulator lives in a context scratch slot that is zeroed whenever it
// is (re)allocated; k_count leaves it zeroed.
static int count_acc(spade_ctx *ctx, int64_t M, unsigned long long **acc, unsigned int **done)
{
    DevBuf &b = ctx->scratch[S_PROBE];
    const size_t need = sizeof(unsigned long long) * (size_t)(M + 1);
    if (b.cap < need) {
        if (ensure(ctx, b, need)) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipMemsetAsync(b.p, 0, b.cap, ctx->stream));
    }
    *acc = (unsigned long long *)b.p;
    *done = (unsigned int *)((unsigned long long *)b.p + M);
    return SPADE_OK;
}

static size_t coarse_bytes_of(const CanvasView &v)
{
    return ((size_t)v.Wc * v.Hc * (v.cbyte ? 1 : 2) + 15) & ~(size_t)15;
}

int probe_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint64_t *out_counts)
{
    hipStream_t st = ctx->stream;
    const CanvasView &v = cv->view;
    const int64_t M = v.M;
    if (M == 0) return SPADE_OK;
    unsigned long long *acc = nullptr;
    unsigned int *done = nullptr;
    int rc = count_acc(ctx, M, &acc, &done);
    if (rc) return rc;
    const int cus = num_cus(ctx);
    const bool ldshist = M <= HIST_MAX;
    const size_t lds = coarse_bytes_of(v) + (ldshist ? (((size_t)M * 4 + 15) & ~(size_t)15) : 0) + QUEUE_BYTES;
    if (lds + LDS_RESERVE > LDS_TOTAL) return set_error(ctx, SPADE_E_HIP, "internal: probe LDS budget exceeded");
    const int64_t need = std::max<int64_t>(1, (pts->n + CNT_THREADS * CNT_UNROLL - 1) / (CNT_THREADS * CNT_UNROLL));
    // one workgroup per CU even where the LDS would hold two: a second one
    // slows the stream down (measured), so spare LDS goes to a finer coarse
    // level instead
    const int grid = (int)std::min<int64_t>(need, (int64_t)cus);
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (ldshist) {
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_count<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_count<true>, dim3(grid), dim3(CNT_THREADS), lds, st, v, pts->n, pts->x,
                           pts->y, acc, done, (unsigned long long *)out_counts);
    } else {
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_count<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_count<false>, dim3(grid), dim3(CNT_THREADS), lds, st, v, pts->n, pts->x,
                           pts->y, acc, done, (unsigned long long *)out_counts);
    }
    SPADE_HIP(ctx, hipGetLastError());
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    return SPADE_OK;
}

// ------------------------------------------------------------ ordered emit

constexpr unsigned long long LB_AGG = 1ull << 62;
constexpr unsigned long long LB_PRE = 2ull << 62;
constexpr unsigned long long LB_VAL = (1ull << 62) - 1;

// Block-wide exclusive scan of one value per thread (EMIT_THREADS threads).
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
    for (int q = 0; q < EMIT_THREADS / 64; ++q) {
        uint32_t s = wsum[q];
        if (q < wv) pre += s;
        total += s;
    }
    __syncthreads();
    return pre + inc - v;
}

__global__ __launch_bounds__(EMIT_THREADS) void k_emit(CanvasView cv, int64_t n, const double *X,
                                                       const double *Y, uint32_t *out_pt,
                                                       uint32_t *out_poly, int64_t cap,
                                                       unsigned long long *status,
                                                       unsigned int *chunk_ctr, int64_t nchunks,
                                                       unsigned long long *total_out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_chunk;
    __shared__ uint32_t wsum[EMIT_THREADS / 64];
    __shared__ unsigned long long s_prefix;
    uint16_t *coarse = (uint16_t *)smem;
    load_coarse(cv, coarse, EMIT_THREADS);
    __syncthreads();
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
            const int64_t i = base + (int64_t)it * EMIT_THREADS + threadIdx.x;
            cnt[it] = 0;
            lab[it] = 0;
            if (i >= n) continue;
            const double x = __builtin_nontemporal_load(X + i), y = __builtin_nontemporal_load(Y + i);
            const uint32_t w = lookup(cv, coarse, x, y);
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
            const int64_t i = base + (int64_t)it * EMIT_THREADS + threadIdx.x;
            unsigned long long pos = prefix + excl[it];
            if (cnt[it] == 1) {
                if ((int64_t)pos < cap) {
                    out_pt[pos] = (uint32_t)i;
                    if (out_poly) out_poly[pos] = lab[it];
                }
                continue;
            }
            // several polygons contain the point (the pixel's records are in
            // no particular order): emit them in ascending polygon order, each
            // pass taking the smallest matching polygon above the last one
            const double x = X[i], y = Y[i];
            uint32_t prev = 0;
            for (uint32_t t = 0; t < cnt[it]; ++t) {
                uint32_t best = 0xffffffffu;
                uint32_t rec = lab[it];
                while (true) {
                    const Cand cd = cv.cands[rec];
                    if ((t == 0 || cd.poly > prev) && cd.poly < best && cand_inside(cv, cd, x, y)) best = cd.poly;
                    if (cd.meta & CAND_LAST) break;
                    ++rec;
                }
                if ((int64_t)pos < cap) {
                    out_pt[pos] = (uint32_t)i;
                    if (out_poly) out_poly[pos] = best;
                }
                ++pos;
                prev = best;
            }
        }
        __syncthreads();
    }
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
    const size_t lds = coarse_bytes_of(cv->view);
    const int per_cu = std::max<int>(1, (int)(LDS_TOTAL / (lds + LDS_RESERVE)));
    const int cus = num_cus(ctx);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, (int64_t)cus * std::min(per_cu, 4)));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_emit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    hipLaunchKernelGGL(k_emit, dim3(grid), dim3(EMIT_THREADS), lds, st, cv->view, n, pts->x, pts->y,
                       out_pt, out_poly, cap, status, ctr, nchunks, total);
    SPADE_HIP(ctx, hipGetLastError());
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, total, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *n_out = (int64_t)h[0];
    if (*n_out > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // namespace spade
