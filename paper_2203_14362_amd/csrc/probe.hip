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
//            the paper's two-step Map (a count pass per wavefront segment of
//            points, a scan of the segment counts, a write pass).
#include "common.h"
#include "exact.h"
#include "lookup.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <mutex>
#include <string>

namespace spade {

constexpr int CNT_THREADS = 1024;         // count probe workgroup
constexpr int CNT_UNROLL = 5;             // points per thread per iteration (6 spills)
constexpr int QCAP = 64;                  // boundary queue entries per wavefront
constexpr int HIST_MAX = 8192;            // polygons counted in LDS
constexpr int EMIT_THREADS = 1024;
constexpr int EMIT_GROUP = 8;             // points per lane in flight (count pass)
constexpr int EMIT_WGROUP = 4;            // points per lane in flight (write pass)
constexpr int EMIT_WDRAIN = 8;            // words of the write pass sharing one boundary queue
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

// Exact test of a point against the records of its boundary pixel, two
// records at a time (most pixels have two; the slot after the last record
// exists and is never used); add(poly) for every polygon containing it.
template <typename Add>
__device__ __forceinline__ void test_records(const CanvasView &cv, uint32_t rec, double x, double y, Add &&add)
{
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

// Counts accumulate in a context-owned accumulator `acc` that is all zero
// between calls: the last workgroup to finish (found with a counter, after a
// device-scope fence) copies acc into the caller's output and clears acc and
// the counter again, so a query needs no memset.  Each wavefront tests its
// queued boundary points itself whenever 64 have gathered.
template <bool LDSHIST, int UNROLL>
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
    // exact tests of the queued points lo .. qn-1
    auto drain = [&](uint32_t lo) {
        __builtin_amdgcn_wave_barrier();
        if (lane >= lo && lane < qn) test_records(cv, qr[lane], qx[lane], qy[lane], add);
        __builtin_amdgcn_wave_barrier();
        qn = 0;
    };

    // software pipeline: the next iteration's points are in flight while the
    // current ones are classified
    const int64_t step = (int64_t)gridDim.x * CNT_THREADS * UNROLL;
    double xn[UNROLL], yn[UNROLL];
    auto fetch = [&](int64_t b) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = b + (int64_t)u * CNT_THREADS + threadIdx.x;
            xn[u] = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            yn[u] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
        }
    };
    int64_t base = (int64_t)blockIdx.x * CNT_THREADS * UNROLL;
    if (base < n) fetch(base);
    for (; base < n; base += step) {
        double xs[UNROLL], ys[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) { xs[u] = xn[u]; ys[u] = yn[u]; }
        if (base + step < n) fetch(base + step);
        // the coarse words of all points of this iteration first, then
        // their full-canvas reads, all issued before any result is used
        Look lk[UNROLL];
        uint32_t ws[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) lk[u] = look_coarse(cv, coarse, xs[u], ys[u]);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            ws[u] = lk[u].full ? ((gu32p)cv.cells)[lk[u].fidx] : lk[u].word;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint32_t w = ws[u];
            const bool bnd = (w & BFLAG) != 0;
            if (w != 0u && !bnd) add(w - 1u);
            const unsigned long long mask = __ballot(bnd);
            const uint32_t nnew = (uint32_t)__popcll(mask);
            if (nnew == 0) continue;
            if (qn + nnew > QCAP) drain(0);
            if (bnd) {
                const uint32_t slot = qn + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                qx[slot] = xs[u];
                qy[slot] = ys[u];
                qr[slot] = w & ~BFLAG;
            }
            qn += nnew;
        }
    }
    if (qn) drain(0);

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

// Launches the count probe with the accumulator acc[M] and the finish
// counter *done, both zero on entry and left zero by the kernel.
static int launch_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint64_t *out_counts,
                        unsigned long long *acc, unsigned int *done)
{
    hipStream_t st = ctx->stream;
    const CanvasView &v = cv->view;
    const int64_t M = v.M;
    const int cus = num_cus(ctx);
    const bool ldshist = M <= HIST_MAX;
    const size_t lds = coarse_bytes_of(v) + (ldshist ? (((size_t)M * 4 + 15) & ~(size_t)15) : 0) + QUEUE_BYTES;
    if (lds + LDS_RESERVE > LDS_TOTAL) return set_error(ctx, SPADE_E_HIP, "internal: probe LDS budget exceeded");
    const int64_t need = std::max<int64_t>(1, (pts->n + CNT_THREADS * CNT_UNROLL - 1) / (CNT_THREADS * CNT_UNROLL));
    // one workgroup per CU even where the LDS would hold two: a second one
    // slows the stream down (measured), so spare LDS goes to a finer coarse
    // level instead
    const int grid = (int)std::min<int64_t>(need, (int64_t)cus);
    unsigned long long *o = (unsigned long long *)out_counts;
    auto go = [&](auto kern) -> int {
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(CNT_THREADS), lds, st, v, pts->n, pts->x, pts->y, acc, done, o);
        SPADE_HIP(ctx, hipGetLastError());
        return SPADE_OK;
    };
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    int rc = ldshist ? go(k_count<true, CNT_UNROLL>) : go(k_count<false, CNT_UNROLL>);
    if (rc) return rc;
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    return SPADE_OK;
}

int probe_count(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint64_t *out_counts)
{
    const int64_t M = cv->view.M;
    if (M == 0) return SPADE_OK;
    unsigned long long *acc = nullptr;
    unsigned int *done = nullptr;
    int rc = count_acc(ctx, M, &acc, &done);
    if (rc) return rc;
    return launch_count(ctx, cv, pts, out_counts, acc, done);
}

// ------------------------------------------------- stream-read reference

// Reads every point's two coordinates once (the probe's algorithmic bytes)
// and sums them, nothing else: the ceiling a point stream can reach.
// Shape 0 is the count probe's (one 1024-thread workgroup per CU, UNROLL
// points per thread in flight); shape 1 uses 256-thread workgroups, eight
// per CU.
template <int THREADS, int UNROLL>
__global__ __launch_bounds__(THREADS) void k_stream(int64_t n, const double *X, const double *Y, double *out)
{
    __shared__ double part[THREADS / 64];
    double acc = 0.0;
    const int64_t step = (int64_t)gridDim.x * THREADS * UNROLL;
    for (int64_t b = (int64_t)blockIdx.x * THREADS * UNROLL; b < n; b += step) {
        double xs[UNROLL], ys[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = b + (int64_t)u * THREADS + threadIdx.x;
            xs[u] = i < n ? __builtin_nontemporal_load(X + i) : 0.0;
            ys[u] = i < n ? __builtin_nontemporal_load(Y + i) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) acc += xs[u] + ys[u];
    }
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < THREADS / 64; ++w) t += part[w];
        atomicAdd(out, t);
    }
}

int stream_read(spade_ctx *ctx, const spade_points *pts, int shape, double *out)
{
    hipStream_t st = ctx->stream;
    const int cus = num_cus(ctx);
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (shape == 0) {
        const int64_t need = std::max<int64_t>(1, (pts->n + 1024 * 8 - 1) / (1024 * 8));
        hipLaunchKernelGGL((k_stream<1024, 8>), dim3((int)std::min<int64_t>(need, cus)), dim3(1024), 0, st, pts->n,
                           pts->x, pts->y, out);
    } else {
        const int64_t need = std::max<int64_t>(1, (pts->n + 256 * 8 - 1) / (256 * 8));
        hipLaunchKernelGGL((k_stream<256, 8>), dim3((int)std::min<int64_t>(need, (int64_t)cus * 8)), dim3(256), 0,
                           st, pts->n, pts->x, pts->y, out);
    }
    SPADE_HIP(ctx, hipGetLastError());
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    return SPADE_OK;
}

// ------------------------------------------------- join-count without allocation
//
// The count probe's only scratch is its accumulator (one u64 per polygon)
// and finish counter.  For callers that cannot allocate device memory they
// live in a fixed array of this source file instead of a context slot.  Its
// device address differs per GPU and is looked up once per device when a
// context is created there; host code passes that address, never the
// array's own name.  Calls that overlap on one GPU share the array and race.
constexpr int64_t NOALLOC_MAX_POLYS = 65536;
static __device__ __align__(256) unsigned long long scratch[NOALLOC_MAX_POLYS + 1];
constexpr int MAX_DEVICES = 64;
static void *g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

int noalloc_init(spade_ctx *ctx)
{
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        return set_error(ctx, SPADE_E_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[ctx->device]) return SPADE_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_error(ctx, SPADE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[ctx->device] = p;
    return SPADE_OK;
}

__global__ void k_fill_u64(int64_t n, unsigned long long *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

int probe_count_noalloc(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint64_t *out_counts)
{
    const int64_t M = cv->view.M;
    if (M > NOALLOC_MAX_POLYS)
        return set_error(ctx, SPADE_E_UNSUPPORTED,
                         "join-count without allocation supports at most 65536 polygons");
    if (M == 0) return SPADE_OK;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[ctx->device];
    }
    if (!base) return set_error(ctx, SPADE_E_HIP, "scratch address of the device was not looked up");
    unsigned long long *acc = (unsigned long long *)base;
    unsigned int *done = (unsigned int *)(acc + M);
    // the array keeps the last call's contents: clear what must start at
    // zero with a kernel (no memset node, so the call can be captured)
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>((M + 256) / 256, 256)), dim3(256), 0,
                       ctx->stream, M + 1, acc);
    SPADE_HIP(ctx, hipGetLastError());
    return launch_count(ctx, cv, pts, out_counts, acc, done);
}

// ------------------------------------------------------------ ordered emit

// Write pass.  Every wavefront owns segments of EMIT_SEG consecutive points
// (grid-stride over segments), EMIT_WGROUP points per lane in flight at a
// time.  The boundary points of a group are queued in LDS and tested a full
// wavefront at a time (as in k_count); each lane then takes the results of
// its own queued points back with a shuffle.  The entries of segment s are
// written in point order (ascending polygon order for a point in several
// polygons) from position offs[s] on; positions at or beyond cap are not
// written.  No barriers after the coarse canvas is loaded.
template <bool MULTI>
__global__ __launch_bounds__(EMIT_THREADS) void k_emit(CanvasView cv, int64_t n, const double *X,
                                                       const double *Y, int64_t nseg,
                                                       const unsigned long long *offs, uint32_t *out_pt,
                                                       uint32_t *out_poly, int64_t cap, const unsigned *multi)
{
    static_assert(EMIT_THREADS == CNT_THREADS, "the queue area is sized for CNT_THREADS");
    // both variants are launched; the one that does not fit the count
    // pass's finding returns at once
    if ((*multi != 0u) != MULTI) return;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *coarse = (uint16_t *)smem;
    const size_t coarse_bytes = ((size_t)cv.Wc * cv.Hc * (cv.cbyte ? 1 : 2) + 15) & ~(size_t)15;
    unsigned char *qbase = smem + coarse_bytes;
    const int wv = threadIdx.x >> 6;
    double *qx = (double *)(qbase) + wv * QCAP;
    double *qy = (double *)(qbase) + (EMIT_THREADS / 64) * QCAP + wv * QCAP;
    uint32_t *qr = (uint32_t *)((double *)(qbase) + 2 * (EMIT_THREADS / 64) * QCAP) + wv * QCAP;
    load_coarse(cv, coarse, EMIT_THREADS);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = ((int64_t)gridDim.x * EMIT_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * EMIT_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        const int64_t i0 = sg * EMIT_SEG + lane;
        unsigned long long pos = offs[sg];
        // EMIT_WDRAIN words share one boundary queue (drained when full and
        // at their end); their points are loaded EMIT_WGROUP words at a time
        for (int g0 = 0; g0 < EMIT_SEG / 64; g0 += EMIT_WDRAIN) {
            // per word: the entry count (the queue slot while its boundary
            // point waits in the queue) and the label or first record
            uint32_t cs[EMIT_WDRAIN], lab[EMIT_WDRAIN];
            uint32_t qn = 0, pend = 0;   // wave-uniform: queue length, words queued
            uint32_t mine = 0;           // words whose point of this lane is queued
            auto drain = [&]() {
                __builtin_amdgcn_wave_barrier();
                uint32_t m = 0, first = 0, rec0 = 0;
                if (lane < (int)qn) {
                    const double x = qx[lane], y = qy[lane];
                    rec0 = qr[lane];
                    uint32_t rec = rec0;
                    while (true) {   // two records at a time (the slot after the last exists)
                        const Cand c0 = cv.cands[rec];
                        const Cand c1 = cv.cands[rec + 1];
                        if (cand_inside(cv, c0, x, y)) { if (m == 0) first = c0.poly; ++m; }
                        if (c0.meta & CAND_LAST) break;
                        if (cand_inside(cv, c1, x, y)) { if (m == 0) first = c1.poly; ++m; }
                        if (c1.meta & CAND_LAST) break;
                        rec += 2;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                const uint32_t rl = m == 1 ? first : (m > 1 ? rec0 : 0u);
#pragma unroll
                for (int k = 0; k < EMIT_WDRAIN; ++k) {
                    if (!(pend & (1u << k))) continue;
                    const int from = (mine & (1u << k)) ? (int)cs[k] : 0;
                    const uint32_t c = (uint32_t)__shfl((int)m, from, 64);
                    const uint32_t l = (uint32_t)__shfl((int)rl, from, 64);
                    if (mine & (1u << k)) { cs[k] = c; lab[k] = l; }
                }
                pend = 0;
                mine = 0;
                qn = 0;
            };
#pragma unroll
            for (int g = 0; g < EMIT_WDRAIN; g += EMIT_WGROUP) {
                // the group's points, then their canvas words, level by level
                double xs[EMIT_WGROUP], ys[EMIT_WGROUP];
#pragma unroll
                for (int k = 0; k < EMIT_WGROUP; ++k) {
                    const int64_t i = i0 + 64 * (g0 + g + k);
                    xs[k] = i < n ? __builtin_nontemporal_load(X + i) : NAN;   // NaN: outside
                    ys[k] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
                }
                uint32_t ws[EMIT_WGROUP];
#pragma unroll
                for (int k = 0; k < EMIT_WGROUP; ++k) {
                    const Look lk = look_coarse(cv, coarse, xs[k], ys[k]);
                    ws[k] = lk.full ? ((gu32p)cv.cells)[lk.fidx] : lk.word;
                }
                // matches of every point: interior words at once, boundary
                // points through the queue
#pragma unroll
                for (int k = 0; k < EMIT_WGROUP; ++k) {
                    const int kk = g + k;
                    const uint32_t w = ws[k];
                    const bool bnd = (w & BFLAG) != 0;
                    cs[kk] = (w != 0u && !bnd) ? 1u : 0u;
                    lab[kk] = (w != 0u && !bnd) ? w - 1u : 0u;
                    const unsigned long long mask = __ballot(bnd);
                    const uint32_t nnew = (uint32_t)__popcll(mask);
                    if (nnew == 0) continue;
                    if (qn + nnew > QCAP) drain();
                    if (bnd) {
                        const uint32_t sl = qn + (uint32_t)__popcll(mask & below);
                        qx[sl] = xs[k];
                        qy[sl] = ys[k];
                        qr[sl] = w & ~BFLAG;
                        cs[kk] = sl;
                        mine |= 1u << kk;
                    }
                    qn += nnew;
                    pend |= 1u << kk;
                }
            }
            if (qn) drain();
#pragma unroll
            for (int k = 0; k < EMIT_WDRAIN; ++k) {
                // inclusive scan of the entry counts across the wavefront
                const uint32_t cnt = cs[k];
                uint32_t inc = cnt;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t t = __shfl_up(inc, d, 64);
                    if (lane >= d) inc += t;
                }
                const uint32_t tot = __shfl(inc, 63, 64);
                if (cnt) {
                    const int64_t i = i0 + 64 * (g0 + k);
                    const uint32_t pt = (uint32_t)i;
                    unsigned long long p = pos + (inc - cnt);
                    if (cnt == 1) {
                        if ((int64_t)p < cap) {
                            out_pt[p] = pt;
                            if (out_poly) out_poly[p] = lab[k];
                        }
                    } else if (MULTI && (int64_t)p < cap) {
                        // several polygons: the smallest L of them (all when
                        // below cap), ascending, kept in out_poly[p, p + L)
                        // by insertion during one pass over the pixel's
                        // records (this lane's own range, read back by this
                        // lane only)
                        const uint32_t L = (int64_t)(p + cnt) <= cap ? cnt : (uint32_t)(cap - (int64_t)p);
                        if (out_poly) {
                            const double x = X[i], y = Y[i];
                            uint32_t rec = lab[k], j = 0;
                            while (true) {
                                const Cand cd = cv.cands[rec];
                                if (cand_inside(cv, cd, x, y)) {
                                    const uint32_t v = cd.poly;
                                    uint32_t at = j;
                                    if (j < L) ++j;
                                    else at = out_poly[p + L - 1] > v ? L - 1 : L;   // L: v is not kept
                                    if (at < L) {
                                        while (at > 0) {
                                            const uint32_t u = out_poly[p + at - 1];
                                            if (u < v) break;
                                            out_poly[p + at] = u;
                                            --at;
                                        }
                                        out_poly[p + at] = v;
                                    }
                                }
                                if (cd.meta & CAND_LAST) break;
                                ++rec;
                            }
                        }
                        for (uint32_t t = 0; t < L; ++t) out_pt[p + t] = pt;
                    }
                }
                pos += tot;
            }
        }
    }
}

// Count pass with the boundary points of a wavefront queued in LDS and
// tested a full wavefront at a time (as in k_count): counts[s] = output
// entries of segment s.  The same records and the same test as k_emit,
// so the counts match what the write pass writes.
__global__ __launch_bounds__(EMIT_THREADS) void k_emit_count(CanvasView cv, int64_t n, const double *X,
                                                             const double *Y, int64_t nseg,
                                                             unsigned long long *counts, unsigned *multi)
{
    static_assert(EMIT_THREADS == CNT_THREADS, "the queue area is sized for CNT_THREADS");
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *coarse = (uint16_t *)smem;
    const size_t coarse_bytes = ((size_t)cv.Wc * cv.Hc * (cv.cbyte ? 1 : 2) + 15) & ~(size_t)15;
    unsigned char *qbase = smem + coarse_bytes;
    const int wv = threadIdx.x >> 6;
    double *qx = (double *)(qbase) + wv * QCAP;
    double *qy = (double *)(qbase) + (EMIT_THREADS / 64) * QCAP + wv * QCAP;
    uint32_t *qr = (uint32_t *)((double *)(qbase) + 2 * (EMIT_THREADS / 64) * QCAP) + wv * QCAP;
    load_coarse(cv, coarse, EMIT_THREADS);
    __syncthreads();
    const uint32_t lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = ((int64_t)gridDim.x * EMIT_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * EMIT_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        const int64_t i0 = sg * EMIT_SEG + lane;
        unsigned long long total = 0;   // wave-uniform
        uint32_t qn = 0;                // wave-uniform queue length
        auto drain = [&]() {
            __builtin_amdgcn_wave_barrier();
            uint32_t m = 0;
            if (lane < qn) {
                const double x = qx[lane], y = qy[lane];
                uint32_t rec = qr[lane];
                while (true) {   // two records at a time (the slot after the last exists)
                    const Cand c0 = cv.cands[rec];
                    const Cand c1 = cv.cands[rec + 1];
                    m += cand_inside(cv, c0, x, y) ? 1u : 0u;
                    if (c0.meta & CAND_LAST) break;
                    m += cand_inside(cv, c1, x, y) ? 1u : 0u;
                    if (c1.meta & CAND_LAST) break;
                    rec += 2;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // a point in several polygons: the write pass takes its
            // several-polygon variant
            if (__ballot(m > 1u) && lane == 0) *multi = 1u;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) m += __shfl_xor(m, d, 64);
            total += m;
            qn = 0;
        };
        for (int g = 0; g < EMIT_SEG / 64; g += EMIT_GROUP) {
            double xs[EMIT_GROUP], ys[EMIT_GROUP];
#pragma unroll
            for (int k = 0; k < EMIT_GROUP; ++k) {
                const int64_t i = i0 + 64 * (g + k);
                xs[k] = i < n ? __builtin_nontemporal_load(X + i) : NAN;   // NaN: outside
                ys[k] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
            }
            uint32_t ws[EMIT_GROUP];
#pragma unroll
            for (int k = 0; k < EMIT_GROUP; ++k) {
                const Look lk = look_coarse(cv, coarse, xs[k], ys[k]);
                ws[k] = lk.full ? ((gu32p)cv.cells)[lk.fidx] : lk.word;
            }
#pragma unroll
            for (int k = 0; k < EMIT_GROUP; ++k) {
                const uint32_t w = ws[k];
                const bool bnd = (w & BFLAG) != 0;
                total += (unsigned long long)__popcll(__ballot(w != 0u && !bnd));
                const unsigned long long mask = __ballot(bnd);
                const uint32_t nnew = (uint32_t)__popcll(mask);
                if (nnew == 0) continue;
                if (qn + nnew > QCAP) drain();
                if (bnd) {
                    const uint32_t slot = qn + (uint32_t)__popcll(mask & below);
                    qx[slot] = xs[k];
                    qy[slot] = ys[k];
                    qr[slot] = w & ~BFLAG;
                }
                qn += nnew;
            }
        }
        if (qn) drain();
        if (lane == 0) counts[sg] = total;
    }
}

// Count pass for a canvas of one polygon (a point matches at most once)
// that also keeps every point's result, so that the write pass reads bits
// instead of the points: bits[sg * (EMIT_SEG / 64) + j] holds the matches of
// points sg * EMIT_SEG + 64 j + lane (bit = lane).  Boundary points are
// queued and tested a wavefront at a time as in k_emit; each lane takes its
// own points' results back with a shuffle.
__global__ __launch_bounds__(EMIT_THREADS) void k_emit_count_bits(CanvasView cv, int64_t n, const double *X,
                                                                  const double *Y, int64_t nseg,
                                                                  unsigned long long *counts,
                                                                  unsigned long long *bits)
{
    static_assert(EMIT_THREADS == CNT_THREADS, "the queue area is sized for CNT_THREADS");
    static_assert(EMIT_SEG / 64 <= 64, "a segment's words are held one per lane");
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *coarse = (uint16_t *)smem;
    const size_t coarse_bytes = ((size_t)cv.Wc * cv.Hc * (cv.cbyte ? 1 : 2) + 15) & ~(size_t)15;
    unsigned char *qbase = smem + coarse_bytes;
    const int wv = threadIdx.x >> 6;
    double *qx = (double *)(qbase) + wv * QCAP;
    double *qy = (double *)(qbase) + (EMIT_THREADS / 64) * QCAP + wv * QCAP;
    uint32_t *qr = (uint32_t *)((double *)(qbase) + 2 * (EMIT_THREADS / 64) * QCAP) + wv * QCAP;
    load_coarse(cv, coarse, EMIT_THREADS);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = ((int64_t)gridDim.x * EMIT_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * EMIT_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        const int64_t i0 = sg * EMIT_SEG + lane;
        unsigned long long total = 0;   // wave-uniform
        unsigned long long segw = 0;    // lane j < EMIT_SEG / 64: the word of points 64 j ..
        // the segment's words share one boundary queue (drained when full
        // and at the segment's end); points are loaded EMIT_WGROUP words at
        // a time
        constexpr int NW = EMIT_SEG / 64;
        uint32_t hit = 0, slot[NW];   // hit: bit k for this lane's point of word k
        uint32_t qn = 0, pend = 0, mine = 0;
        auto drain = [&]() {
            __builtin_amdgcn_wave_barrier();
            uint32_t m = 0;
            if (lane < (int)qn) {
                const double x = qx[lane], y = qy[lane];
                uint32_t rec = qr[lane];
                while (true) {
                    const Cand c0 = cv.cands[rec];
                    if (cand_inside(cv, c0, x, y)) m = 1u;
                    if (c0.meta & CAND_LAST) break;
                    ++rec;
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                if (!(pend & (1u << k))) continue;
                const uint32_t c = (uint32_t)__shfl((int)m, (int)slot[k], 64);
                if ((mine & (1u << k)) && c) hit |= 1u << k;
            }
            pend = 0;
            mine = 0;
            qn = 0;
        };
#pragma unroll
        for (int g = 0; g < NW; g += EMIT_WGROUP) {
            double xs[EMIT_WGROUP], ys[EMIT_WGROUP];
#pragma unroll
            for (int k = 0; k < EMIT_WGROUP; ++k) {
                const int64_t i = i0 + 64 * (g + k);
                xs[k] = i < n ? __builtin_nontemporal_load(X + i) : NAN;   // NaN: outside
                ys[k] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
            }
            uint32_t ws[EMIT_WGROUP];
#pragma unroll
            for (int k = 0; k < EMIT_WGROUP; ++k) {
                const Look lk = look_coarse(cv, coarse, xs[k], ys[k]);
                ws[k] = lk.full ? ((gu32p)cv.cells)[lk.fidx] : lk.word;
            }
#pragma unroll
            for (int k = 0; k < EMIT_WGROUP; ++k) {
                const int kk = g + k;
                const uint32_t w = ws[k];
                const bool bnd = (w & BFLAG) != 0;
                if (w != 0u && !bnd) hit |= 1u << kk;
                slot[kk] = 0;
                const unsigned long long mask = __ballot(bnd);
                const uint32_t nnew = (uint32_t)__popcll(mask);
                if (nnew == 0) continue;
                if (qn + nnew > QCAP) drain();
                if (bnd) {
                    const uint32_t sl = qn + (uint32_t)__popcll(mask & below);
                    qx[sl] = xs[k];
                    qy[sl] = ys[k];
                    qr[sl] = w & ~BFLAG;
                    slot[kk] = sl;
                    mine |= 1u << kk;
                }
                qn += nnew;
                pend |= 1u << kk;
            }
        }
        if (qn) drain();
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const unsigned long long word = __ballot((hit >> k) & 1u);
            total += (unsigned long long)__popcll(word);
            if (lane == k) segw = word;
        }
        if (lane < EMIT_SEG / 64) bits[sg * (EMIT_SEG / 64) + lane] = segw;
        if (lane == 0) counts[sg] = total;
    }
}

// Write pass from the count pass's bits: each wavefront takes segments and
// walks a segment's words in point order; lane l writes point 64 j + l of
// word j, so the ids of a word are stored to consecutive positions (below
// cap; polygon 0 into out_poly), from offs[segment] on.
__global__ __launch_bounds__(256) void k_emit_bits(int64_t nseg, const unsigned long long *offs,
                                                   const unsigned long long *bits, uint32_t *out_pt,
                                                   uint32_t *out_poly, int64_t cap)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        int64_t pos = (int64_t)offs[sg];
        const unsigned long long mine = lane < EMIT_SEG / 64 ? bits[sg * (EMIT_SEG / 64) + lane] : 0ull;
        for (int j = 0; j < EMIT_SEG / 64; ++j) {
            const unsigned long long word = (unsigned long long)__shfl((long long)mine, j, 64);
            if (!word) continue;   // uniform over the wavefront
            if ((word >> lane) & 1ull) {
                const int64_t p = pos + __popcll(word & below);
                if (p < cap) {
                    out_pt[p] = (uint32_t)(sg * EMIT_SEG + 64 * j + lane);
                    if (out_poly) out_poly[p] = 0u;
                }
            }
            pos += __popcll(word);
        }
    }
}

__global__ void k_emit_zero(unsigned long long *p) { *p = 0ull; }
__global__ void k_emit_flag0(unsigned *p) { *p = 0u; }

int probe_emit(spade_ctx *ctx, const spade_canvas *cv, const spade_points *pts, uint32_t *out_pt,
               uint32_t *out_poly, int64_t cap, int64_t *n_out)
{
    hipStream_t st = ctx->stream;
    const int64_t n = pts->n;
    *n_out = 0;
    if (n == 0 || cv->view.M == 0) return SPADE_OK;
    const int64_t nseg = (n + EMIT_SEG - 1) / EMIT_SEG;
    DevBuf &lb = ctx->scratch[S_LOOKBACK];
    if (ensure(ctx, lb, sizeof(unsigned long long) * (2 * (size_t)(nseg + 1) + 1))) return SPADE_E_NOMEM;
    unsigned long long *counts = (unsigned long long *)lb.p;
    unsigned long long *offs = counts + (nseg + 1);
    unsigned *multi = (unsigned *)(offs + (nseg + 1));   // set by the count pass: a point in several polygons
    const size_t lds = coarse_bytes_of(cv->view);
    if (lds + QUEUE_BYTES + LDS_RESERVE > LDS_TOTAL)
        return set_error(ctx, SPADE_E_HIP, "internal: emit probe LDS budget exceeded");
    const int per_cu = std::max<int>(1, (int)(LDS_TOTAL / (lds + LDS_RESERVE)));
    const int cus = num_cus(ctx);
    const int64_t wpb = EMIT_THREADS / 64;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + wpb - 1) / wpb, (int64_t)cus * std::min(per_cu, 2)));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_emit_count, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(lds + QUEUE_BYTES)));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_emit<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(lds + QUEUE_BYTES)));
    SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_emit<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(lds + QUEUE_BYTES)));
    // a canvas of one polygon keeps every point's result in the count pass
    // (one bit per point), so that the write pass need not read the points
    unsigned long long *bits = nullptr;
    if (cv->view.M == 1 && cap > 0) {
        DevBuf &bb = ctx->scratch[S_BITS];
        if (ensure(ctx, bb, sizeof(unsigned long long) * (EMIT_SEG / 64) * (size_t)nseg) == SPADE_OK)
            bits = (unsigned long long *)bb.p;
        else
            ctx->err.clear();   // read the points twice instead
    }
    if (bits)
        SPADE_HIP(ctx, hipFuncSetAttribute((const void *)k_emit_count_bits, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(lds + QUEUE_BYTES)));
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (bits)
        hipLaunchKernelGGL(k_emit_count_bits, dim3(grid), dim3(EMIT_THREADS), lds + QUEUE_BYTES, st, cv->view, n,
                           pts->x, pts->y, nseg, counts, bits);
    else {
        hipLaunchKernelGGL(k_emit_flag0, dim3(1), dim3(1), 0, st, multi);
        hipLaunchKernelGGL(k_emit_count, dim3(grid), dim3(EMIT_THREADS), lds + QUEUE_BYTES, st, cv->view, n, pts->x,
                           pts->y, nseg, counts, multi);
    }
    hipLaunchKernelGGL(k_emit_zero, dim3(1), dim3(1), 0, st, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, counts, offs, (int)(nseg + 1), st));
    if (cap > 0 && bits) {
        const int bg = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + 3) / 4, (int64_t)cus * 16));
        hipLaunchKernelGGL(k_emit_bits, dim3(bg), dim3(256), 0, st, nseg, offs, bits, out_pt, out_poly, cap);
        SPADE_HIP(ctx, hipGetLastError());
    } else if (cap > 0) {
        hipLaunchKernelGGL(k_emit<false>, dim3(grid), dim3(EMIT_THREADS), lds + QUEUE_BYTES, st, cv->view, n, pts->x,
                           pts->y, nseg, offs, out_pt, out_poly, cap, (const unsigned *)multi);
        hipLaunchKernelGGL(k_emit<true>, dim3(grid), dim3(EMIT_THREADS), lds + QUEUE_BYTES, st, cv->view, n, pts->x,
                           pts->y, nseg, offs, out_pt, out_poly, cap, (const unsigned *)multi);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *n_out = (int64_t)h[0];
    if (*n_out > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

}  // namespace spade
