// Distance selection from a point (Sec. 4.2, canvases for distance-based
// queries; Sec. 5.2, distance-based selections): the ids of the points whose
// distance to a centre is at most r, in ascending order.
//
// The paper draws the disk into a canvas and tests the points against it.
// A single disk needs no canvas here: its exact closed-disk predicate
// (disk.h) is evaluated per point while the points stream from HBM.
//
// Output follows the paper's two-step Map (Sec. 5.1): a count pass writes
// the number of selected points of every wavefront segment of DISK_SEG
// points and keeps one result bit per point, an exclusive scan gives each
// segment its start, and the write pass (k_emit_bits, shared with the
// selection probe) writes the ids in order from the bits, so the points are
// read once.
#include "common.h"
#include "disk.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

namespace spade {

constexpr int DISK_THREADS = 256;
constexpr int DISK_ROUNDS = 16;   // 64-point rounds per wavefront segment
constexpr int64_t DISK_SEG = 64 * DISK_ROUNDS;

// Every wavefront owns segments of DISK_SEG consecutive points (grid-stride
// over segments): counts[s] = selected points of segment s, and word k of
// segment s in bits holds the results of points s * DISK_SEG + 64 k + lane
// (the layout k_emit_bits reads).  No barriers: a wavefront counts its
// points by ballot.
static_assert(DISK_SEG == EMIT_SEG, "the write pass reads the count pass's bits per EMIT_SEG points");
__global__ __launch_bounds__(DISK_THREADS) void k_disk(int64_t n, const double *X, const double *Y, double cx,
                                                       double cy, double r, double r2, int64_t nseg,
                                                       unsigned long long *counts, unsigned long long *bits)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * DISK_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * DISK_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        const int64_t i0 = sg * DISK_SEG + lane;
        // all loads of the segment in flight before the first test
        double xs[DISK_ROUNDS], ys[DISK_ROUNDS];
#pragma unroll
        for (int k = 0; k < DISK_ROUNDS; ++k) {
            const int64_t i = i0 + 64 * k;
            xs[k] = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            ys[k] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
        }
        unsigned long long pos = 0ull, segw = 0ull;
#pragma unroll
        for (int k = 0; k < DISK_ROUNDS; ++k) {
            const bool in = in_disk(xs[k], ys[k], cx, cy, r, r2);   // NaN padding is outside
            const unsigned long long m = __ballot(in);
            if (lane == k) segw = m;
            pos += (unsigned long long)__popcll(m);
        }
        if (lane < DISK_ROUNDS) bits[sg * DISK_ROUNDS + lane] = segw;
        if (lane == 0) counts[sg] = pos;
    }
}

__global__ void k_disk_zero(unsigned long long *p) { *p = 0ull; }


int select_disk(spade_ctx *ctx, const spade_points *pts, double cx, double cy, double r, uint32_t *out_ids,
                int64_t cap, int64_t *n_out)
{
    hipStream_t st = ctx->stream;
    if (!(std::isfinite(cx) && std::isfinite(cy) && std::isfinite(r) && r >= 0.0))
        return set_error(ctx, SPADE_E_INVALID, "disk centre and radius must be finite and the radius >= 0");
    if (cap < 0) return set_error(ctx, SPADE_E_INVALID, "negative capacity");
    if (cap > 0 && !out_ids) return set_error(ctx, SPADE_E_INVALID, "out_ids is NULL");
    const int64_t n = pts->n;
    if (n == 0) {
        if (n_out) *n_out = 0;
        return SPADE_OK;
    }
    const int64_t nseg = (n + DISK_SEG - 1) / DISK_SEG;
    DevBuf &cb = ctx->scratch[S_LOOKBACK], &bb = ctx->scratch[S_BITS];
    if (ensure(ctx, cb, sizeof(unsigned long long) * 2 * (size_t)(nseg + 1)) ||
        ensure(ctx, bb, sizeof(unsigned long long) * DISK_ROUNDS * (size_t)nseg))
        return SPADE_E_NOMEM;
    unsigned long long *counts = (unsigned long long *)cb.p;
    unsigned long long *offs = counts + (nseg + 1);
    unsigned long long *bits = (unsigned long long *)bb.p;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        cus = 256;
    const int grid = (int)std::min<int64_t>((nseg + DISK_THREADS / 64 - 1) / (DISK_THREADS / 64), (int64_t)cus * 8);
    const double r2 = r * r;
    hipLaunchKernelGGL(k_disk, dim3(grid), dim3(DISK_THREADS), 0, st, n, pts->x, pts->y, cx, cy, r, r2, nseg, counts,
                       bits);
    hipLaunchKernelGGL(k_disk_zero, dim3(1), dim3(1), 0, st, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, counts, offs, (int)(nseg + 1), st));
    // the write pass also runs when the buffer is too small: the first cap
    // ids are written (two-step Map), the call then reports the shortfall
    if (cap > 0) {
        const int eg = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + 3) / 4, (int64_t)cus * 16));
        hipLaunchKernelGGL(k_emit_bits, dim3(eg), dim3(256), 0, st, nseg, (const unsigned long long *)offs,
                           (const unsigned long long *)bits, out_ids, (uint32_t *)nullptr, cap);
        SPADE_HIP(ctx, hipGetLastError());
    }
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const int64_t total = (int64_t)h[0];
    if (n_out) *n_out = total;
    if (total > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small for the selection");
    return SPADE_OK;
}

}  // namespace spade
