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
// points, an exclusive scan gives each segment its start, and a write pass
// recomputes the predicate and writes the ids in order (ballot ranks within
// the wavefront).  Both passes evaluate the same function on the same
// inputs, so the write pass fills exactly the counted slots.
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
// over segments).  WRITE == false: counts[s] = selected points of segment s.
// WRITE == true: the ids of segment s's selected points, ascending, from
// out[offs[s]] on; positions at or beyond cap are not written.  No barriers:
// a wavefront ranks its points by ballot.
template <bool WRITE>
__global__ __launch_bounds__(DISK_THREADS) void k_disk(int64_t n, const double *X, const double *Y, double cx,
                                                       double cy, double r, double r2, int64_t nseg,
                                                       uint32_t *counts, const uint32_t *offs, uint32_t *out,
                                                       int64_t cap)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
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
        uint32_t pos = WRITE ? offs[sg] : 0u;
#pragma unroll
        for (int k = 0; k < DISK_ROUNDS; ++k) {
            const bool in = in_disk(xs[k], ys[k], cx, cy, r, r2);   // NaN padding is outside
            const unsigned long long m = __ballot(in);
            if (WRITE && in) {
                const uint32_t at = pos + (uint32_t)__popcll(m & below);
                if ((int64_t)at < cap) out[at] = (uint32_t)(i0 + 64 * k);
            }
            pos += (uint32_t)__popcll(m);
        }
        if (!WRITE && lane == 0) counts[sg] = pos;
    }
}

__global__ void k_disk_zero(uint32_t *p) { *p = 0u; }

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
    DevBuf &cb = ctx->scratch[S_LOOKBACK];
    if (ensure(ctx, cb, sizeof(uint32_t) * 2 * (size_t)(nseg + 1))) return SPADE_E_NOMEM;
    uint32_t *counts = (uint32_t *)cb.p;
    uint32_t *offs = counts + (nseg + 1);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        cus = 256;
    const int grid = (int)std::min<int64_t>((nseg + DISK_THREADS / 64 - 1) / (DISK_THREADS / 64), (int64_t)cus * 8);
    const double r2 = r * r;
    hipLaunchKernelGGL(k_disk<false>, dim3(grid), dim3(DISK_THREADS), 0, st, n, pts->x, pts->y, cx, cy, r, r2,
                       nseg, counts, nullptr, nullptr, (int64_t)0);
    hipLaunchKernelGGL(k_disk_zero, dim3(1), dim3(1), 0, st, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, counts, offs, (int)(nseg + 1), st));
    uint32_t *h = (uint32_t *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const int64_t total = (int64_t)h[0];
    if (n_out) *n_out = total;
    // the write pass also runs when the buffer is too small: the first cap
    // ids are written (two-step Map), the call then reports the shortfall
    if (total > 0 && cap > 0) {
        hipLaunchKernelGGL(k_disk<true>, dim3(grid), dim3(DISK_THREADS), 0, st, n, pts->x, pts->y, cx, cy, r, r2,
                           nseg, nullptr, offs, out_ids, cap);
        SPADE_HIP(ctx, hipGetLastError());
        SPADE_HIP(ctx, hipStreamSynchronize(st));
    }
    if (total > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small for the selection");
    return SPADE_OK;
}

}  // namespace spade
