// Distance joins between a point set and a set of disks (Sec. 4.2,
// canvases for distance-based queries; Sec. 5.2, distance-based joins):
//   type (1): all pairs (point i, disk j) with |p_i - c_j| <= r (one radius);
//   type (2): the same with a radius r_j per disk.
// Counts per disk (the aggregation over the join) come from the same probe.
//
// The disks play the paper's constraint canvases: a grid of cells over the
// disks' union box whose cells list the disks that can reach them (the
// boundary index of the disk set, ascending disk ids).  Each point reads its
// cell's list and every listed disk gets the exact closed-disk predicate, so
// results are exact and independent of the grid.  Pairs come out ascending
// by (point id, disk id) from the paper's two-step Map (count pass per
// wavefront segment, scan, write pass), with no sort.  The disk tests of a
// wavefront's points are spread over its lanes (wave_round), so that a
// wavefront's rounds follow its candidates in total rather than its longest
// list.
#include "common.h"
#include "disk.h"
#include "wavewalk.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace spade {

constexpr int DJ_THREADS = 256;
constexpr int DJ_ROUNDS = 8;                  // 64-point rounds per wavefront segment
constexpr int64_t DJ_SEG = 64 * DJ_ROUNDS;
constexpr int DJ_GRID_MAX = 4096;             // cells per grid side
constexpr int DJ_HIST_MAX = 8192;             // disks counted in LDS

struct DiskGrid {
    double X0, Y0, sx, sy;   // cell (floor((x - X0) * sx), floor((y - Y0) * sy))
    double bx0, by0, bx1, by1;   // closed box of all disks
    int W, H;
};

struct DiskArgs {
    const double *cx, *cy, *r;   // r: per-disk radii or NULL
    double r_all;
};

__device__ __forceinline__ double radius_of(const DiskArgs &D, int64_t j)
{
    return D.r ? D.r[j] : D.r_all;
}

// Validation and union box: flags bit 0 = a non-finite centre or radius or a
// negative radius; box as order keys (min x, -max x, min y, -max y) of the
// disks' extents, and the sum of radii.
__device__ __forceinline__ unsigned long long okey_d(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_disks_box(int64_t n, DiskArgs D, unsigned long long *bb, unsigned *bad,
                                                   double *rsum)
{
    __shared__ unsigned long long s[4][256];
    __shared__ double sr[256];
    unsigned long long k0 = ~0ull, k1 = ~0ull, k2 = ~0ull, k3 = ~0ull;
    double rs = 0.0;
    unsigned nb = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double cx = D.cx[j], cy = D.cy[j], r = radius_of(D, j);
        if (!(isfinite(cx) && isfinite(cy) && isfinite(r) && r >= 0.0)) { nb = 1; continue; }
        k0 = min(k0, okey_d(cx - r)); k1 = min(k1, okey_d(-(cx + r)));
        k2 = min(k2, okey_d(cy - r)); k3 = min(k3, okey_d(-(cy + r)));
        rs += r;
    }
    if (nb) atomicOr(bad, 1u);
    s[0][threadIdx.x] = k0; s[1][threadIdx.x] = k1; s[2][threadIdx.x] = k2; s[3][threadIdx.x] = k3;
    sr[threadIdx.x] = rs;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = min(s[q][threadIdx.x], s[q][threadIdx.x + w]);
            sr[threadIdx.x] += sr[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) atomicMin(&bb[threadIdx.x], s[threadIdx.x][0]);
    if (threadIdx.x == 0) atomicAdd(rsum, sr[0]);
}

// Cells a disk can reach: its box widened by one cell (so that rounding in a
// point's cell index never loses a candidate), without the cells whose
// (slightly enlarged) square lies entirely outside the disk.
__device__ __forceinline__ void disk_cells(const DiskGrid &g, double cx, double cy, double r, int &c0, int &c1,
                                           int &r0, int &r1)
{
    c0 = (int)fmax(0.0, floor((cx - r - g.X0) * g.sx) - 1.0);
    c1 = (int)fmin((double)(g.W - 1), floor((cx + r - g.X0) * g.sx) + 1.0);
    r0 = (int)fmax(0.0, floor((cy - r - g.Y0) * g.sy) - 1.0);
    r1 = (int)fmin((double)(g.H - 1), floor((cy + r - g.Y0) * g.sy) + 1.0);
}

__device__ __forceinline__ bool cell_reached(const DiskGrid &g, double cx, double cy, double r, int c, int rr)
{
    // the cell's square enlarged by a quarter cell on every side
    const double x0 = g.X0 + ((double)c - 0.25) / g.sx, x1 = g.X0 + ((double)c + 1.25) / g.sx;
    const double y0 = g.Y0 + ((double)rr - 0.25) / g.sy, y1 = g.Y0 + ((double)rr + 1.25) / g.sy;
    const double dx = fmax(fmax(x0 - cx, cx - x1), 0.0), dy = fmax(fmax(y0 - cy, cy - y1), 0.0);
    return dx * dx + dy * dy <= r * r * 1.0000001;
}

// COUNT: cells per disk.  Otherwise keys (cell << 32 | disk) from off[j].
template <bool FILL>
__global__ __launch_bounds__(256) void k_disk_cells(int64_t n, DiskArgs D, DiskGrid g, unsigned long long *count,
                                                    const unsigned long long *off, unsigned long long *keys)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double cx = D.cx[j], cy = D.cy[j], r = radius_of(D, j);
        int c0, c1, r0, r1;
        disk_cells(g, cx, cy, r, c0, c1, r0, r1);
        unsigned long long m = 0, at = FILL ? off[j] : 0ull;
        for (int rr = r0; rr <= r1; ++rr)
            for (int c = c0; c <= c1; ++c) {
                if (!cell_reached(g, cx, cy, r, c, rr)) continue;
                if (FILL) keys[at++] = ((unsigned long long)((int64_t)rr * g.W + c) << 32) | (unsigned long long)j;
                else ++m;
            }
        if (!FILL) count[j] = m;
    }
}

// cell_off[c] = first sorted key of cell c (c = 0 .. ncell).
__global__ void k_dcell_off(int64_t nk, const unsigned long long *skeys, int64_t ncell, uint32_t *cell_off,
                            uint32_t *cell_disk)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nk; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ki = i < nk ? (int64_t)(skeys[i] >> 32) : ncell;
        const int64_t kp = i == 0 ? -1 : (int64_t)(skeys[i - 1] >> 32);
        for (int64_t c = kp + 1; c <= ki; ++c) cell_off[c] = (uint32_t)i;
        if (i < nk) cell_disk[i] = (uint32_t)skeys[i];
    }
}

struct DiskCanvas {
    DiskGrid g;
    const uint32_t *cell_off, *cell_disk;
    DiskArgs D;
};

// The candidates of point (x, y): its cell's disks cell_disk[k, k + rem)
// (none outside the disks' box; NaN fails the test too).
__device__ __forceinline__ void disk_range(const DiskCanvas &K, double x, double y, uint32_t &k, uint32_t &rem)
{
    k = 0u;
    rem = 0u;
    if (!(K.g.bx0 <= x && x <= K.g.bx1 && K.g.by0 <= y && y <= K.g.by1)) return;
    const int c = min((int)((x - K.g.X0) * K.g.sx), K.g.W - 1);
    const int r = min((int)((y - K.g.Y0) * K.g.sy), K.g.H - 1);
    const int64_t cell = (int64_t)max(r, 0) * K.g.W + max(c, 0);
    k = K.cell_off[cell];
    rem = K.cell_off[cell + 1] - k;
}

// The (point, disk) pairs of a wavefront's points with the disk tests
// balanced over the lanes: for each pair the testing lane calls pair(o,
// slot, j) with o the point's lane and slot = base of lane o + the pair's
// rank among the point's pairs (ascending disk id, the order of the cell
// lists); on return cnt holds the number of pairs of this lane's point.
// Called by every lane of the wavefront.
template <typename Pair>
__device__ __forceinline__ void disk_wave_walk(const DiskCanvas &K, double x, double y, uint32_t k, uint32_t rem,
                                               uint32_t base, int lane, uint32_t &cnt, Pair &&pair)
{
    cnt = 0u;
    while (__ballot(rem != 0u)) {
        const WaveRound w = wave_round(rem, lane);
        const uint32_t ok = __shfl(k, w.o, 64);
        const uint32_t ocnt = __shfl(cnt, w.o, 64);
        const uint32_t obase = __shfl(base, w.o, 64);
        const double ox = __shfl(x, w.o, 64), oy = __shfl(y, w.o, 64);
        bool h = false;
        uint32_t j = 0u;
        if ((uint32_t)lane < w.ntake) {
            j = K.cell_disk[ok + ((uint32_t)lane - w.opre)];
            const double rj = radius_of(K.D, j);
            h = in_disk(ox, oy, K.D.cx[j], K.D.cy[j], rj, rj * rj);
        }
        const unsigned long long hm = __ballot(h);
        if (h) pair(w.o, obase + ocnt + (uint32_t)__popcll(hm & wave_round_before(w, lane)), j);
        cnt += (uint32_t)__popcll(hm & wave_round_mask(w));
        const uint32_t len = wave_round_len(w);
        k += len;
        rem -= len;
    }
}

// MODE 0: counts per wavefront segment (and, with pcount, the pairs of every
// point, so that the write pass walks each point's candidates once); 1: pairs
// written from offs[s] on (positions at or beyond cap are not written); 2:
// per-disk counts.
template <int MODE>
__global__ __launch_bounds__(DJ_THREADS) void k_djoin(DiskCanvas K, int64_t n, const double *X, const double *Y,
                                                      int64_t nseg, unsigned long long *counts,
                                                      const unsigned long long *offs, uint32_t *out_pt,
                                                      uint32_t *out_disk, int64_t cap, int64_t ndisk,
                                                      unsigned long long *dcount, uint32_t *pcount)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *hist = (uint32_t *)smem;
    const bool ldsh = MODE == 2 && ndisk <= DJ_HIST_MAX;
    if (MODE == 2) {
        if (ldsh)
            for (int64_t k = threadIdx.x; k < ndisk; k += DJ_THREADS) hist[k] = 0;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * DJ_THREADS) >> 6;
    for (int64_t sg = ((int64_t)blockIdx.x * DJ_THREADS + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
        const int64_t i0 = sg * DJ_SEG + lane;
        double xs[DJ_ROUNDS], ys[DJ_ROUNDS];
#pragma unroll
        for (int k = 0; k < DJ_ROUNDS; ++k) {
            const int64_t i = i0 + 64 * k;
            xs[k] = i < n ? __builtin_nontemporal_load(X + i) : NAN;
            ys[k] = i < n ? __builtin_nontemporal_load(Y + i) : NAN;
        }
        unsigned long long pos = MODE == 1 ? offs[sg] : 0ull;
        for (int k = 0; k < DJ_ROUNDS; ++k) {
            uint32_t c0, rem, m;
            disk_range(K, xs[k], ys[k], c0, rem);
            if (MODE == 2) {
                disk_wave_walk(K, xs[k], ys[k], c0, rem, 0u, lane, m, [&](int, uint32_t, uint32_t j) {
                    if (ldsh) atomicAdd(&hist[j], 1u);
                    else atomicAdd(&dcount[j], 1ull);
                });
                continue;
            }
            const int64_t ip = i0 + 64 * k;
            if (MODE == 1 && pcount) {
                m = ip < n ? pcount[ip] : 0u;   // the count pass's pairs of this point
            } else {
                disk_wave_walk(K, xs[k], ys[k], c0, rem, 0u, lane, m, [](int, uint32_t, uint32_t) {});
                if (MODE == 0 && pcount && ip < n) pcount[ip] = m;
            }
            uint32_t inc = m;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = __shfl_up(inc, d, 64);
                if (lane >= d) inc += t;
            }
            const uint32_t tot = __shfl(inc, 63, 64);
            if (MODE == 1 && tot) {
                // again, writing each pair at pos + (pairs of earlier lanes) + rank
                const int64_t w0 = sg * DJ_SEG + 64 * k;
                uint32_t m2;
                disk_wave_walk(K, xs[k], ys[k], c0, m ? rem : 0u, inc - m, lane, m2,
                               [&](int o, uint32_t slot, uint32_t j) {
                                   const unsigned long long p = pos + slot;
                                   if ((int64_t)p < cap) {
                                       out_pt[p] = (uint32_t)(w0 + o);
                                       out_disk[p] = j;
                                   }
                               });
            }
            pos += tot;
        }
        if (MODE == 0 && lane == 0) counts[sg] = pos;
    }
    if (MODE == 2 && ldsh) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k < ndisk; k += DJ_THREADS)
            if (hist[k]) atomicAdd(&dcount[k], (unsigned long long)hist[k]);
    }
}

__global__ void k_dj_zero(int64_t n, unsigned long long *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

static int dj_grid(int64_t n, int64_t cap = 65536)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

static int dj_bits(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// Builds the disk canvas in ctx scratch (cell lists valid until the next
// call on ctx).
static int build_disk_canvas(spade_ctx *ctx, const spade_disks *dk, DiskCanvas &K)
{
    hipStream_t st = ctx->stream;
    const int64_t n = dk->n;
    K.D.cx = dk->cx;
    K.D.cy = dk->cy;
    K.D.r = dk->r;
    K.D.r_all = dk->r_all;
    DevBuf &bb = ctx->scratch[S_BLOCKRED];
    if (ensure(ctx, bb, 128)) return SPADE_E_NOMEM;
    unsigned long long *dbb = (unsigned long long *)bb.p;
    unsigned *bad = (unsigned *)(dbb + 4);
    double *rsum = (double *)(dbb + 6);
    // box keys start at all-ones, the flag and the radius sum at zero
    hipLaunchKernelGGL(k_dj_zero, dim3(1), dim3(64), 0, st, (int64_t)8, dbb);
    SPADE_HIP(ctx, hipGetLastError());
    SPADE_HIP(ctx, hipMemsetAsync(dbb, 0xff, 32, st));
    hipLaunchKernelGGL(k_disks_box, dim3(dj_grid(n, 1024)), dim3(256), 0, st, n, K.D, dbb, bad, rsum);
    SPADE_HIP(ctx, hipGetLastError());
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 128);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, dbb, 64, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    if (((unsigned *)(h + 4))[0]) return set_error(ctx, SPADE_E_INVALID, "disk centres and radii must be finite, radii >= 0");
    auto from_key = [](unsigned long long k) {
        const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
        double d;
        std::memcpy(&d, &b, sizeof d);
        return d;
    };
    double mr;
    std::memcpy(&mr, h + 6, sizeof mr);
    mr /= (double)n;
    DiskGrid &g = K.g;
    g.bx0 = from_key(h[0]);
    g.bx1 = -from_key(h[1]);
    g.by0 = from_key(h[2]);
    g.by1 = -from_key(h[3]);
    // cells about the mean radius on a side (at most DJ_GRID_MAX per side,
    // at least one), so a disk reaches a few cells
    const double w = g.bx1 - g.bx0, hgt = g.by1 - g.by0;
    const double cell = std::max(mr, std::max(w, hgt) / DJ_GRID_MAX);
    g.W = (w > 0 && cell > 0) ? (int)std::min<double>(DJ_GRID_MAX, std::max(1.0, std::ceil(w / cell))) : 1;
    g.H = (hgt > 0 && cell > 0) ? (int)std::min<double>(DJ_GRID_MAX, std::max(1.0, std::ceil(hgt / cell))) : 1;
    g.X0 = g.bx0;
    g.Y0 = g.by0;
    g.sx = w > 0 ? g.W / w : 0.0;
    g.sy = hgt > 0 ? g.H / hgt : 0.0;
    const int64_t ncell = (int64_t)g.W * g.H;
    // (cell, disk) keys: count, scan, fill, sort
    DevBuf &bc = ctx->scratch[S_NROWS], &bo = ctx->scratch[S_ROWOFF];
    if (ensure(ctx, bc, 8 * (size_t)(n + 1)) || ensure(ctx, bo, 8 * (size_t)(n + 1))) return SPADE_E_NOMEM;
    unsigned long long *cnt = (unsigned long long *)bc.p, *off = (unsigned long long *)bo.p;
    hipLaunchKernelGGL(k_disk_cells<false>, dim3(dj_grid(n)), dim3(256), 0, st, n, K.D, g, cnt, nullptr, nullptr);
    hipLaunchKernelGGL(k_dj_zero, dim3(1), dim3(64), 0, st, (int64_t)1, cnt + n);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)(n + 1), st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, cnt, off, (int)(n + 1), st));
    SPADE_HIP(ctx, hipMemcpyAsync(h, off + n, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    const int64_t nk = (int64_t)h[0];
    if (nk >= (int64_t)0xffffffffLL) return set_error(ctx, SPADE_E_UNSUPPORTED, "too many (cell, disk) entries");
    DevBuf &bk = ctx->scratch[S_KEYS], &bk2 = ctx->scratch[S_KEYS2], &bl = ctx->scratch[S_VALS];
    if (ensure(ctx, bk, 8 * (size_t)std::max<int64_t>(nk, 1)) || ensure(ctx, bk2, 8 * (size_t)std::max<int64_t>(nk, 1)) ||
        ensure(ctx, bl, 4 * (size_t)(ncell + 1) + 4 * (size_t)std::max<int64_t>(nk, 1) + 64))
        return SPADE_E_NOMEM;
    uint32_t *cell_off = (uint32_t *)bl.p;
    uint32_t *cell_disk = cell_off + (ncell + 1);
    if (nk > 0) {
        hipLaunchKernelGGL(k_disk_cells<true>, dim3(dj_grid(n)), dim3(256), 0, st, n, K.D, g, nullptr, off,
                           (unsigned long long *)bk.p);
        SPADE_HIP(ctx, hipGetLastError());
        const int kb = 32 + std::max(1, dj_bits((uint64_t)ncell));
        tb = 0;
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(nullptr, tb, (const unsigned long long *)bk.p,
                                                         (unsigned long long *)bk2.p, (int)nk, 0, kb, st));
        if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
        SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(cub.p, tb, (const unsigned long long *)bk.p,
                                                         (unsigned long long *)bk2.p, (int)nk, 0, kb, st));
    }
    hipLaunchKernelGGL(k_dcell_off, dim3(dj_grid(nk + 1)), dim3(256), 0, st, nk, (const unsigned long long *)bk2.p,
                       ncell, cell_off, cell_disk);
    SPADE_HIP(ctx, hipGetLastError());
    K.cell_off = cell_off;
    K.cell_disk = cell_disk;
    return SPADE_OK;
}

static int check_disks(spade_ctx *ctx, const spade_disks *dk)
{
    if (!dk) return set_error(ctx, SPADE_E_INVALID, "disks is NULL");
    if (dk->n < 0) return set_error(ctx, SPADE_E_INVALID, "negative disk count");
    if (dk->n >= (int64_t)0x7fffffffLL) return set_error(ctx, SPADE_E_TOO_LARGE, "disk ids must be < 2^31 - 1");
    if (dk->n > 0 && (!dk->cx || !dk->cy)) return set_error(ctx, SPADE_E_INVALID, "disk centre array is NULL");
    if (!dk->r && !(std::isfinite(dk->r_all) && dk->r_all >= 0.0))
        return set_error(ctx, SPADE_E_INVALID, "r_all must be finite and >= 0");
    return SPADE_OK;
}

static int num_cus_dj(int device)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0) v = 256;
    return v;
}

int distance_join(spade_ctx *ctx, const spade_points *pts, const spade_disks *dk, uint32_t *out_pt,
                  uint32_t *out_disk, int64_t cap, int64_t *n_out, uint64_t *out_counts)
{
    int rc = check_disks(ctx, dk);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    if (n_out) *n_out = 0;
    const int64_t n = pts->n, m = dk->n;
    const bool counting = out_counts != nullptr;
    if (counting && m > 0) {
        hipLaunchKernelGGL(k_dj_zero, dim3(dj_grid(m, 4096)), dim3(256), 0, st, m, (unsigned long long *)out_counts);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (n == 0 || m == 0) {
        if (counting) SPADE_HIP(ctx, hipStreamSynchronize(st));
        return SPADE_OK;
    }
    DiskCanvas K;
    if ((rc = build_disk_canvas(ctx, dk, K))) return rc;
    const int64_t nseg = (n + DJ_SEG - 1) / DJ_SEG;
    const int cus = num_cus_dj(ctx->device);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nseg + DJ_THREADS / 64 - 1) / (DJ_THREADS / 64),
                                                                 (int64_t)cus * 8));
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    if (counting) {
        const size_t lds = m <= DJ_HIST_MAX ? 4 * (size_t)m : 16;
        hipLaunchKernelGGL(k_djoin<2>, dim3(grid), dim3(DJ_THREADS), lds, st, K, n, pts->x, pts->y, nseg, nullptr,
                           nullptr, nullptr, nullptr, (int64_t)0, m, (unsigned long long *)out_counts,
                           (uint32_t *)nullptr);
        SPADE_HIP(ctx, hipGetLastError());
        if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        return SPADE_OK;
    }
    DevBuf &lb = ctx->scratch[S_LOOKBACK];
    if (ensure(ctx, lb, sizeof(unsigned long long) * 2 * (size_t)(nseg + 1))) return SPADE_E_NOMEM;
    unsigned long long *counts = (unsigned long long *)lb.p, *offs = counts + (nseg + 1);
    // pairs per point, kept by the count pass for the write pass (without the
    // room, the write pass counts again)
    DevBuf &pb = ctx->scratch[S_BITS];
    uint32_t *pcount = nullptr;
    if (cap > 0) {
        if (ensure(ctx, pb, sizeof(uint32_t) * (size_t)n) == SPADE_OK) pcount = (uint32_t *)pb.p;
        else ctx->err.clear();
    }
    hipLaunchKernelGGL(k_djoin<0>, dim3(grid), dim3(DJ_THREADS), 0, st, K, n, pts->x, pts->y, nseg, counts, nullptr,
                       nullptr, nullptr, (int64_t)0, m, nullptr, pcount);
    hipLaunchKernelGGL(k_dj_zero, dim3(1), dim3(64), 0, st, (int64_t)1, counts + nseg);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, counts, offs, (int)(nseg + 1), st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub.p, tb, counts, offs, (int)(nseg + 1), st));
    if (cap > 0) {
        hipLaunchKernelGGL(k_djoin<1>, dim3(grid), dim3(DJ_THREADS), 0, st, K, n, pts->x, pts->y, nseg, nullptr, offs,
                           out_pt, out_disk, cap, m, nullptr, pcount);
        SPADE_HIP(ctx, hipGetLastError());
    }
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    unsigned long long *h = (unsigned long long *)ensure_pinned(ctx, 64);
    if (!h) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(h, offs + nseg, 8, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *n_out = (int64_t)h[0];
    if (*n_out > cap) return set_error(ctx, SPADE_E_CAPACITY, "output capacity too small");
    return SPADE_OK;
}

// ------------------------------------------------------------ kNN selection
//
// The paper's plan (Sec. 5.2, "kNN Queries"): nested circles around the
// query point with radii in a geometric progression, one aggregation pass
// that counts the points in every circle, a distance selection with the
// smallest circle that holds at least k points, and a sort of those
// candidates by distance.  The paper anchors the circles at r_max (the
// largest distance from the point to a corner of the points' bounding box)
// with r_i = r_max / alpha^i.  Here alpha = 2 and the circles are first the
// powers of two r_j = 2^j, -511 <= j <= 511 (r_j^2 is a normal double, so
// the exact closed-disk test applies): they need no bounding box, so the
// aggregation is the only pass before the selection.  Only when more than
// the points inside r_511 are needed (distances beyond 6.7e153) does the
// query fall back to circles r_max 2^-i (i <= KNN_LEVELS) from the bounding
// box.  Every comparison is exact: the circle counts use the exact
// closed-disk test, and the candidates are ordered by their FP64 squared
// distance, then every run of keys too close to tell apart is re-ordered
// exactly (ties in distance: smaller id first).

constexpr int KNN_LEVELS = 48;
constexpr int KNN_THREADS = 256;

// Points' bounding box (finite points) as order keys.
__global__ __launch_bounds__(256) void k_knn_box(int64_t n, const double *X, const double *Y,
                                                 unsigned long long *bb)
{
    __shared__ unsigned long long s[4][256];
    unsigned long long k0 = ~0ull, k1 = ~0ull, k2 = ~0ull, k3 = ~0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = X[i], y = Y[i];
        if (!isfinite(x) || !isfinite(y)) continue;
        k0 = min(k0, okey_d(x)); k1 = min(k1, okey_d(-x));
        k2 = min(k2, okey_d(y)); k3 = min(k3, okey_d(-y));
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

struct KnnCircles {
    double px, py;
    double r[KNN_LEVELS + 1];
    double r2[KNN_LEVELS + 1];
};

// Aggregation over the nested circles: level[i] counts the points whose
// innermost containing circle is circle i (binary search with the exact
// predicate; the circles are nested).  The radii (device array cr, r then
// r^2) are read into LDS.
__global__ __launch_bounds__(KNN_THREADS) void k_knn_levels(int64_t n, const double *X, const double *Y, double px,
                                                            double py, const double *cr, unsigned long long *level)
{
    __shared__ unsigned int h[KNN_LEVELS + 1];
    __shared__ double sr[2 * (KNN_LEVELS + 1)];
    for (int k = threadIdx.x; k <= KNN_LEVELS; k += KNN_THREADS) h[k] = 0;
    for (int k = threadIdx.x; k < 2 * (KNN_LEVELS + 1); k += KNN_THREADS) sr[k] = cr[k];
    __syncthreads();
    const double *r = sr, *r2 = sr + (KNN_LEVELS + 1);
    for (int64_t i = (int64_t)blockIdx.x * KNN_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * KNN_THREADS) {
        const double x = X[i], y = Y[i];
        if (!in_disk(x, y, px, py, r[0], r2[0])) continue;   // non-finite points too
        int lo = 0, hi = KNN_LEVELS;   // in circle lo; find the innermost
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (in_disk(x, y, px, py, r[mid], r2[mid])) lo = mid; else hi = mid - 1;
        }
        atomicAdd(&h[lo], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= KNN_LEVELS; k += KNN_THREADS)
        if (h[k]) atomicAdd(&level[k], (unsigned long long)h[k]);
}

constexpr int KNN_JMIN = -511, KNN_JMAX = 511;
constexpr int KNN_BINS = KNN_JMAX - KNN_JMIN + 2;   // + the points outside every circle

__device__ __forceinline__ bool in_circle_pow2(double x, double y, double px, double py, int j)
{
    return in_disk(x, y, px, py, ldexp(1.0, j), ldexp(1.0, 2 * j));
}

// Aggregation over the circles r_j = 2^j: bins[j - KNN_JMIN] counts the
// finite points whose innermost containing circle is j, bins[KNN_BINS - 1]
// those outside circle KNN_JMAX.  The FP64 squared distance only gives the
// first guess at j (4^j <= d2 up to rounding); the exact test settles it,
// usually with two tests: j is outside, j + 1 inside.
// Only bins that were hit are added to the global counts.
__global__ __launch_bounds__(KNN_THREADS) void k_knn_pow2(int64_t n, const double *X, const double *Y, double px,
                                                          double py, unsigned long long *bins)
{
    __shared__ unsigned int h[KNN_BINS];
    for (int k = threadIdx.x; k < KNN_BINS; k += KNN_THREADS) h[k] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * KNN_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * KNN_THREADS) {
        const double x = __builtin_nontemporal_load(X + i), y = __builtin_nontemporal_load(Y + i);
        if (!(fabs(x) <= 1.7976931348623157e308 && fabs(y) <= 1.7976931348623157e308)) continue;
        const double dx = x - px, dy = y - py;
        const double d2 = dx * dx + dy * dy;
        int j;
        if (!(d2 > 0.0)) j = KNN_JMIN;
        else if (!(d2 <= 1.7976931348623157e308)) j = KNN_JMAX + 1;
        else j = min(max(ilogb(d2) >> 1, KNN_JMIN), KNN_JMAX + 1);   // 4^j <= d2 up to rounding
        if (j <= KNN_JMAX && !in_circle_pow2(x, y, px, py, j)) {
            do ++j;
            while (j <= KNN_JMAX && !in_circle_pow2(x, y, px, py, j));
        } else {
            // in circle j (or j past the last one): move inwards while inside
            while (j > KNN_JMIN && in_circle_pow2(x, y, px, py, j - 1)) --j;
        }
        atomicAdd(&h[j - KNN_JMIN], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < KNN_BINS; k += KNN_THREADS)
        if (h[k]) atomicAdd(&bins[k], (unsigned long long)h[k]);
}

// Candidate keys: FP64 squared distance (non-negative, so its bits order it)
// and the id.
__global__ void k_knn_keys(int64_t m, const uint32_t *ids, const double *X, const double *Y, double px, double py,
                           unsigned long long *key)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = ids[t];
        key[t] = (unsigned long long)__double_as_longlong(dist2(X[i], Y[i], px, py));
    }
}

__device__ __forceinline__ bool knn_close(unsigned long long a, unsigned long long b)
{
    const double qa = __longlong_as_double((long long)a), qb = __longlong_as_double((long long)b);
    return fabs(qa - qb) <= 1.7763568394002505e-15 * (qa + qb);
}

// Runs of consecutive keys too close to tell apart, starting before `upto`,
// are re-ordered by the exact comparison (ids break exact ties); one thread
// per run, insertion sort.
__global__ void k_knn_fix(int64_t m, int64_t upto, const unsigned long long *key, uint32_t *ids, const double *X,
                          const double *Y, double px, double py)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < upto && t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t > 0 && knn_close(key[t - 1], key[t])) continue;   // not a run start
        int64_t e = t + 1;
        while (e < m && knn_close(key[e - 1], key[e])) ++e;
        if (e - t < 2) continue;
        for (int64_t a = t + 1; a < e; ++a) {
            const uint32_t v = ids[a];
            int64_t b = a;
            while (b > t) {
                const uint32_t u = ids[b - 1];
                const int c = dist_cmp(X[u], Y[u], X[v], Y[v], px, py);
                if (c < 0 || (c == 0 && u < v)) break;
                ids[b] = u;
                --b;
            }
            ids[b] = v;
        }
    }
}

int knn_select(spade_ctx *ctx, const spade_points *pts, double px, double py, int64_t k, uint32_t *out_ids,
               int64_t *n_out)
{
    hipStream_t st = ctx->stream;
    *n_out = 0;
    if (!(std::isfinite(px) && std::isfinite(py))) return set_error(ctx, SPADE_E_INVALID, "query point must be finite");
    if (k < 0) return set_error(ctx, SPADE_E_INVALID, "negative k");
    if (k > 0 && !out_ids) return set_error(ctx, SPADE_E_INVALID, "out_ids is NULL");
    const int64_t n = pts->n;
    if (k == 0 || n == 0) return SPADE_OK;
    const int cus = num_cus_dj(ctx->device);
    // circles r_j = 2^j: bins of the innermost containing circle
    DevBuf &bb = ctx->scratch[S_BLOCKRED];
    const size_t bin_bytes = 8 * (size_t)KNN_BINS;
    if (ensure(ctx, bb, std::max<size_t>(bin_bytes, 64 + 8 * (KNN_LEVELS + 1) + 16 * (KNN_LEVELS + 1))))
        return SPADE_E_NOMEM;
    unsigned long long *dbins = (unsigned long long *)bb.p;
    hipLaunchKernelGGL(k_dj_zero, dim3(4), dim3(256), 0, st, (int64_t)KNN_BINS, dbins);
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[2], st));
    hipLaunchKernelGGL(k_knn_pow2, dim3((unsigned)std::min<int64_t>((n + KNN_THREADS - 1) / KNN_THREADS, cus * 8)),
                       dim3(KNN_THREADS), 0, st, n, pts->x, pts->y, px, py, dbins);
    SPADE_HIP(ctx, hipGetLastError());
    unsigned long long *hb = (unsigned long long *)ensure_pinned(ctx, bin_bytes + 16 * (KNN_LEVELS + 8));
    if (!hb) return set_error(ctx, SPADE_E_NOMEM, "pinned staging allocation failed");
    SPADE_HIP(ctx, hipMemcpyAsync(hb, dbins, bin_bytes, hipMemcpyDeviceToHost, st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    int64_t total = 0;
    for (int b = 0; b < KNN_BINS; ++b) total += (int64_t)hb[b];
    if (total == 0) return SPADE_OK;   // no finite point
    const int64_t want = std::min<int64_t>(k, total);
    int64_t cum = 0;
    double rsel = -1.0;
    for (int b = 0; b + 1 < KNN_BINS; ++b) {
        cum += (int64_t)hb[b];
        if (cum >= want) {
            rsel = std::ldexp(1.0, KNN_JMIN + b);
            break;
        }
    }
    if (rsel < 0.0) {
        // more points are needed than lie within 2^511: the circles
        // r_max 2^-i from the points' bounding box
        unsigned long long *dbb = dbins;
        unsigned long long *level = dbb + 4;
        SPADE_HIP(ctx, hipMemsetAsync(dbb, 0xff, 32, st));
        hipLaunchKernelGGL(k_dj_zero, dim3(1), dim3(64), 0, st, (int64_t)(KNN_LEVELS + 1), level);
        hipLaunchKernelGGL(k_knn_box, dim3(dj_grid(n, 1024)), dim3(256), 0, st, n, pts->x, pts->y, dbb);
        SPADE_HIP(ctx, hipGetLastError());
        unsigned long long *h = hb;
        SPADE_HIP(ctx, hipMemcpyAsync(h, dbb, 32, hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        auto from_key = [](unsigned long long kk) {
            const unsigned long long b = (kk & 0x8000000000000000ull) ? (kk & 0x7fffffffffffffffull) : ~kk;
            double d;
            std::memcpy(&d, &b, sizeof d);
            return d;
        };
        const double x0 = from_key(h[0]), x1 = -from_key(h[1]), y0 = from_key(h[2]), y1 = -from_key(h[3]);
        double rmax = 0.0;
        for (double cx : {x0, x1})
            for (double cy : {y0, y1}) rmax = std::max(rmax, std::hypot(cx - px, cy - py));
        // round up by a relative 2^-40: every finite point is then in circle 0
        // (the exact test decides), whatever the rounding of hypot
        rmax = rmax * (1.0 + std::ldexp(1.0, -40)) + std::ldexp(1.0, -1000);
        KnnCircles C;
        C.px = px;
        C.py = py;
        for (int i = 0; i <= KNN_LEVELS; ++i) {
            C.r[i] = std::ldexp(rmax, -i);
            C.r2[i] = C.r[i] * C.r[i];
        }
        double *cr = (double *)(level + (KNN_LEVELS + 1));
        double *hr = (double *)(hb + KNN_LEVELS + 8);
        std::memcpy(hr, C.r, 8 * (KNN_LEVELS + 1));
        std::memcpy(hr + KNN_LEVELS + 1, C.r2, 8 * (KNN_LEVELS + 1));
        SPADE_HIP(ctx, hipMemcpyAsync(cr, hr, 16 * (KNN_LEVELS + 1), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_knn_levels, dim3((unsigned)std::min<int64_t>((n + KNN_THREADS - 1) / KNN_THREADS, cus * 8)),
                           dim3(KNN_THREADS), 0, st, n, pts->x, pts->y, px, py, (const double *)cr, level);
        SPADE_HIP(ctx, hipGetLastError());
        SPADE_HIP(ctx, hipMemcpyAsync(h, level, 8 * (KNN_LEVELS + 1), hipMemcpyDeviceToHost, st));
        SPADE_HIP(ctx, hipStreamSynchronize(st));
        // count(r_i) = points whose innermost circle is i or deeper
        int64_t ltot = 0;
        for (int i = 0; i <= KNN_LEVELS; ++i) ltot += (int64_t)h[i];
        cum = 0;
        int sel = 0;
        for (int i = KNN_LEVELS; i >= 0; --i) {
            cum += (int64_t)h[i];
            if (cum >= std::min<int64_t>(k, ltot)) { sel = i; break; }
        }
        rsel = C.r[sel];
    }
    // distance selection with circle sel: the candidates, ascending ids
    int64_t m = 0;
    DevBuf &bc = ctx->scratch[S_VALS2];
    if (ensure(ctx, bc, 4 * (size_t)std::max<int64_t>(cum, 1))) return SPADE_E_NOMEM;
    int rc = select_disk(ctx, pts, px, py, rsel, (uint32_t *)bc.p, cum, &m);
    if (rc) return rc;
    if (m != cum) return set_error(ctx, SPADE_E_HIP, "internal: circle count and selection disagree");
    // order by distance, exactly; the first k are the result
    DevBuf &bk = ctx->scratch[S_KEYS], &bk2 = ctx->scratch[S_KEYS2], &bi = ctx->scratch[S_VALS];
    if (ensure(ctx, bk, 8 * (size_t)std::max<int64_t>(m, 1)) || ensure(ctx, bk2, 8 * (size_t)std::max<int64_t>(m, 1)) ||
        ensure(ctx, bi, 4 * (size_t)std::max<int64_t>(m, 1)))
        return SPADE_E_NOMEM;
    hipLaunchKernelGGL(k_knn_keys, dim3(dj_grid(m)), dim3(256), 0, st, m, (const uint32_t *)bc.p, pts->x, pts->y, px,
                       py, (unsigned long long *)bk.p);
    SPADE_HIP(ctx, hipGetLastError());
    DevBuf &cub = ctx->scratch[S_CUBTMP];
    size_t tb = 0;
    SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const unsigned long long *)bk.p,
                                                      (unsigned long long *)bk2.p, (const uint32_t *)bc.p,
                                                      (uint32_t *)bi.p, (int)m, 0, 64, st));
    if (ensure(ctx, cub, std::max<size_t>(tb, 1))) return SPADE_E_NOMEM;
    SPADE_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub.p, tb, (const unsigned long long *)bk.p,
                                                      (unsigned long long *)bk2.p, (const uint32_t *)bc.p,
                                                      (uint32_t *)bi.p, (int)m, 0, 64, st));
    const int64_t kk = std::min<int64_t>(k, m);
    hipLaunchKernelGGL(k_knn_fix, dim3(dj_grid(kk + 1)), dim3(256), 0, st, m, kk + 1,
                       (const unsigned long long *)bk2.p, (uint32_t *)bi.p, pts->x, pts->y, px, py);
    SPADE_HIP(ctx, hipGetLastError());
    SPADE_HIP(ctx, hipMemcpyAsync(out_ids, bi.p, 4 * (size_t)kk, hipMemcpyDeviceToDevice, st));
    if (ctx->timing) SPADE_HIP(ctx, hipEventRecord(ctx->ev[3], st));
    SPADE_HIP(ctx, hipStreamSynchronize(st));
    *n_out = kk;
    return SPADE_OK;
}

}  // namespace spade
