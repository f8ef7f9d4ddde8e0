// Device-side canvas lookup shared by the probe kernels (single canvas and
// canvas sets): pixel mapping, the coarse and full canvas levels, and the
// exact test of one boundary-index record.
#pragma once

#include "common.h"
#include "exact.h"

namespace spade {

__device__ __forceinline__ size_t tile_index(int Wt, int c, int r)
{
    return ((size_t)(r >> 4) * Wt + (c >> 4)) * 256 + ((r & 15) << 4) + (c & 15);
}

// Global-memory views: loads through these are known not to touch LDS, so
// the compiler may issue them ahead of the LDS histogram updates.
typedef const uint32_t __attribute__((address_space(1))) *gu32p;
typedef const uint16_t __attribute__((address_space(1))) *gu16p;
typedef const uint64_t __attribute__((address_space(1))) *gu64p;

// Canvas lookup state of one point: the word once known, or where to read it.
struct Look {
    uint32_t word;   // final canvas word when !full
    uint32_t full;   // the word is read from the full canvas
    uint32_t fidx;   // full-canvas index (full)
};

// Level 1: bbox test, pixel mapping, coarse word from LDS.
__device__ __forceinline__ Look look_coarse(const CanvasView &cv, const uint16_t *coarse, double x, double y)
{
    Look L{0u, 0u, 0u};
    // exact half-open bbox test; NaN fails every comparison
    if (!(cv.bx0 <= x && x < cv.bx1 && cv.by0 <= y && y < cv.by1)) return L;
    const double u = __dmul_rn(__dsub_rn(x, cv.X0), cv.sx);
    const double v = __dmul_rn(__dsub_rn(y, cv.Y0), cv.sy);
    const int c = min((int)u, cv.W - 1);
    const int r = min((int)v, cv.H - 1);
    const int ci = (r >> cv.blog) * cv.Wc + (c >> cv.blog);
    const uint32_t cw = cv.cbyte ? ((const uint8_t *)coarse)[ci] : coarse[ci];
    if (cw != (cv.cbyte ? COARSE_BYTE_FULL : (uint32_t)COARSE_FULL)) { L.word = cw; return L; }
    L.full = 1u;
    L.fidx = (uint32_t)tile_index(cv.Wt, c, r);
    return L;
}

// Canvas word of (x, y): 0, label + 1, or BFLAG | first candidate record.
__device__ __forceinline__ uint32_t lookup(const CanvasView &cv, const uint16_t *coarse, double x, double y)
{
    const Look L = look_coarse(cv, coarse, x, y);
    return L.full ? ((gu32p)cv.cells)[L.fidx] : L.word;
}

__device__ __forceinline__ bool cand_inside(const Edge *ledges, const double2 *pspan, const Cand &cd, double x,
                                            double y)
{
    bool in = (cd.meta & CAND_S) != 0;
    const uint32_t nloc = (cd.meta >> 2) & 0x7fffu;
    const uint32_t npart = cd.meta >> 17;
    if (nloc > 0) in ^= crosses(cd.e0.xlo, cd.e0.ylo, cd.e0.xhi, cd.e0.yhi, x, y);
    if (npart > 0) in ^= straddles(cd.s0.x, cd.s0.y, y);
    const Edge *le = ledges + cd.eoff;   // local edges after the first
    for (uint32_t t = 1; t < nloc; ++t) {
        const Edge e = le[t - 1];
        in ^= crosses(e.xlo, e.ylo, e.xhi, e.yhi, x, y);
    }
    const double2 *ps = pspan + cd.poff;
    for (uint32_t t = 1; t < npart; ++t) {
        const double2 s = ps[t];
        in ^= straddles(s.x, s.y, y);
    }
    return in;
}

__device__ __forceinline__ bool cand_inside(const CanvasView &cv, const Cand &cd, double x, double y)
{
    return cand_inside(cv.ledges, cv.pspan, cd, x, y);
}

// Cooperative copy of the coarse canvas into LDS (whole 32-bit words; the
// device array is padded to them).
__device__ __forceinline__ void load_coarse(const CanvasView &cv, uint16_t *dst, int nthreads)
{
    const int n = cv.Wc * cv.Hc;
    const int nw = cv.cbyte ? (n + 3) >> 2 : (n + 1) >> 1;
    const uint32_t *src = (const uint32_t *)cv.coarse;
    uint32_t *d = (uint32_t *)dst;
    for (int i = threadIdx.x; i < nw; i += nthreads) d[i] = src[i];
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

}  // namespace spade
