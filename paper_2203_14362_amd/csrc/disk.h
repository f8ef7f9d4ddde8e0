// Exact closed-disk predicate on the device: is (x, y) within distance r of
// (cx, cy)?  Decided as the sign of r^2 - (x - cx)^2 - (y - cy)^2 on the
// FP64 inputs.  A floating-point evaluation with rounding-exact operations
// is accepted when it clears an error bound of 16 eps (r^2 + (x-cx)^2 +
// (y-cy)^2), eps = 2^-53 (each of the three terms carries at most three
// roundings, the sum and the difference one each); otherwise the expression
// is rebuilt as a non-overlapping expansion from error-free transformations
// (TwoDiff of the differences, TwoProduct of their parts:
// (d + t)^2 = d^2 + 2dt + t^2).  Exact whenever no square overflows or
// underflows into subnormals.  Points with a non-finite coordinate are
// outside.
#pragma once

#include "exact.h"

namespace spade {

// Sign of r^2 - (x-cx)^2 - (y-cy)^2 from an exact expansion.
__device__ __noinline__ int disk_sign_exact(double x, double y, double cx, double cy, double r)
{
    double h[16];   // 14 error-free terms, grown one at a time
    int n = 0;
    double p, e;
    two_prod(r, r, p, e);
    n = grow_expansion(h, n, e);
    n = grow_expansion(h, n, p);
    double d[2], t[2];
    two_diff(x, cx, d[0], t[0]);
    two_diff(y, cy, d[1], t[1]);
    for (int k = 0; k < 2; ++k) {
        two_prod(d[k], d[k], p, e);
        n = grow_expansion(h, n, -e);
        n = grow_expansion(h, n, -p);
        two_prod(2.0 * d[k], t[k], p, e);
        n = grow_expansion(h, n, -e);
        n = grow_expansion(h, n, -p);
        two_prod(t[k], t[k], p, e);
        n = grow_expansion(h, n, -e);
        n = grow_expansion(h, n, -p);
    }
    if (n == 0) return 0;
    const double top = h[n - 1];
    return (top > 0.0) - (top < 0.0);
}

// The closed-disk test; r2 = fl(r * r).
__device__ __forceinline__ bool in_disk(double x, double y, double cx, double cy, double r, double r2)
{
    if (!(fabs(x) <= 1.7976931348623157e308 && fabs(y) <= 1.7976931348623157e308)) return false;
    const double dx = __dsub_rn(x, cx), dy = __dsub_rn(y, cy);
    const double q = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
    const double s = __dsub_rn(r2, q);
    const double bound = __dmul_rn(1.7763568394002505e-15, __dadd_rn(r2, q));   // 16 * 2^-53
    if (s > bound) return true;
    if (-s > bound) return false;
    return disk_sign_exact(x, y, cx, cy, r) >= 0;
}

// Sign of |a - c|^2 - |b - c|^2, exactly: which of two points is nearer to
// c (negative: a is nearer).  Same filter and expansion construction.
__device__ __noinline__ int dist_cmp_exact(double ax, double ay, double bx, double by, double cx, double cy)
{
    double h[26];
    int n = 0;
    const double px[2] = {ax, bx}, py[2] = {ay, by};
    for (int w = 0; w < 2; ++w) {
        const double sg = w == 0 ? 1.0 : -1.0;
        double d[2], t[2], p, e;
        two_diff(px[w], cx, d[0], t[0]);
        two_diff(py[w], cy, d[1], t[1]);
        for (int k = 0; k < 2; ++k) {
            two_prod(d[k], d[k], p, e);
            n = grow_expansion(h, n, sg * e);
            n = grow_expansion(h, n, sg * p);
            two_prod(2.0 * d[k], t[k], p, e);
            n = grow_expansion(h, n, sg * e);
            n = grow_expansion(h, n, sg * p);
            two_prod(t[k], t[k], p, e);
            n = grow_expansion(h, n, sg * e);
            n = grow_expansion(h, n, sg * p);
        }
    }
    if (n == 0) return 0;
    const double top = h[n - 1];
    return (top > 0.0) - (top < 0.0);
}

}  // namespace spade

namespace spade {

// Squared distance of (x, y) to c in FP64 (the filter's value).
__device__ __forceinline__ double dist2(double x, double y, double cx, double cy)
{
    const double dx = __dsub_rn(x, cx), dy = __dsub_rn(y, cy);
    return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

// Exact sign of |a - c|^2 - |b - c|^2 with the FP64 filter first.
__device__ __forceinline__ int dist_cmp(double ax, double ay, double bx, double by, double cx, double cy)
{
    const double qa = dist2(ax, ay, cx, cy), qb = dist2(bx, by, cx, cy);
    const double s = __dsub_rn(qa, qb);
    const double bound = __dmul_rn(1.7763568394002505e-15, __dadd_rn(qa, qb));   // 16 * 2^-53
    if (s > bound) return 1;
    if (-s > bound) return -1;
    return dist_cmp_exact(ax, ay, bx, by, cx, cy);
}

}  // namespace spade
