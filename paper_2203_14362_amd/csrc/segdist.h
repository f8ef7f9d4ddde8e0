// Exact distance-to-segment predicate on the device: is (px, py) within
// closed distance r of the segment ab?  Used for the distance constraints
// around lines and polygon edges (the rounded rectangles of Sec. 4.2).
//
// With t = (p - a).(b - a), L = |b - a|^2 and C = cross(b - a, p - a), the
// point is within distance r iff |p - a| <= r when t <= 0, |p - b| <= r when
// t >= L, and C^2 <= r^2 L when 0 < t < L (for a == b the first test
// alone).  The endpoint tests are the exact closed-disk predicate; the signs
// of t and of (p - b).(a - b) = L - t are decided like an orientation
// determinant (same a-priori bound, then an expansion from TwoDiff /
// TwoProduct); the sign of
// r^2 L - C^2 is accepted from FP64 values when an interval enclosing C (the
// orientation bound) and L clears it by a relative 1e-12 margin, and is
// otherwise rebuilt as an expansion: C and L as expansions of their exact
// terms, each shortened by Shewchuk's compression (Adaptive Precision
// Floating-Point Arithmetic, 1997), then r^2 L - C^2 accumulated product by
// product.  Exact whenever no product overflows or underflows into
// subnormals.
#pragma once

#include "disk.h"
#include "exact.h"

namespace spade {

struct Seg {
    double ax, ay, bx, by;
};

// In-place compression of a non-overlapping expansion e[0..m) (increasing
// magnitude) into a non-adjacent one with the same value; returns its
// length.  Two passes: from the largest component down, then back up.
__device__ __forceinline__ int compress_expansion(double *e, int m)
{
    if (m <= 1) return m;
    int bottom = m - 1;
    double q = e[m - 1];
    for (int i = m - 2; i >= 0; --i) {
        double s, t;
        two_sum(q, e[i], s, t);
        if (t != 0.0) {
            e[bottom--] = s;
            q = t;
        } else {
            q = s;
        }
    }
    e[bottom] = q;
    int top = 0;
    for (int i = bottom + 1; i < m; ++i) {
        double s, t;
        two_sum(e[i], q, s, t);
        if (t != 0.0) e[top++] = t;
        q = s;
    }
    e[top++] = q;
    return top;
}

// Sign of (p - a).(b - a) from an exact expansion.
__device__ __noinline__ int dot_sign_exact(double px, double py, double ax, double ay, double bx, double by)
{
    double u[2], v[2], w[2], z[2];
    two_diff(px, ax, u[0], u[1]);
    two_diff(bx, ax, v[0], v[1]);
    two_diff(py, ay, w[0], w[1]);
    two_diff(by, ay, z[0], z[1]);
    double h[18];
    int n = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double p, e;
            two_prod(u[i], v[j], p, e);
            n = grow_expansion(h, n, e);
            n = grow_expansion(h, n, p);
            two_prod(w[i], z[j], p, e);
            n = grow_expansion(h, n, e);
            n = grow_expansion(h, n, p);
        }
    if (n == 0) return 0;
    const double top = h[n - 1];
    return (top > 0.0) - (top < 0.0);
}

// Sign of (p - a).(b - a), exactly.
__device__ __forceinline__ int dot_sign(double px, double py, double ax, double ay, double bx, double by)
{
    const double l = __dmul_rn(__dsub_rn(px, ax), __dsub_rn(bx, ax));
    const double rr = __dmul_rn(__dsub_rn(py, ay), __dsub_rn(by, ay));
    const double s = __dadd_rn(l, rr);
    const double bound = __dmul_rn(3.3306690738754716e-16, __dadd_rn(fabs(l), fabs(rr)));
    if (s > bound) return 1;
    if (-s > bound) return -1;
    return dot_sign_exact(px, py, ax, ay, bx, by);
}

// Sign of r^2 L - C^2 from exact expansions.
__device__ __noinline__ int perp_sign_exact(double px, double py, const Seg &s, double r)
{
    double ex[2], ey[2], dx[2], dy[2];
    two_diff(s.bx, s.ax, ex[0], ex[1]);
    two_diff(s.by, s.ay, ey[0], ey[1]);
    two_diff(px, s.ax, dx[0], dx[1]);
    two_diff(py, s.ay, dy[0], dy[1]);
    // C = ex * dy - ey * dx
    double c[18];
    int nc = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double p, e;
            two_prod(ex[i], dy[j], p, e);
            nc = grow_expansion(c, nc, e);
            nc = grow_expansion(c, nc, p);
            two_prod(ey[i], dx[j], p, e);
            nc = grow_expansion(c, nc, -e);
            nc = grow_expansion(c, nc, -p);
        }
    nc = compress_expansion(c, nc);
    // L = ex^2 + ey^2 with (d + t)^2 = d^2 + 2dt + t^2
    double l[14];
    int nl = 0;
    for (int k = 0; k < 2; ++k) {
        const double *w = k == 0 ? ex : ey;
        double p, e;
        two_prod(w[0], w[0], p, e);
        nl = grow_expansion(l, nl, e);
        nl = grow_expansion(l, nl, p);
        two_prod(2.0 * w[0], w[1], p, e);
        nl = grow_expansion(l, nl, e);
        nl = grow_expansion(l, nl, p);
        two_prod(w[1], w[1], p, e);
        nl = grow_expansion(l, nl, e);
        nl = grow_expansion(l, nl, p);
    }
    nl = compress_expansion(l, nl);
    double r2[2];
    two_prod(r, r, r2[1], r2[0]);
    double acc[56];
    int n = 0;
    auto add = [&](double a, double b, double sign) {
        double p, e;
        two_prod(a, b, p, e);
        n = grow_expansion(acc, n, sign * e);
        n = grow_expansion(acc, n, sign * p);
        if (n > 48) n = compress_expansion(acc, n);
    };
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < nl; ++j) add(r2[i], l[j], 1.0);
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) add(c[i], c[j], -1.0);
    if (n == 0) return 0;
    const double top = acc[n - 1];
    return (top > 0.0) - (top < 0.0);
}

// Sign of r^2 L - C^2, exactly; r2 = fl(r * r).
__device__ __forceinline__ int perp_sign(double px, double py, const Seg &s, double r, double r2)
{
    const double ex = __dsub_rn(s.bx, s.ax), ey = __dsub_rn(s.by, s.ay);
    const double c1 = __dmul_rn(ex, __dsub_rn(py, s.ay));
    const double c2 = __dmul_rn(ey, __dsub_rn(px, s.ax));
    const double c = fabs(__dsub_rn(c1, c2));
    const double ec = __dmul_rn(3.3306690738754716e-16, __dadd_rn(fabs(c1), fabs(c2)));
    const double l2 = __dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey));
    const double rl = __dmul_rn(r2, l2);
    const double hi = __dadd_rn(c, ec);
    const double lo = fmax(__dsub_rn(c, ec), 0.0);
    const double hi2 = __dmul_rn(hi, hi), lo2 = __dmul_rn(lo, lo);
    if (rl > 1e-250 && hi2 < 1e250) {
        if (__dmul_rn(hi2, 1.0 + 1e-12) < __dmul_rn(rl, 1.0 - 1e-12)) return 1;
        if (__dmul_rn(lo2, 1.0 - 1e-12) > __dmul_rn(rl, 1.0 + 1e-12)) return -1;
    }
    return perp_sign_exact(px, py, s, r);
}

// The closed-distance test of (px, py) against segment s; r2 = fl(r * r).
// The nearest point of the segment is a when t <= 0, b when t >= L, else
// the foot of the perpendicular, whose distance is at most both endpoint
// distances: so one endpoint disk or the perpendicular test decides (a
// point segment is its disk).  Points with a non-finite coordinate are never
// within.
__device__ __forceinline__ bool seg_near(double px, double py, const Seg &s, double r, double r2)
{
    if (!(fabs(px) <= 1.7976931348623157e308 && fabs(py) <= 1.7976931348623157e308)) return false;
    if ((s.ax == s.bx && s.ay == s.by) || dot_sign(px, py, s.ax, s.ay, s.bx, s.by) <= 0)   // t <= 0
        return in_disk(px, py, s.ax, s.ay, r, r2);
    if (dot_sign(px, py, s.bx, s.by, s.ax, s.ay) <= 0)                                      // t >= L
        return in_disk(px, py, s.bx, s.by, r, r2);
    return perp_sign(px, py, s, r, r2) >= 0;
}

}  // namespace spade
