// Exact geometric predicates on the device (FP64, gfx950).
//
// orient_sign(a, b, c) = sign((b.x-a.x)(c.y-a.y) - (b.y-a.y)(c.x-a.x)),
// exactly.  A floating-point evaluation with rounding-exact operations
// (no contraction into FMA) is accepted when it clears the a-priori error
// bound of Shewchuk 1997 for this determinant form, (3 + 16 eps) eps
// (|l| + |r|) with eps = 2^-53.  Otherwise the determinant is rebuilt as a
// non-overlapping floating-point expansion from error-free transformations
// (Knuth's TwoSum / TwoDiff and the FMA-based TwoProduct) and its sign is the
// sign of its most significant non-zero component.  Exact whenever no
// product underflows into subnormals and nothing overflows.
//
// cross(e, p) implements the crossing rule of the containment test: the edge
// (lo, hi), lo.y <= hi.y, straddles the horizontal line through p half-openly
// (lo.y <= p.y < hi.y) and meets it strictly to the right of p.
#pragma once

#include <hip/hip_runtime.h>

namespace spade {

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = __dadd_rn(a, b);
    double bv = __dsub_rn(s, a);
    double av = __dsub_rn(s, bv);
    double br = __dsub_rn(b, bv);
    double ar = __dsub_rn(a, av);
    e = __dadd_rn(ar, br);
}

__device__ __forceinline__ void two_diff(double a, double b, double &d, double &e)
{
    d = __dsub_rn(a, b);
    double bv = __dsub_rn(a, d);
    double av = __dadd_rn(d, bv);
    double br = __dsub_rn(bv, b);
    double ar = __dsub_rn(a, av);
    e = __dadd_rn(ar, br);
}

__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e)
{
    p = __dmul_rn(a, b);
    e = __fma_rn(a, b, -p);
}

// Adds q into the non-overlapping expansion h[0..n) (increasing magnitude),
// dropping zero components; returns the new length (at most n + 1).
__device__ __forceinline__ int grow_expansion(double *h, int n, double q)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        double s, e;
        two_sum(q, h[i], s, e);
        q = s;
        if (e != 0.0) h[m++] = e;
    }
    if (q != 0.0) h[m++] = q;
    return m;
}

__device__ __noinline__ int orient_sign_exact(double ax, double ay, double bx, double by,
                                              double cx, double cy)
{
    // (b - a) and (c - a) as exact two-term differences
    double d1, e1, d2, e2, d3, e3, d4, e4;
    two_diff(bx, ax, d1, e1);   // bx - ax
    two_diff(cy, ay, d2, e2);   // cy - ay
    two_diff(by, ay, d3, e3);   // by - ay
    two_diff(cx, ax, d4, e4);   // cx - ax
    double u[2] = {d1, e1}, v[2] = {d2, e2}, w[2] = {d3, e3}, z[2] = {d4, e4};
    double h[18];
    int n = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double p, e;
            two_prod(u[i], v[j], p, e);
            n = grow_expansion(h, n, e);
            n = grow_expansion(h, n, p);
            two_prod(w[i], z[j], p, e);
            n = grow_expansion(h, n, -e);
            n = grow_expansion(h, n, -p);
        }
    if (n == 0) return 0;
    double top = h[n - 1];
    return (top > 0.0) - (top < 0.0);
}

__device__ __forceinline__ int orient_sign(double ax, double ay, double bx, double by,
                                           double cx, double cy)
{
    double detleft = __dmul_rn(__dsub_rn(bx, ax), __dsub_rn(cy, ay));
    double detright = __dmul_rn(__dsub_rn(by, ay), __dsub_rn(cx, ax));
    double det = __dsub_rn(detleft, detright);
    // (3 + 16 eps) eps with eps = 2^-53
    const double errbound = 3.3306690738754716e-16;
    double bound = __dmul_rn(errbound, __dadd_rn(fabs(detleft), fabs(detright)));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient_sign_exact(ax, ay, bx, by, cx, cy);
}

// Half-open straddle of the horizontal line through py.
__device__ __forceinline__ bool straddles(double ylo, double yhi, double py)
{
    return ylo <= py && py < yhi;
}

// cross(e, p) for an edge stored with ylo <= yhi.
__device__ __forceinline__ bool crosses(double xlo, double ylo, double xhi, double yhi,
                                        double px, double py)
{
    if (!straddles(ylo, yhi, py)) return false;
    return orient_sign(xlo, ylo, xhi, yhi, px, py) > 0;
}

}  // namespace spade
