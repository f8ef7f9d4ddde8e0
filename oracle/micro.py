"""Exact-rational micro-oracle for tiny inputs (test infrastructure only).

An independent second route to the same definition as ``oracle.c``: every
coordinate is converted to ``fractions.Fraction`` (exact for finite doubles),
so the orientation determinant is evaluated in exact rational arithmetic
instead of a floating-point filter plus big-integer fallback.  Pure Python
loops: only for inputs of at most a few thousand point-edge tests.

Definition (paper Sec. 5.2 selection / join / aggregation, with the
half-open crossing rule used throughout this repository): a point p is inside
a polygon iff an odd number of its edges (a, b) satisfy
``(a.y > p.y) != (b.y > p.y)`` and have their crossing with the horizontal
line through p strictly to the right of p.
"""
from __future__ import annotations

from fractions import Fraction


def orient(a, b, c) -> int:
    """Exact sign of (b - a) x (c - a) for 2-tuples of floats."""
    ax, ay = Fraction(a[0]), Fraction(a[1])
    bx, by = Fraction(b[0]), Fraction(b[1])
    cx, cy = Fraction(c[0]), Fraction(c[1])
    d = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    return (d > 0) - (d < 0)


def crossing_right(a, b, p) -> bool:
    """True iff the edge a-b crosses the ray from p towards +x.

    Computes the crossing abscissa exactly instead of an orientation sign, so
    it is a different formulation of the same rule: the edge must straddle
    p.y half-openly and meet the line y = p.y strictly right of p.
    """
    ay, by, py = Fraction(a[1]), Fraction(b[1]), Fraction(p[1])
    if (ay > py) == (by > py):
        return False
    ax, bx, px = Fraction(a[0]), Fraction(b[0]), Fraction(p[0])
    t = (py - ay) / (by - ay)
    xc = ax + t * (bx - ax)
    return xc > px


def inside(p, rings) -> bool:
    """rings: list of lists of (x, y) vertices, each implicitly closed."""
    par = False
    for ring in rings:
        n = len(ring)
        for j in range(n):
            if crossing_right(ring[j], ring[(j + 1) % n], p):
                par = not par
    return par


def polys_to_rings(polys):
    """CSR polygon set -> list (per polygon) of rings (lists of vertices)."""
    M = int(polys["n_polys"])
    pro = polys.get("poly_ring_off")
    rvo = polys["ring_vtx_off"]
    vx, vy = polys["vx"], polys["vy"]
    out = []
    for k in range(M):
        r0, r1 = (int(pro[k]), int(pro[k + 1])) if pro is not None else (k, k + 1)
        rings = []
        for r in range(r0, r1):
            v0, v1 = int(rvo[r]), int(rvo[r + 1])
            rings.append([(float(vx[v]), float(vy[v])) for v in range(v0, v1)])
        out.append(rings)
    return out


def join_count(xs, ys, polys):
    rings = polys_to_rings(polys)
    counts = [0] * len(rings)
    for x, y in zip(xs, ys):
        for k, rr in enumerate(rings):
            if inside((float(x), float(y)), rr):
                counts[k] += 1
    return counts
