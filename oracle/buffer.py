"""CPU oracle for distance selection from lines and from a polygon.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this; the product path never does.

Sec. 4.2 (canvases for distance-based queries) gives the shapes a distance
constraint draws: around a line, the union of one rounded rectangle per
segment (every position within distance r of that segment); around a polygon,
the polygon itself together with the rounded rectangles of its edges.
Sec. 5.2's distance selection keeps the points of the stream inside that
shape.  This oracle evaluates the definition, not the drawing:

* near a set of lines: the point's Euclidean distance to some segment is at
  most r (closed);
* within r of a polygon: the point is inside the polygon (the selection
  oracle's test) or within distance r of one of its edges.

The distance of p to the closed segment ab is |p - a| when a == b; otherwise,
with t = (p - a).(b - a) and L = |b - a|^2, it is |p - a| for t <= 0,
|p - b| for t >= L and |cross(b - a, p - a)| / sqrt(L) in between, so the
comparison with r is made on squares: |p - a|^2 <= r^2, |p - b|^2 <= r^2, or
0 < t < L and cross^2 <= r^2 L.  Every decision is exact on the FP64 inputs:
numpy classifies each (point, segment) pair in FP64 first, and a pair whose
FP64 quantities lie within a generous margin of a decision boundary (1e-9 of
the magnitudes of the terms, far above the few ulps the evaluation can be off
by), or whose magnitudes leave the safe range, is decided again with
``fractions.Fraction``.  Points with a non-finite coordinate are never kept.

Geometry uses the polygon-set CSR layout (``ring_vtx_off``, ``vx``, ``vy``).
As lines, every ring is an open polyline (segments between consecutive
vertices; a one-vertex ring is a point); as a polygon, rings are closed.

The distance join with lines (Sec. 5.2, types (1) and (2)) takes every ring
as one line object: the pairs (point, line) of every point within r (one
distance, or one per line) of that line, ascending by (point, line).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

MARGIN = 1e-9


def segments(polys, closed: bool):
    """Segment endpoints (ax, ay, bx, by), float64 arrays, of a polygon set's
    rings: consecutive vertices, plus the closing edge when ``closed``; a
    one-vertex ring gives one point-segment (a == b)."""
    rvo = np.asarray(polys["ring_vtx_off"], dtype=np.int64)
    vx = np.asarray(polys["vx"], dtype=np.float64)
    vy = np.asarray(polys["vy"], dtype=np.float64)
    a, b = [], []
    for r in range(rvo.size - 1):
        o, e = int(rvo[r]), int(rvo[r + 1])
        n = e - o
        if n == 0:
            continue
        if n == 1:
            a.append(o)
            b.append(o)
            continue
        idx = np.arange(o, e)
        if closed:
            a.extend(idx.tolist())
            b.extend(np.roll(idx, -1).tolist())
        else:
            a.extend(idx[:-1].tolist())
            b.extend(idx[1:].tolist())
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    return vx[a], vy[a], vx[b], vy[b]


def seg_within_exact(px: float, py: float, ax: float, ay: float, bx: float, by: float, r: float) -> bool:
    """The closed-distance test of one pair in rational arithmetic."""
    P = (Fraction(px), Fraction(py))
    A = (Fraction(ax), Fraction(ay))
    B = (Fraction(bx), Fraction(by))
    r2 = Fraction(r) * Fraction(r)
    dax, day = P[0] - A[0], P[1] - A[1]
    if dax * dax + day * day <= r2:
        return True
    dbx, dby = P[0] - B[0], P[1] - B[1]
    if dbx * dbx + dby * dby <= r2:
        return True
    ex, ey = B[0] - A[0], B[1] - A[1]
    L = ex * ex + ey * ey
    if L == 0:
        return False
    t = dax * ex + day * ey
    if t <= 0 or t >= L:
        return False
    c = ex * day - ey * dax
    return c * c <= r2 * L


def _pairs_within(px, py, ax, ay, bx, by, r):
    """Vectorised FP64 decision of pairs (arrays broadcast together), with the
    undecided pairs settled exactly.  Returns a bool array."""
    with np.errstate(over="ignore", invalid="ignore"):
        r2 = r * r
        dax, day = px - ax, py - ay
        dbx, dby = px - bx, py - by
        da2 = dax * dax + day * day
        db2 = dbx * dbx + dby * dby
        ex, ey = bx - ax, by - ay
        L = ex * ex + ey * ey
        t1, t2 = dax * ex, day * ey
        t = t1 + t2
        tmag = np.abs(t1) + np.abs(t2)
        u1, u2 = -dbx * ex, -dby * ey           # (p - b).(a - b)
        u = u1 + u2
        umag = np.abs(u1) + np.abs(u2)
        c1, c2 = ex * day, ey * dax
        c = c1 - c2
        cmag = np.abs(c1) + np.abs(c2)
        lhs = c * c
        rhs = r2 * L
        cscale = cmag * cmag + rhs
        a_in = da2 - r2 < -MARGIN * (da2 + r2)
        a_out = da2 - r2 > MARGIN * (da2 + r2)
        b_in = db2 - r2 < -MARGIN * (db2 + r2)
        b_out = db2 - r2 > MARGIN * (db2 + r2)
        t_pos = t > MARGIN * tmag
        t_neg = t < -MARGIN * tmag
        u_pos = u > MARGIN * umag
        u_neg = u < -MARGIN * umag
        c_in = lhs - rhs < -MARGIN * cscale
        c_out = lhs - rhs > MARGIN * cscale
        degenerate = (ex == 0) & (ey == 0)
        known_in = a_in | b_in | (~degenerate & t_pos & u_pos & c_in)
        known_out = a_out & b_out & (degenerate | t_neg | u_neg | c_out)
        scale = np.maximum.reduce([np.broadcast_to(v, da2.shape) for v in (da2, db2, r2, L, cscale)])
        safe = np.isfinite(scale) & (scale > 1e-250) & (scale < 1e250)
    within = np.array(known_in & safe)
    unsure = ~(safe & (known_in | known_out))
    if unsure.any():
        shape = within.shape
        P = np.broadcast_arrays(px, py, ax, ay, bx, by, np.full(shape, r))
        for idx in zip(*np.nonzero(unsure)):
            within[idx] = seg_within_exact(*(float(v[idx]) for v in P))
    return within


def select_near_segments(x, y, ax, ay, bx, by, r: float, chunk: int = 1 << 22) -> np.ndarray:
    """Ascending ids (int64) of the points within distance r of some segment
    (ax[k], ay[k]) - (bx[k], by[k])."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if not (math.isfinite(r) and r >= 0):
        raise ValueError("radius must be finite and >= 0")
    ax, ay, bx, by = (np.asarray(v, dtype=np.float64) for v in (ax, ay, bx, by))
    if not (np.isfinite(ax).all() and np.isfinite(ay).all() and np.isfinite(bx).all() and np.isfinite(by).all()):
        raise ValueError("segment coordinates must be finite")
    keep = np.zeros(x.size, dtype=bool)
    fin = np.isfinite(x) & np.isfinite(y)
    order = np.argsort(np.where(fin, x, np.inf), kind="stable")
    xs = np.where(fin, x, np.inf)[order]
    for k in range(ax.size):
        # candidates: the segment's box widened by r (and a relative margin)
        pad = r + 1e-9 * (abs(ax[k]) + abs(bx[k]) + abs(ay[k]) + abs(by[k]) + r) + 1e-300
        lo = np.searchsorted(xs, min(ax[k], bx[k]) - pad, side="left")
        hi = np.searchsorted(xs, max(ax[k], bx[k]) + pad, side="right")
        cand = order[lo:hi]
        cand = cand[~keep[cand]]
        yc = y[cand]
        cand = cand[(yc >= min(ay[k], by[k]) - pad) & (yc <= max(ay[k], by[k]) + pad)]
        for s in range(0, cand.size, chunk):
            cc = cand[s:s + chunk]
            keep[cc] |= _pairs_within(x[cc], y[cc], ax[k], ay[k], bx[k], by[k], r)
    return np.nonzero(keep & fin)[0].astype(np.int64)


def select_near_lines(x, y, lines, r: float) -> np.ndarray:
    """Points within distance r of a set of polylines (each ring of the CSR
    set an open polyline)."""
    return select_near_segments(x, y, *segments(lines, closed=False), r)


def select_within_polygon(x, y, poly, r: float) -> np.ndarray:
    """Points inside one polygon (the selection oracle's containment test) or
    within distance r of one of its edges (rings closed)."""
    from . import select
    inside = select(x, y, poly)
    near = select_near_segments(x, y, *segments(poly, closed=True), r)
    return np.union1d(inside, near).astype(np.int64)


def seg_within_clamped(px, py, ax, ay, bx, by, r) -> bool:
    """The same test written another way (for pins): the squared distance to
    the nearest point a + s (b - a), s = clamp(t / L, 0, 1), in rationals."""
    P = (Fraction(px), Fraction(py))
    A = (Fraction(ax), Fraction(ay))
    B = (Fraction(bx), Fraction(by))
    ex, ey = B[0] - A[0], B[1] - A[1]
    L = ex * ex + ey * ey
    s = Fraction(0) if L == 0 else min(Fraction(1), max(Fraction(0), ((P[0] - A[0]) * ex + (P[1] - A[1]) * ey) / L))
    qx, qy = A[0] + s * ex, A[1] + s * ey
    return (P[0] - qx) ** 2 + (P[1] - qy) ** 2 <= Fraction(r) * Fraction(r)


def distance_join_lines(x, y, lines, r):
    """Distance join of the points with a set of lines (Sec. 5.2, types (1)
    and (2)): (point ids, line ids) int64, ascending by (point, line), of
    every point within distance r[j] (or the scalar r) of line j, ring j of
    the CSR set as an open polyline.  One exact selection per line."""
    rvo = np.asarray(lines["ring_vtx_off"], dtype=np.int64)
    nl = rvo.size - 1
    rr = np.broadcast_to(np.asarray(r, dtype=np.float64), (nl,))
    pts, lns = [], []
    for j in range(nl):
        one = {"ring_vtx_off": np.array([0, rvo[j + 1] - rvo[j]]),
               "vx": np.asarray(lines["vx"])[rvo[j]:rvo[j + 1]], "vy": np.asarray(lines["vy"])[rvo[j]:rvo[j + 1]]}
        ids = select_near_lines(x, y, one, float(rr[j]))
        pts.append(ids)
        lns.append(np.full(ids.size, j, dtype=np.int64))
    if not pts:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    p = np.concatenate(pts)
    q = np.concatenate(lns)
    order = np.lexsort((q, p))
    return p[order], q[order]


def distance_join_lines_count(x, y, lines, r):
    _, q = distance_join_lines(x, y, lines, r)
    return np.bincount(q, minlength=np.asarray(lines["ring_vtx_off"]).size - 1).astype(np.uint64)
