"""CPU oracle for distance selection from a point, distance joins and kNN.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this; the product path never does.

Distance selection (Sec. 4.2, canvases for distance-based queries; Sec. 5.2,
distance-based queries) keeps the points whose Euclidean distance to a centre
is at most r.  The distance join of types (1) and (2) (Sec. 5.2) is the
collection of such selections, one per disk; the kNN selection (Sec. 5.2)
returns the k points of smallest exact distance, equal distances ordered by
id.  The decision is made in exact rational arithmetic on the FP64
inputs: (x - cx)^2 + (y - cy)^2 <= r^2.  Points with a non-finite coordinate
are outside.

For speed on large inputs a point is first classified with numpy in FP64; only
points whose FP64 value of r^2 - (x-cx)^2 - (y-cy)^2 lies within a generous
margin of zero (1e-9 of the sum of the three squares, far above the few ulps
that evaluation can be off by), or whose squares overflow or come near the
subnormal range, are decided again with ``fractions.Fraction``.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

MARGIN = 1e-9


def _exact_inside(xi: float, yi: float, cx: float, cy: float, r: float) -> bool:
    dx = Fraction(xi) - Fraction(cx)
    dy = Fraction(yi) - Fraction(cy)
    return dx * dx + dy * dy <= Fraction(r) * Fraction(r)


def select_disk(x, y, cx: float, cy: float, r: float) -> np.ndarray:
    """Ascending ids (int64) of the points within distance r of (cx, cy)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if not (math.isfinite(cx) and math.isfinite(cy) and math.isfinite(r) and r >= 0):
        raise ValueError("centre and radius must be finite, radius >= 0")
    finite = np.isfinite(x) & np.isfinite(y)
    with np.errstate(over="ignore", invalid="ignore"):
        dx = x - cx
        dy = y - cy
        sq = dx * dx + dy * dy
        s = r * r - sq
        scale = r * r + sq
    # tiny scales (squares near or below the subnormal range) and overflowed
    # ones are always decided exactly
    normal = (scale > 1e-280) & np.isfinite(scale)
    inside = finite & normal & (s > MARGIN * scale)
    decided = normal & ((s > MARGIN * scale) | (-s > MARGIN * scale))
    unsure = np.nonzero(finite & ~decided)[0]
    for i in unsure.tolist():
        inside[i] = _exact_inside(float(x[i]), float(y[i]), cx, cy, r)
    return np.nonzero(inside)[0].astype(np.int64)


def select_disk_exact(x, y, cx: float, cy: float, r: float) -> np.ndarray:
    """Every point decided in rational arithmetic (small inputs only)."""
    out = [i for i, (xi, yi) in enumerate(zip(np.asarray(x, dtype=np.float64).tolist(),
                                               np.asarray(y, dtype=np.float64).tolist()))
           if math.isfinite(xi) and math.isfinite(yi) and _exact_inside(xi, yi, cx, cy, r)]
    return np.array(out, dtype=np.int64)


def distance_join(x, y, cx, cy, r):
    """(point ids, disk ids) int64, ascending by (point, disk), of every
    point within distance r[j] (or the scalar r) of centre j: one exact
    selection per disk."""
    cx = np.asarray(cx, dtype=np.float64)
    cy = np.asarray(cy, dtype=np.float64)
    rr = np.broadcast_to(np.asarray(r, dtype=np.float64), cx.shape)
    pts, dks = [], []
    for j in range(cx.size):
        ids = select_disk(x, y, float(cx[j]), float(cy[j]), float(rr[j]))
        pts.append(ids)
        dks.append(np.full(ids.size, j, dtype=np.int64))
    if not pts:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    p = np.concatenate(pts)
    d = np.concatenate(dks)
    order = np.lexsort((d, p))
    return p[order], d[order]


def distance_join_count(x, y, cx, cy, r):
    _, d = distance_join(x, y, cx, cy, r)
    return np.bincount(d, minlength=np.asarray(cx).size).astype(np.uint64)


def _exact_d2(xi, yi, px, py):
    dx = Fraction(xi) - Fraction(px)
    dy = Fraction(yi) - Fraction(py)
    return dx * dx + dy * dy


def knn(x, y, px: float, py: float, k: int) -> np.ndarray:
    """Ids (int64) of the k points nearest to (px, py) by exact distance,
    nearest first, equal distances by ascending id; points with a non-finite
    coordinate are never chosen.  FP64 squared distances shortlist the
    candidates (everything within a relative margin of the k-th one), whose
    order is then decided in rational arithmetic."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    fin = np.nonzero(np.isfinite(x) & np.isfinite(y))[0]
    k = min(int(k), fin.size)
    if k <= 0:
        return np.zeros(0, np.int64)
    with np.errstate(over="ignore"):
        d2 = (x[fin] - px) ** 2 + (y[fin] - py) ** 2
    kth = np.partition(d2, k - 1)[k - 1]
    cut = kth * (1 + 1e-9) + 1e-300
    cand = fin[d2 <= cut]
    keyed = sorted(((_exact_d2(float(x[i]), float(y[i]), px, py), int(i)) for i in cand.tolist()))
    return np.array([i for _, i in keyed[:k]], dtype=np.int64)
