"""Pins of the distance-selection oracle (closed disk, exact on FP64 inputs).

The pins do not use the oracle's own arithmetic: integer lattices are decided
with Python integers, and FP64 inputs near the circle with their exact
integer ratios (``float.as_integer_ratio``)."""
import math

import numpy as np
import pytest

from oracle import disk


def _by_ratios(x, y, cx, cy, r):
    """Exact decision from the integer ratios of the FP64 values (their
    denominators are powers of two): scale everything to one denominator."""
    out = []
    vals = [v.as_integer_ratio() for v in (cx, cy, r)]
    for i, (xi, yi) in enumerate(zip(x.tolist(), y.tolist())):
        if not (math.isfinite(xi) and math.isfinite(yi)):
            continue
        q = [xi.as_integer_ratio(), yi.as_integer_ratio()] + vals
        D = max(d for _, d in q)
        (nx, _), (ny, _), (ncx, _), (ncy, _), (nr, _) = [(n * (D // d), D) for n, d in q]
        if (nx - ncx) ** 2 + (ny - ncy) ** 2 <= nr * nr:
            out.append(i)
    return np.array(out, dtype=np.int64)


def test_integer_lattice_including_points_on_the_circle():
    g = np.arange(-12, 13, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    for (cx, cy, r) in [(0.0, 0.0, 5.0), (1.0, -2.0, 10.0), (3.0, 3.0, 0.0), (0.0, 0.0, 12.0)]:
        want = [i for i in range(x.size)
                if (int(x[i]) - int(cx)) ** 2 + (int(y[i]) - int(cy)) ** 2 <= int(r) ** 2]
        assert np.array_equal(disk.select_disk(x, y, cx, cy, r), want)
        assert np.array_equal(disk.select_disk_exact(x, y, cx, cy, r), want)
    # the 3-4-5 points lie on the circle of radius 5 and are inside (closed disk)
    on = disk.select_disk(np.array([3.0, 4.0, -3.0, 5.0, 5.0]), np.array([4.0, 3.0, -4.0, 0.0, 1e-300]),
                          0.0, 0.0, 5.0)
    assert on.tolist() == [0, 1, 2, 3]


def test_points_near_the_circle_match_integer_ratios():
    rng = np.random.default_rng(5)
    cx, cy, r = 0.1, -0.7, 0.3
    th = rng.uniform(0, 2 * np.pi, 4000)
    # points rounded onto and one ulp around the circle
    x = cx + r * np.cos(th)
    y = cy + r * np.sin(th)
    x = np.concatenate([x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf)])
    y = np.concatenate([y, y, y])
    got = disk.select_disk(x, y, cx, cy, r)
    assert np.array_equal(got, _by_ratios(x, y, cx, cy, r))
    # both outcomes occur, so the test separates a dropped term or a wrong sign
    assert 0 < got.size < x.size


def test_plain_fp64_would_be_wrong_somewhere_near_the_circle():
    """Some near-circle points are decided differently by a naive FP64
    evaluation: the oracle follows the exact ratios there."""
    rng = np.random.default_rng(6)
    cx, cy, r = 0.1, 0.2, 0.7
    th = rng.uniform(0, 2 * np.pi, 20000)
    x = cx + r * np.cos(th)
    y = cy + r * np.sin(th)
    naive = np.nonzero((x - cx) ** 2 + (y - cy) ** 2 <= r * r)[0]
    exact = _by_ratios(x, y, cx, cy, r)
    assert not np.array_equal(naive, exact)
    assert np.array_equal(disk.select_disk(x, y, cx, cy, r), exact)


def test_non_finite_points_and_degenerate_disks():
    x = np.array([0.0, np.nan, np.inf, 1.0, -np.inf, 0.0])
    y = np.array([0.0, 0.0, 0.0, 0.0, 1.0, np.nan])
    assert disk.select_disk(x, y, 0.0, 0.0, 1.0).tolist() == [0, 3]
    assert disk.select_disk(x, y, 0.0, 0.0, 0.0).tolist() == [0]
    assert disk.select_disk(x[:0], y[:0], 0.0, 0.0, 1.0).size == 0
    with pytest.raises(ValueError):
        disk.select_disk(x, y, 0.0, 0.0, -1.0)
    with pytest.raises(ValueError):
        disk.select_disk(x, y, np.nan, 0.0, 1.0)


def test_tiny_and_huge_scales_are_decided_exactly():
    # squares near the subnormal range and beyond the FP64 range
    x = np.array([3e-160, 4e-160, 1e200, 3e200])
    y = np.array([4e-160, 3e-160, 0.0, 4e200])
    assert np.array_equal(disk.select_disk(x, y, 0.0, 0.0, 5e-160), _by_ratios(x, y, 0.0, 0.0, 5e-160))
    assert np.array_equal(disk.select_disk(x, y, 0.0, 0.0, 5e200), _by_ratios(x, y, 0.0, 0.0, 5e200))


# ------------------------------------------------ distance joins and kNN

def _lattice(m):
    g = np.arange(-m, m + 1, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    return X.ravel(), Y.ravel()


def test_distance_join_gauss_circle_counts():
    """Disks centred on lattice points with integer radii: each count is the
    number of integer points (a, b) with a^2 + b^2 <= r^2 (the Gauss circle
    numbers 1, 5, 13, 29, 49, 81, ... when the disk lies inside the lattice),
    and the pairs are exactly those decided with Python integers."""
    x, y = _lattice(20)
    cx = np.array([0.0, 3.0, -5.0, 7.0, 0.0])
    cy = np.array([0.0, -2.0, 4.0, 7.0, 0.0])
    r = np.array([5.0, 7.0, 0.0, 3.0, 1.0])
    pt, dk = disk.distance_join(x, y, cx, cy, r)
    want = sorted((i, j) for j in range(cx.size) for i in range(x.size)
                  if (int(x[i]) - int(cx[j])) ** 2 + (int(y[i]) - int(cy[j])) ** 2 <= int(r[j]) ** 2)
    assert list(zip(pt.tolist(), dk.tolist())) == want
    counts = disk.distance_join_count(x, y, cx, cy, r)
    assert counts.tolist() == [81, 149, 1, 29, 5]
    # type (1): one radius for every disk
    c1 = disk.distance_join_count(x, y, cx, cy, 4.0)
    assert c1.tolist() == [49] * 5


def test_knn_lattice_order_and_ties():
    """Lattice points around a lattice centre: distances are square roots of
    integers, so the nearest-first order is the order of the integer
    a^2 + b^2, equal values by ascending id."""
    x, y = _lattice(15)
    for (px, py, k) in [(0.0, 0.0, 1), (0.0, 0.0, 37), (2.0, -3.0, 200), (15.0, 15.0, 961)]:
        key = sorted(((int(x[i]) - int(px)) ** 2 + (int(y[i]) - int(py)) ** 2, i) for i in range(x.size))
        want = [i for _, i in key[:k]]
        assert disk.knn(x, y, px, py, k).tolist() == want


def test_knn_one_ulp_apart_and_non_finite():
    """Two points one ulp apart in distance are ordered by the exact
    distance, not by FP64 rounding; non-finite points are never chosen;
    k beyond the finite points returns them all."""
    px, py = 0.1, 0.2
    d = 0.3
    a = (px + d, py)
    b = (np.nextafter(px + d, np.inf), py)
    x = np.array([b[0], a[0], np.nan, px - d, np.inf])
    y = np.array([b[1], a[1], 0.0, py, 0.0])
    got = disk.knn(x, y, px, py, 10)
    from fractions import Fraction
    key = sorted(((Fraction(float(x[i])) - Fraction(px)) ** 2 + (Fraction(float(y[i])) - Fraction(py)) ** 2, i)
                 for i in (0, 1, 3))
    assert [i for _, i in key][1:] == [1, 0]      # a is nearer than b by one ulp
    assert got.tolist() == [i for _, i in key]
