"""GPU parity of the distance selections from lines (rounded rectangles
around segments) and from a polygon (the polygon with its edges' rounded
rectangles) against the exact CPU oracle, element by element: road-like
polylines over clustered points, points placed at exactly distance r from
segments and just beyond, degenerate geometry, the capacity protocol and
invalid input."""
import numpy as np
import pytest
import torch

from oracle import buffer as B
from oracle import disk as D
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M
E = 2.0 ** -30


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _ids(t):
    return t.cpu().numpy().astype(np.int64)


def _lines(rings):
    return gen.polys_from_rings([[np.asarray(r, dtype=np.float64)] for r in rings])


@pytest.fixture(scope="module")
def pts():
    x, y = gen.mixture_points(300_000, seed=41, L=L)
    return x, y


@pytest.fixture(scope="module")
def roads():
    return gen.road_lines(40, 60, 400.0, seed=42, L=L)


def _on_circle_points(lines, r, rng, n):
    """Points at distance exactly r from segment interiors (3-4-5 offsets
    along and across segments whose direction is (4, 3) / 5 scaled), plus
    the same moved outwards by a few ulps; the segments are appended."""
    xs, ys, rings = [], [], []
    for k in range(n):
        ax = float(np.round(rng.uniform(5000, L - 5000)))
        ay = float(np.round(rng.uniform(5000, L - 5000)))
        s = float(rng.integers(1, 200))
        bx, by = ax + 4 * s, ay + 3 * s                   # direction (4, 3) / 5, length 5 s
        t = float(rng.integers(1, 4 * int(s))) / 4.0       # along the segment
        # normal (-3, 4) / 5 scaled to r = 5 q: offset (-3 q, 4 q)
        q = r / 5.0
        px, py = ax + 4 * t - 3 * q, ay + 3 * t + 4 * q
        xs += [px, px - 3 * q * E, px + 3 * q * E]
        ys += [py, py + 4 * q * E, py - 4 * q * E]
        rings.append([[ax, ay], [bx, by]])
    return np.array(xs), np.array(ys), rings


@pytest.mark.parametrize("r", [0.0, 25.0, 160.0, 1500.0])
def test_near_lines_matches_oracle(ctx, pts, roads, r):
    x, y = pts
    rng = np.random.default_rng(43)
    ex, ey, extra = _on_circle_points(roads, max(r, 40.0), rng, 30) if r > 0 else (np.zeros(0), np.zeros(0), [])
    lines = gen.concat_polys(roads, _lines(extra)) if extra else roads
    xx = np.concatenate([x, ex, [np.nan, 1.0]])
    yy = np.concatenate([y, ey, [2.0, np.inf]])
    got = _ids(ctx.select_near_lines(_dev(xx), _dev(yy), lines, r))
    want = B.select_near_lines(xx, yy, lines, r)
    assert np.array_equal(got, want)
    if r > 0:
        assert want.size > 100
        # the exact-distance points are in, the ones moved outwards are not
        base = x.size
        inn = set(want.tolist())
        assert all(base + 3 * k in inn for k in range(len(extra)) if r >= 40.0)


def test_point_rings_equal_disk_selection(ctx, pts):
    x, y = pts
    c = (float(np.round(x[7])), float(np.round(y[7])))
    lines = _lines([[c]])
    for r in (0.0, 300.0, 2500.0):
        got = _ids(ctx.select_near_lines(_dev(x), _dev(y), lines, r))
        assert np.array_equal(got, D.select_disk(x, y, c[0], c[1], r))
        assert np.array_equal(got, _ids(ctx.select_disk(_dev(x), _dev(y), c[0], c[1], r)))


@pytest.mark.parametrize("r", [0.0, 60.0, 900.0])
def test_within_polygon_matches_oracle(ctx, pts, r):
    x, y = pts
    star = gen.star_polygon(400, 0.02, (L * 0.45, L * 0.55), L=L, seed=44)
    # a polygon with a hole: the star with a smaller star inside, reversed
    hole = gen.star_polygon(60, 0.002, (L * 0.45, L * 0.55), L=L, seed=45)
    holed = gen.polys_from_rings([[np.stack([star["vx"], star["vy"]], 1),
                                   np.stack([hole["vx"][::-1], hole["vy"][::-1]], 1)]])
    for poly in (star, holed):
        got = _ids(ctx.select_within(_dev(x), _dev(y), poly, r))
        want = B.select_within_polygon(x, y, poly, r)
        assert np.array_equal(got, want)
        inside = _ids(ctx.select(_dev(x), _dev(y), poly))
        assert np.isin(inside, got).all()


def test_resolutions_agree(ctx, pts):
    """The polygon part comes from the canvas: the result must not depend on
    its resolution."""
    x, y = pts
    star = gen.star_polygon(300, 0.03, (L * 0.5, L * 0.5), L=L, seed=46)
    want = B.select_within_polygon(x, y, star, 120.0)
    old = ctx.pixels_per_vertex()
    try:
        for ppv in (2.0, 64.0, 2000.0):
            ctx.set_pixels_per_vertex(ppv)
            assert np.array_equal(_ids(ctx.select_within(_dev(x), _dev(y), star, 120.0)), want), ppv
    finally:
        ctx.set_pixels_per_vertex(old)


def test_capacity_and_degenerate(ctx, pts, roads):
    from paper_2203_14362_amd import SpadeError
    x, y = pts
    full = _ids(ctx.select_near_lines(_dev(x), _dev(y), roads, 200.0))
    small = _ids(ctx.select_near_lines(_dev(x), _dev(y), roads, 200.0, cap=7))   # retried with the total
    assert np.array_equal(full, small)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert ctx.select_near_lines(e, e, roads, 200.0).numel() == 0
    # zero-length segments (repeated vertices) and an empty ring
    odd = gen.polys_from_rings([[np.array([[1000.0, 1000.0], [1000.0, 1000.0], [3000.0, 1000.0]])],
                                [np.zeros((0, 2))]])
    got = _ids(ctx.select_near_lines(_dev(x), _dev(y), odd, 500.0))
    assert np.array_equal(got, B.select_near_lines(x, y, odd, 500.0))
    with pytest.raises(SpadeError):
        ctx.select_near_lines(_dev(x), _dev(y), roads, -1.0)
    with pytest.raises(SpadeError):
        ctx.select_near_lines(_dev(x), _dev(y), roads, float("nan"))
    bad = dict(roads)
    bad["vx"] = roads["vx"].copy()
    bad["vx"][5] = np.nan
    with pytest.raises(SpadeError):
        ctx.select_near_lines(_dev(x), _dev(y), bad, 10.0)
    two = gen.concat_polys(gen.star_polygon(10, 0.01, (L / 3, L / 3), L=L), gen.star_polygon(10, 0.01, (L / 2, L / 2), L=L))
    with pytest.raises(SpadeError):
        ctx.select_within(_dev(x), _dev(y), two, 10.0)


@pytest.mark.parametrize("r", [30.0, 400.0])
def test_offset_frame(ctx, pts, roads, r):
    """Web-Mercator-sized coordinates (+(-8.27e6, 4.94e6) m): the differences
    of large coordinates are where the FP64 filters give way to the exact
    expansions."""
    x, y = pts
    ox, oy, lines = gen.offset_frame(x, y, roads, L=L)
    got = _ids(ctx.select_near_lines(_dev(ox), _dev(oy), lines, r))
    assert np.array_equal(got, B.select_near_lines(ox, oy, lines, r))
    star = gen.star_polygon(500, 0.01, (L * 0.55, L * 0.45), L=L, seed=47)
    sx, sy, sp = gen.offset_frame(x, y, star, L=L)
    got = _ids(ctx.select_within(_dev(sx), _dev(sy), sp, r))
    assert np.array_equal(got, B.select_within_polygon(sx, sy, sp, r))
