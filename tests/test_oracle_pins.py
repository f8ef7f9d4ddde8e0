"""Pins of the CPU oracle against facts other than itself (no GPU).

Each test fixes the oracle to something the mathematics or the paper
determines independently of oracle.c: closed-form lattice counts, exact
rational arithmetic via ``fractions``, invariants of the crossing-number
definition, tessellation coverage (every point of the extent in exactly one
cell) and brute force on tiny inputs.  The half-open rule (a boundary point
belongs to the polygon on its +x side, or above a horizontal edge) is the
reading of the paper's intersection predicate used throughout.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import micro
from workloads import gen


# ------------------------------------------------------------ exact orientation

def _frac_orient(a, b, c):
    ax, ay, bx, by, cx, cy = (Fraction(v) for v in (*a, *b, *c))
    d = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    return (d > 0) - (d < 0)


def _adversarial_triples(seed=11, n=3000):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        kind = rng.integers(0, 6)
        a = rng.uniform(-1e3, 1e3, 2)
        b = rng.uniform(-1e3, 1e3, 2)
        if kind == 0:                      # random
            c = rng.uniform(-1e3, 1e3, 2)
        elif kind == 1:                    # exactly collinear dyadic
            a = rng.integers(-2 ** 20, 2 ** 20, 2) / 1024.0
            d = rng.integers(-2 ** 10, 2 ** 10, 2) / 1024.0
            b = a + d
            c = a + rng.integers(-8, 8) * d
        elif kind == 2:                    # rounded collinear: tiny true determinant
            t = rng.uniform(-2, 2)
            c = a + t * (b - a)
        elif kind == 3:                    # one ulp off a collinear point
            t = rng.integers(-4, 5) / 4.0
            c = a + t * (b - a)
            c = np.array([np.nextafter(c[0], np.inf), c[1]])
        elif kind == 4:                    # large offsets, Web-Mercator-like frame
            off = np.array([-8.27e6, 4.94e6])
            a, b = a + off, b + off
            t = rng.uniform(-1, 2)
            c = a + t * (b - a)
        else:                              # horizontal / vertical / coincident
            c = np.array([a[0] + rng.uniform(-5, 5), a[1]])
            b = np.array([b[0], a[1]]) if rng.random() < 0.5 else a.copy()
        out.append((tuple(map(float, a)), tuple(map(float, b)), tuple(map(float, c))))
    return out


def test_orient_matches_exact_rationals():
    trip = _adversarial_triples()
    zeros = 0
    for a, b, c in trip:
        want = _frac_orient(a, b, c)
        zeros += want == 0
        assert oracle.orient_sign(*a, *b, *c) == want, (a, b, c)
    assert zeros > 300            # the degenerate branch is exercised


def test_orient_bigint_path_alone():
    """The big-integer fallback by itself (filter disabled) is exact."""
    oracle.set_filter(False)
    try:
        for a, b, c in _adversarial_triples(seed=12, n=2000):
            assert oracle.orient_sign(*a, *b, *c) == _frac_orient(a, b, c)
        # extreme exponents inside the exactness domain
        rng = np.random.default_rng(3)
        for _ in range(300):
            e = rng.integers(-400, 400)
            a = tuple(float(v) * 2.0 ** e for v in rng.uniform(-1, 1, 2))
            b = tuple(float(v) * 2.0 ** (e + rng.integers(-60, 60)) for v in rng.uniform(-1, 1, 2))
            c = tuple(float(v) * 2.0 ** (e - rng.integers(0, 60)) for v in rng.uniform(-1, 1, 2))
            assert oracle.orient_sign(*a, *b, *c) == _frac_orient(a, b, c)
    finally:
        oracle.set_filter(True)


def test_orient_symmetries():
    rng = np.random.default_rng(5)
    for _ in range(500):
        a, b, c = (tuple(rng.integers(-50, 50, 2) / 8.0) for _ in range(3))
        s = oracle.orient_sign(*a, *b, *c)
        assert oracle.orient_sign(*b, *a, *c) == -s           # swap -> sign flip
        assert oracle.orient_sign(*b, *c, *a) == s            # cyclic rotation
        assert oracle.orient_sign(*c, *a, *b) == s


# ------------------------------------------------------------ closed forms

def _half_open_count(lo, hi, h, n, x0):
    """#{i in [0,n): lo <= x0 + i h < hi} for dyadic inputs (exact)."""
    i = np.arange(n)
    v = x0 + i * h
    return int(((v >= lo) & (v < hi)).sum())


def test_lattice_rectangles_closed_form():
    h = 2.0 ** -8
    nx = ny = 300
    x0 = y0 = -10 * h
    x, y = gen.lattice_points(nx, ny, h, x0, y0)
    rng = np.random.default_rng(21)
    rects = []
    for _ in range(12):
        a, b = sorted(rng.integers(-5, 280, 2))
        c, d = sorted(rng.integers(-5, 280, 2))
        b, d = b + 1, d + 1
        rects.append((a * h, b * h, c * h, d * h))
    polys = gen.polys_from_rings([[np.array([[a, c], [b, c], [b, d], [a, d]])] for a, b, c, d in rects])
    got = oracle.join_count(x, y, polys)
    for k, (a, b, c, d) in enumerate(rects):
        want = _half_open_count(a, b, h, nx, x0) * _half_open_count(c, d, h, ny, y0)
        assert int(got[k]) == want


def test_rect_grid_tessellation_closed_form():
    h = 2.0 ** -6
    x, y = gen.lattice_points(140, 140, h, x0=-3 * h, y0=-3 * h)
    polys = gen.rect_grid(4, 4, 0.0, 0.0, 0.5, 0.5)
    got = oracle.join_count(x, y, polys)
    assert got.tolist() == [32 * 32] * 16
    nm = oracle.point_nmatch(x, y, polys)
    inside = (x >= 0) & (x < 2) & (y >= 0) & (y < 2)
    assert np.array_equal(nm, inside.astype(np.int32))


@pytest.mark.parametrize("A,B", [(7, 5), (16, 16), (13, 29), (40, 3)])
def test_right_triangle_closed_form(A, B):
    """Triangle (0,0),(A,0),(0,B) over integer lattice points: the half-open
    rule keeps the two legs and drops the hypotenuse, so the count is
    #{(i,j) >= 0 : B i + A j < A B}."""
    x, y = gen.lattice_points(A + 3, B + 3, 1.0, x0=-1.0, y0=-1.0)
    polys = gen.right_triangle(float(A), float(B))
    got = int(oracle.join_count(x, y, polys)[0])
    want = sum(max(0, -(-(A * B - B * i) // A)) for i in range(A + 1))
    assert got == want
    # the same triangle scaled by a power of two (exact) over the scaled lattice
    s = 2.0 ** -7
    polys2 = gen.right_triangle(A * s, B * s, 3 * s, -5 * s)
    got2 = int(oracle.join_count(x * s + 3 * s, y * s - 5 * s, polys2)[0])
    assert got2 == want


# ------------------------------------------------------------ tessellations

def test_voronoi_jitter_counts_each_point_once():
    x, y = gen.uniform_points(50_000, seed=1)
    polys = gen.voronoi_jitter(64, 8, 64, seed=1, L=1.0)
    nm = oracle.point_nmatch(x, y, polys)
    assert nm.min() == 1 and nm.max() == 1
    assert int(oracle.join_count(x, y, polys).sum()) == x.size


def test_voronoi_jitter_metre_extent_edges_and_corners():
    """Points exactly on shared vertices, on jittered shared edges and on the
    extent sides are still counted exactly once."""
    L = 60000.0
    polys = gen.voronoi_jitter(40, 20, 60, seed=4, L=L)
    vx, vy = polys["vx"], polys["vy"]
    inside = (vx < L) & (vy < L)
    px = np.concatenate([vx[inside], (vx[inside] + np.roll(vx, 1)[inside]) / 2, [0.0, 0.0, L / 2]])
    py = np.concatenate([vy[inside], (vy[inside] + np.roll(vy, 1)[inside]) / 2, [0.0, L / 2, 0.0]])
    nm = oracle.point_nmatch(px, py, polys)
    assert nm.min() == 1 and nm.max() == 1


# ------------------------------------------------------------ invariants

def _rings_polys(rings_per_poly):
    return gen.polys_from_rings([[np.asarray(r, dtype=float) for r in rr] for rr in rings_per_poly])


def test_hole_invariant():
    x, y = gen.uniform_points(20000, seed=4)
    R = np.array([[0.1, 0.1], [0.9, 0.15], [0.85, 0.9], [0.12, 0.8]])
    P = gen.star_polygon(40, 0.05, (0.5, 0.5), L=1.0, seed=8).copy()
    Pr = np.stack([P["vx"], P["vy"]], 1)
    polys = _rings_polys([[R, Pr], [Pr], [R]])
    c = oracle.join_count(x, y, polys)
    assert int(c[0]) + int(c[1]) == int(c[2])
    assert int(c[1]) > 0


def test_orientation_rotation_permutation_invariance():
    x, y = gen.uniform_points(20000, seed=6)
    polys = gen.voronoi_jitter(12, 6, 30, seed=6, L=1.0)
    base = oracle.join_count(x, y, polys)
    rv = polys["ring_vtx_off"]
    rings = [np.stack([polys["vx"][rv[k]:rv[k + 1]], polys["vy"][rv[k]:rv[k + 1]]], 1) for k in range(12)]
    rev = _rings_polys([[r[::-1]] for r in rings])
    assert np.array_equal(oracle.join_count(x, y, rev), base)
    rot = _rings_polys([[np.roll(r, 3 + k, axis=0)] for k, r in enumerate(rings)])
    assert np.array_equal(oracle.join_count(x, y, rot), base)
    perm = np.random.default_rng(2).permutation(12)
    per = _rings_polys([[rings[p]] for p in perm])
    assert np.array_equal(oracle.join_count(x, y, per), base[perm])


def test_translation_and_scale_invariance():
    """Dyadic grid inputs translated by a dyadic offset or scaled by 2^k stay
    exact, so every count is unchanged."""
    rng = np.random.default_rng(9)
    x = rng.integers(0, 2 ** 12, 20000) / 2.0 ** 12
    y = rng.integers(0, 2 ** 12, 20000) / 2.0 ** 12
    rings = [np.array([[0.125, 0.25], [0.75, 0.125], [0.875, 0.625], [0.5, 0.5], [0.25, 0.875]]),
             np.array([[0.5, 0.0], [1.0, 0.5], [0.5, 1.0], [0.0, 0.5]])]
    polys = _rings_polys([[r] for r in rings])
    base = oracle.join_count(x, y, polys)
    for dx, dy, s in [(1024.0, -2048.0, 1.0), (0.0, 0.0, 2.0 ** 20), (-3.5, 7.25, 2.0 ** -9)]:
        tp = _rings_polys([[r * s + [dx, dy]] for r in rings])
        assert np.array_equal(oracle.join_count(x * s + dx, y * s + dy, tp), base)


def test_degenerate_polygons_and_points():
    x = np.array([0.5, 0.5, np.nan, 0.25, np.inf, 0.5])
    y = np.array([0.5, 0.25, 0.5, np.nan, 0.5, 0.0])
    polys = _rings_polys([
        [[[0.0, 0.0], [1.0, 1.0]]],                         # two vertices
        [[[0.0, 0.0], [1.0, 1.0], [2.0, 2.0]]],             # collinear, zero area
        [[[0.0, 0.5], [1.0, 0.5], [0.5, 0.5]]],             # horizontal, zero area
        [[[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.0, 0.0]]],  # repeated closing vertex
    ])
    c = oracle.join_count(x, y, polys)
    assert c.tolist() == [0, 0, 0, 3]     # NaN / inf points are in no polygon


# ------------------------------------------------------------ brute force

def test_micro_brute_force_agrees():
    for seed in range(4):
        x, y = gen.uniform_points(250, seed=100 + seed)
        polys = gen.voronoi_jitter(5, 4, 10, seed=100 + seed, L=1.0)
        # add points exactly on vertices and edge midpoints
        x = np.concatenate([x, polys["vx"], (polys["vx"] + np.roll(polys["vx"], 1)) / 2])
        y = np.concatenate([y, polys["vy"], (polys["vy"] + np.roll(polys["vy"], 1)) / 2])
        assert oracle.join_count(x, y, polys).tolist() == micro.join_count(x, y, polys)


def test_pairs_select_consistent_with_counts():
    x, y = gen.uniform_points(30000, seed=13)
    polys = gen.voronoi_jitter(20, 8, 40, seed=13, L=1.0)
    counts = oracle.join_count(x, y, polys)
    pt, pg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(np.bincount(pg, minlength=20), counts)
    key = pt.astype(np.uint64) << np.uint64(32) | pg.astype(np.uint64)
    assert np.all(np.diff(key.astype(np.int64)) > 0)
    for k in (0, 7, 19):
        sel = oracle.select(x, y, polys, k)
        assert np.array_equal(sel, pt[pg == k])


def test_area_sanity_statistical():
    """Not an exactness pin: for uniform points the fraction in each cell
    approaches its shoelace area (5-sigma binomial band)."""
    x, y = gen.uniform_points(200_000, seed=17)
    polys, info = gen.voronoi_jitter(30, 10, 40, seed=17, L=1.0, return_info=True)
    c = oracle.join_count(x, y, polys)
    rv = polys["ring_vtx_off"]
    for k in range(30):
        px, py = polys["vx"][rv[k]:rv[k + 1]], polys["vy"][rv[k]:rv[k + 1]]
        area = 0.5 * abs(np.sum(px * np.roll(py, -1) - np.roll(px, -1) * py))
        sd = math.sqrt(x.size * area * (1 - area))
        assert abs(int(c[k]) - x.size * area) < 5 * sd + 1
    assert abs(info["area_sum"] - 1.0) < 1e-12


# ------------------------------------------------ uniform-grid candidate filter
#
# With more than 64 polygons the oracle lists candidates from a uniform grid
# over the polygons' bounding boxes.  Two pins hold it: the tessellation
# property (each point of the half-open extent in exactly one cell, none
# outside), which a dropped candidate would break, and agreement with the
# same oracle with the grid switched off (one cell listing every polygon,
# bounding-box rejects only, which the lattice closed forms above pin).

def _boundary_points(polys, rng, n_mid=200_000):
    """Every vertex of the set plus FP64 midpoints of randomly chosen edges:
    points on or within an ulp of the shared boundaries."""
    vx, vy = polys["vx"], polys["vy"]
    rvo = polys["ring_vtx_off"]
    nxt = np.arange(vx.size) + 1
    nxt[rvo[1:] - 1] = rvo[:-1]          # last vertex of a ring wraps to its first
    e = rng.integers(0, vx.size, min(n_mid, vx.size))
    mx = 0.5 * (vx[e] + vx[nxt[e]])
    my = 0.5 * (vy[e] + vy[nxt[e]])
    return np.concatenate([vx, mx]), np.concatenate([vy, my])


def _check_tessellation_once(x, y, polys, L):
    nm = oracle.point_nmatch(x, y, polys)
    inside_extent = (x >= 0) & (x < L) & (y >= 0) & (y < L)
    assert np.array_equal(nm, inside_extent.astype(np.int32))
    counts = oracle.join_count(x, y, polys)
    assert int(counts.sum()) == int(inside_extent.sum())


def test_grid_filter_tessellation_c2_cells():
    """260 Voronoi-jitter cells (50-500 vertices) over the 60 km extent: the
    grid filter is active and every point, including points on shared
    vertices and edge midpoints, lies in exactly one cell."""
    L = gen.EXTENT_M
    polys = gen.voronoi_jitter(260, 50, 500, seed=2, L=L)
    assert oracle.filter_grid(polys) > 1
    rng = np.random.default_rng(21)
    bx, by = _boundary_points(polys, rng)
    mx, my = gen.mixture_points(300_000, seed=2, L=L)
    x = np.concatenate([bx, mx, rng.uniform(0, L, 50_000)])
    y = np.concatenate([by, my, rng.uniform(0, L, 50_000)])
    _check_tessellation_once(x, y, polys, L)


@pytest.fixture(scope="module")
def census_40k():
    return gen.census_cells(40_000, 4, 40, seed=9, data_seed=4, L=gen.EXTENT_M)


def test_grid_filter_tessellation_40k_census_cells(census_40k):
    """40,000 mixture-seeded census-like cells (4-40 vertices): every point
    (vertices, edge midpoints, clustered and uniform points) in exactly one."""
    L = gen.EXTENT_M
    polys = census_40k
    assert oracle.filter_grid(polys) == 200
    rng = np.random.default_rng(22)
    bx, by = _boundary_points(polys, rng)
    mx, my = gen.mixture_points(300_000, seed=4, L=L)
    x = np.concatenate([bx, mx, rng.uniform(0, L, 100_000)])
    y = np.concatenate([by, my, rng.uniform(0, L, 100_000)])
    _check_tessellation_once(x, y, polys, L)


def _filtered_vs_unfiltered(x, y, polys):
    try:
        oracle.set_grid(True)
        a_counts = oracle.join_count(x, y, polys)
        a_nm = oracle.point_nmatch(x, y, polys)
        a_pt, a_pg = oracle.join_pairs(x, y, polys)
        oracle.set_grid(False)
        assert oracle.filter_grid(polys) == 1
        b_counts = oracle.join_count(x, y, polys)
        b_nm = oracle.point_nmatch(x, y, polys)
        b_pt, b_pg = oracle.join_pairs(x, y, polys)
    finally:
        oracle.set_grid(True)
    assert np.array_equal(a_counts, b_counts)
    assert np.array_equal(a_nm, b_nm)
    assert np.array_equal(a_pt, b_pt) and np.array_equal(a_pg, b_pg)
    return a_counts


def test_grid_filter_matches_unfiltered_overlapping_stars():
    """300 overlapping stars (pairs of points with several polygons): the grid
    lists every candidate the plain bounding-box scan finds."""
    L = gen.EXTENT_M
    stars, _ = gen.query_stars(300, 8, 400, seed=23, L=L, area=(1e-4, 2e-2), data_seed=2)
    assert oracle.filter_grid(stars) > 1
    x, y = gen.mixture_points(20_000, seed=2, L=L)
    rng = np.random.default_rng(24)
    bx, by = _boundary_points(stars, rng, n_mid=5_000)
    counts = _filtered_vs_unfiltered(np.concatenate([x, bx]), np.concatenate([y, by]), stars)
    assert counts.sum() > x.size        # overlaps: points with several polygons


def test_grid_filter_matches_unfiltered_40k(census_40k):
    L = gen.EXTENT_M
    x, y = gen.mixture_points(5_000, seed=4, L=L)
    rng = np.random.default_rng(25)
    bx, by = _boundary_points(census_40k, rng, n_mid=2_000)
    _filtered_vs_unfiltered(np.concatenate([x, bx[:3000]]), np.concatenate([y, by[:3000]]), census_40k)


def test_offset_frame_tessellation():
    """The Web-Mercator-like offset frame keeps the tessellation exact: every
    kept point in exactly one cell (rounded vertices, shared bit-identically)."""
    L = gen.EXTENT_M
    polys = gen.voronoi_jitter(260, 50, 500, seed=2, L=L)
    x, y = gen.mixture_points(200_000, seed=2, L=L)
    rng = np.random.default_rng(26)
    bx, by = _boundary_points(polys, rng, n_mid=50_000)
    ox, oy, opolys = gen.offset_frame(np.concatenate([x, bx]), np.concatenate([y, by]), polys)
    o = gen.WEB_MERCATOR_ORIGIN
    nm = oracle.point_nmatch(ox, oy, opolys)
    assert np.array_equal(nm, np.ones(ox.size, np.int32))
    assert ox.size > 200_000
    assert np.all(ox >= o[0]) and np.all(ox < o[0] + L)
