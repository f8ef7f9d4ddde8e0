"""Pins of the line-buffer / buffered-polygon distance oracle (oracle/buffer.py)
against closed forms, an independent formulation (nearest point by clamped
projection, in rationals), the disk oracle for point segments, and the
invariances the definition has (reversal, splitting, monotonicity in r)."""
import numpy as np

from oracle import buffer as B
from oracle import disk as D

E = 2.0 ** -40


def _one(px, py, seg, r):
    ax, ay, bx, by = seg
    return B.select_near_segments(np.array([px]), np.array([py]), [ax], [ay], [bx], [by], r).size == 1


def test_closed_forms_axis_segment():
    seg = (0.0, 0.0, 8.0, 0.0)
    r = 5 / 8
    assert _one(4.0, r, seg, r) and _one(4.0, -r, seg, r)              # perpendicular, exactly r
    assert not _one(4.0, r + E, seg, r) and not _one(4.0, -r - E, seg, r)
    assert _one(8 + 3 / 8, 0.5, seg, r)                                  # |p - b| = 5/8 exactly
    assert not _one(8 + 3 / 8, 0.5 + E, seg, r)
    assert _one(-3 / 8, -0.5, seg, r) and not _one(-3 / 8 - E, -0.5, seg, r)   # around a
    assert _one(0.0, r, seg, r) and not _one(0.0, r + E, seg, r)         # t == 0 exactly
    assert _one(8.0, -r, seg, r) and not _one(8.0, -r - E, seg, r)       # t == L exactly
    assert _one(4.0, 0.0, seg, 0.0) and not _one(4.0, E, seg, 0.0)       # r = 0: the segment itself


def test_closed_forms_diagonal_segment():
    # length 10, unit normal (-3/5, 4/5): (4, 3) + 5 * normal = (1, 7) is at distance 5
    seg = (0.0, 0.0, 8.0, 6.0)
    assert _one(1.0, 7.0, seg, 5.0) and _one(7.0, -1.0, seg, 5.0)
    assert not _one(1.0, 7.0 + 1e-9, seg, 5.0) and not _one(7.0 + 1e-9, -1.0, seg, 5.0)
    assert _one(1.0 + 1e-9, 7.0, seg, 5.0)                               # inwards along x


def _random_cases(rng, n, grid):
    out = []
    for it in range(n):
        ax, ay, bx, by = (rng.integers(-grid, grid, 4) / 8.0).tolist()
        if it % 9 == 0:
            bx, by = ax, ay
        r = float(rng.integers(0, grid)) / 8.0
        px, py = (rng.integers(-2 * grid, 2 * grid, 2) / 8.0).tolist()
        out.append((px, py, ax, ay, bx, by, r))
    return out


def test_definition_against_clamped_projection():
    rng = np.random.default_rng(7)
    cases = _random_cases(rng, 4000, 24)
    # off-grid points and radii too
    for _ in range(1000):
        ax, ay, bx, by, px, py = rng.uniform(-3, 3, 6).tolist()
        cases.append((px, py, ax, ay, bx, by, float(rng.uniform(0, 2))))
    for c in cases:
        assert B.seg_within_exact(*c) == B.seg_within_clamped(*c), c


def test_fp64_filter_matches_exact_decisions():
    rng = np.random.default_rng(8)
    cases = _random_cases(rng, 3000, 16)
    # points placed at distance exactly r (Pythagorean offsets) and one ulp-ish off
    for _ in range(600):
        ax, ay = (rng.integers(-64, 64, 2) / 4.0).tolist()
        bx, by = ax + 8.0, ay + 6.0                       # normal (-3/5, 4/5) * 5 = (-3, 4)
        s = float(rng.integers(0, 9)) / 8.0
        px, py = ax + 8.0 * s - 3.0, ay + 6.0 * s + 4.0
        for d in (0.0, E, -E):
            cases.append((px, py + d, ax, ay, bx, by, 5.0))
    got = np.array([bool(B._pairs_within(np.array([c[0]]), np.array([c[1]]), *c[2:6], c[6])[0]) for c in cases])
    want = np.array([B.seg_within_exact(*c) for c in cases])
    assert np.array_equal(got, want)
    assert want.sum() > 300 and (~want).sum() > 300


def test_point_segments_equal_disk_oracle():
    rng = np.random.default_rng(9)
    x = rng.uniform(-10, 10, 30000)
    y = rng.uniform(-10, 10, 30000)
    # points on the circle of radius 5 around (1, 2): (1 +- 3, 2 +- 4), (1 +- 5, 2)
    ring = [(4.0, 6.0), (-2.0, -2.0), (6.0, 2.0), (1.0, -3.0)]
    x = np.concatenate([x, [p[0] for p in ring], [np.nan]])
    y = np.concatenate([y, [p[1] for p in ring], [0.0]])
    got = B.select_near_segments(x, y, [1.0], [2.0], [1.0], [2.0], 5.0)
    want = D.select_disk(x, y, 1.0, 2.0, 5.0)
    assert np.array_equal(got, want)
    assert set(range(30000, 30004)) <= set(got.tolist())


def test_reversal_splitting_and_monotonicity():
    rng = np.random.default_rng(10)
    x = rng.uniform(-20, 20, 50000)
    y = rng.uniform(-20, 20, 50000)
    ax, ay, bx, by = -12.5, 3.25, 9.75, -6.5
    mx, my = (ax + bx) / 2, (ay + by) / 2              # exact: dyadic endpoints
    r = 2.5
    whole = B.select_near_segments(x, y, [ax], [ay], [bx], [by], r)
    rev = B.select_near_segments(x, y, [bx], [by], [ax], [ay], r)
    split = B.select_near_segments(x, y, [ax, mx], [ay, my], [mx, bx], [my, by], r)
    assert np.array_equal(whole, rev) and np.array_equal(whole, split)
    smaller = B.select_near_segments(x, y, [ax], [ay], [bx], [by], 1.0)
    assert np.isin(smaller, whole).all() and smaller.size < whole.size


def test_lines_and_polygon_composition():
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 10, 40000)
    y = rng.uniform(0, 10, 40000)
    # a square ring with a vertex exactly on a sample point
    sq = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, 4]),
          "vx": np.array([2.0, 8.0, 8.0, 2.0]), "vy": np.array([2.0, 2.0, 8.0, 8.0])}
    x[0], y[0] = 2.0, 5.0        # on the left edge
    x[1], y[1] = 1.5, 5.0        # 0.5 left of it
    x[2], y[2] = 5.0, 5.0        # inside, far from the edges
    lines_open = B.select_near_lines(x, y, sq, 0.5)          # three edges, no closing one
    poly = B.select_within_polygon(x, y, sq, 0.5)
    got_in = np.zeros(x.size, bool)
    got_in[poly] = True
    assert got_in[0] and got_in[1] and got_in[2]
    # the square's 0.5-buffer: every point of the square is kept, nothing
    # outside the square widened by 0.5, and of the band around it exactly
    # the points within 0.5 of the nearest corner where both coordinates
    # leave the square
    strict = (x > 2) & (x < 8) & (y > 2) & (y < 8)
    assert got_in[strict].all() and not got_in[~((x >= 1.5) & (x <= 8.5) & (y >= 1.5) & (y <= 8.5))].any()
    ddx = np.maximum(np.maximum(2 - x, x - 8), 0)
    ddy = np.maximum(np.maximum(2 - y, y - 8), 0)
    d2 = ddx * ddx + ddy * ddy
    clear = np.abs(d2 - 0.25) > 1e-9
    assert np.array_equal(got_in[clear], (d2 <= 0.25)[clear])
    # the open polyline lacks the closing edge (2,8)-(2,2): x[1] is near it only
    lo = np.zeros(x.size, bool)
    lo[lines_open] = True
    assert not lo[1] and not lo[2]
    assert np.isin(lines_open, poly).all()
    # r = 0 keeps the points on the boundary and inside
    zero = np.zeros(x.size, bool)
    zero[B.select_within_polygon(x, y, sq, 0.0)] = True
    assert zero[0] and zero[2] and not zero[1]


def test_line_join_pins():
    """The line join against the disk join (point lines), the line selection
    (one line), and type (2) with equal radii against type (1)."""
    rng = np.random.default_rng(12)
    x = rng.uniform(0, 50, 20000)
    y = rng.uniform(0, 50, 20000)
    cx, cy = rng.uniform(0, 50, 30), rng.uniform(0, 50, 30)
    pts_lines = {"ring_vtx_off": np.arange(31), "vx": cx, "vy": cy}
    a = B.distance_join_lines(x, y, pts_lines, 2.5)
    b = D.distance_join(x, y, cx, cy, 2.5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rad = rng.uniform(0.5, 4.0, 30)
    a = B.distance_join_lines(x, y, pts_lines, rad)
    b = D.distance_join(x, y, cx, cy, rad)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    line = {"ring_vtx_off": np.array([0, 4]), "vx": np.array([1.0, 20.0, 30.0, 45.0]),
            "vy": np.array([1.0, 30.0, 5.0, 40.0])}
    p, q = B.distance_join_lines(x, y, line, 1.5)
    assert np.array_equal(p, B.select_near_lines(x, y, line, 1.5)) and (q == 0).all()
    lines = gen_lines(rng)
    a = B.distance_join_lines(x, y, lines, 1.0)
    b = B.distance_join_lines(x, y, lines, np.full(lines["ring_vtx_off"].size - 1, 1.0))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = B.distance_join_lines_count(x, y, lines, 1.0)
    assert c.sum() == a[0].size and (np.diff(a[0]) >= 0).all()


def gen_lines(rng):
    rings, off = [], [0]
    for k in range(12):
        n = int(rng.integers(1, 6))
        rings.append(rng.uniform(0, 50, (n, 2)))
        off.append(off[-1] + n)
    v = np.concatenate(rings)
    return {"ring_vtx_off": np.array(off), "vx": v[:, 0], "vy": v[:, 1]}
