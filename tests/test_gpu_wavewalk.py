"""GPU parity of the distance queries where the walks balanced over a
wavefront's lanes are stressed: hundreds of segments or disks crowded into
a few grid cells, so that a point has far more than 64 candidates (a point's
share of one round is capped at 64), its candidates span several rounds,
and, in the line join, one line's consecutive segments straddle round
boundaries (the repeated-line check across rounds).  Points are dense
around the crowd and sparse elsewhere, so wavefronts mix long, short and
empty lists.  Compared with the exact CPU oracle element by element."""
import numpy as np
import pytest
import torch

from oracle import buffer as B
from oracle import disk as D
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M
C = (L * 0.5, L * 0.5)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _i64(t):
    return t.cpu().numpy().astype(np.int64)


@pytest.fixture(scope="module")
def pts():
    rng = np.random.default_rng(61)
    x, y = gen.mixture_points(120_000, seed=62, L=L)
    cx = C[0] + rng.uniform(-600.0, 600.0, 80_000)
    cy = C[1] + rng.uniform(-600.0, 600.0, 80_000)
    # shuffled, so that a wavefront holds crowded and sparse points alike
    xx = np.concatenate([x, cx])
    yy = np.concatenate([y, cy])
    perm = rng.permutation(xx.size)
    return xx[perm], yy[perm]


def _zigzags(n_lines, n_vertices, half, seed):
    """Lines that wander inside a square of side 2 half around the centre:
    every central cell lists many segments of every line."""
    rng = np.random.default_rng(seed)
    rings = []
    for _ in range(n_lines):
        v = np.stack([C[0] + rng.uniform(-half, half, n_vertices), C[1] + rng.uniform(-half, half, n_vertices)], 1)
        rings.append([np.round(v * 4.0) / 4.0])
    return gen.polys_from_rings(rings)


@pytest.fixture(scope="module")
def crowd():
    return _zigzags(40, 12, 400.0, seed=63)


@pytest.mark.parametrize("r", [0.0, 15.0, 120.0])
def test_crowded_selection(ctx, pts, crowd, r):
    x, y = pts
    got = _i64(ctx.select_near_lines(_dev(x), _dev(y), crowd, r))
    want = B.select_near_lines(x, y, crowd, r)
    assert np.array_equal(got, want)
    if r > 0:
        assert want.size > 1000


def test_crowded_polygon(ctx, pts):
    x, y = pts
    # spikes from 0.1 R to 1.9 R: near the centre the cells list many edges
    star = gen.star_polygon(3000, 0.0004, C, L=L, seed=64, noise=0.9)
    got = _i64(ctx.select_within(_dev(x), _dev(y), star, 40.0))
    assert np.array_equal(got, B.select_within_polygon(x, y, star, 40.0))


def test_crowded_line_join(ctx, pts, crowd):
    x, y = pts
    rad = np.random.default_rng(65).uniform(5.0, 60.0, crowd["n_polys"])
    p, q = ctx.distance_join_lines(_dev(x), _dev(y), crowd, rad)
    wp, wq = B.distance_join_lines(x, y, crowd, rad)
    assert np.array_equal(_i64(p), wp) and np.array_equal(_i64(q), wq)
    p2, q2 = ctx.distance_join_lines(_dev(x), _dev(y), crowd, rad)   # from the remembered total
    assert np.array_equal(_i64(p2), wp) and np.array_equal(_i64(q2), wq)
    # most crowded points meet several lines
    assert wp.size > 2 * np.unique(wp).size
    cnt = ctx.distance_join_lines_count(_dev(x), _dev(y), crowd, rad).cpu().numpy().astype(np.uint64)
    assert np.array_equal(cnt, np.bincount(wq, minlength=crowd["n_polys"]).astype(np.uint64))


def test_crowded_disk_join(ctx, pts):
    x, y = pts
    rng = np.random.default_rng(66)
    cx = C[0] + np.round(rng.uniform(-50.0, 50.0, 300))
    cy = C[1] + np.round(rng.uniform(-50.0, 50.0, 300))
    rad = rng.uniform(100.0, 300.0, 300)
    for r in (250.0, rad):
        p, d = ctx.distance_join(_dev(x), _dev(y), cx, cy, r)
        wp, wd = D.distance_join(x, y, cx, cy, r)
        assert np.array_equal(_i64(p), wp) and np.array_equal(_i64(d), wd)
        assert wp.size > 64 * 1000
        # more pairs than points: the first call retried with the total, a
        # repeated one starts from it
        assert wp.size > x.size
        p2, d2 = ctx.distance_join(_dev(x), _dev(y), cx, cy, r)
        assert np.array_equal(_i64(p2), wp) and np.array_equal(_i64(d2), wd)
        cnt = ctx.distance_join_count(_dev(x), _dev(y), cx, cy, r).cpu().numpy().astype(np.uint64)
        assert np.array_equal(cnt, D.distance_join_count(x, y, cx, cy, r))
