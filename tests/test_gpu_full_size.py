"""Parity at the full workload sizes, on sampled outputs.

At 100M-500M points the oracle cannot recompute whole results, so each test
checks (a) properties that hold at any size (every point of a tessellation
in exactly one pair, ids ascending and unique, counts equal to the pair
histogram) and (b) the GPU's answer for a seeded random sample of points
against the oracle evaluated on exactly those points.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M
SAMPLE = 200_000


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _sample(n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(SAMPLE, n), replace=False))


def _member(sorted_ids, idx):
    """For each index in idx: is it in the ascending id array?"""
    if sorted_ids.size == 0:
        return np.zeros(idx.size, bool)
    pos = np.minimum(np.searchsorted(sorted_ids, idx), sorted_ids.size - 1)
    return sorted_ids[pos] == idx


def test_c2_full_join_pairs_and_counts(ctx):
    """100M clustered points x 260 Voronoi-jitter polygons (50-500 vertices)."""
    N = 100_000_000
    x, y = gen.mixture_points(N, seed=2, L=L)
    polys = gen.voronoi_jitter(260, 50, 500, seed=2, L=L)
    dx, dy = _dev(x), _dev(y)
    counts = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.int64)
    pt, pg = ctx.join_pairs(dx, dy, polys)
    pt = pt.cpu().numpy().astype(np.int64)
    pg = pg.cpu().numpy().astype(np.int64)
    # a tessellation of the extent: every point in exactly one pair, in order
    assert pt.size == N and np.array_equal(pt, np.arange(N))
    assert np.array_equal(np.bincount(pg, minlength=260), counts) and counts.sum() == N
    idx = _sample(N, 5)
    opt, opg = oracle.join_pairs(x[idx], y[idx], polys)
    assert np.array_equal(opt, np.arange(idx.size))
    assert np.array_equal(pg[idx], opg.astype(np.int64))


def test_c3_full_selection(ctx):
    """500M clustered points x one 10k-vertex star (~15% of the extent)."""
    N = 500_000_000
    x, y = gen.mixture_points(N, seed=2, L=L)
    star = gen.star_polygon(10_000, 0.15, (L / 2, L / 2), L=L, seed=3)
    ids = ctx.select(_dev(x), _dev(y), star).cpu().numpy().astype(np.int64)
    assert ids.size > 0 and np.all(np.diff(ids) > 0) and ids[0] >= 0 and ids[-1] < N
    idx = _sample(N, 6)
    want = np.zeros(idx.size, bool)
    want[oracle.select(x[idx], y[idx], star).astype(np.int64)] = True
    assert np.array_equal(_member(ids, idx), want)
    assert want.sum() > 0.02 * idx.size


@pytest.fixture(scope="module")
def c4_points():
    return gen.mixture_points(200_000_000, seed=2, L=L)


def test_c4_full_batched_selection(ctx, c4_points):
    """1024 star selections (8-20000 vertices) over a resident 200M-point table."""
    x, y = c4_points
    N = x.size
    stars, qb = gen.query_stars(1024, 8, 20_000, seed=8, L=L, area=(1e-4, 1e-2), data_seed=2)
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    b = ctx.batch(stars, qb)
    ids, off = ctx.batch_select(b, t)
    ids = ids.cpu().numpy().astype(np.int64)
    idx = _sample(N, 7)
    xs, ys = x[idx], y[idx]
    for q in range(1024):
        got = ids[off[q]:off[q + 1]]
        assert got.size == 0 or np.all(np.diff(got) > 0), q
        want = np.zeros(idx.size, bool)
        want[oracle.select(xs, ys, stars, q).astype(np.int64)] = True
        assert np.array_equal(_member(got, idx), want), q
    # a few queries alone through the plain call on the original arrays
    rvo = stars["ring_vtx_off"]
    for q in (0, 511, 1023):
        one = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, rvo[q + 1] - rvo[q]]),
               "vx": stars["vx"][rvo[q]:rvo[q + 1]], "vy": stars["vy"][rvo[q]:rvo[q + 1]]}
        alone = ctx.select(dx, dy, one).cpu().numpy().astype(np.int64)
        assert np.array_equal(alone, ids[off[q]:off[q + 1]]), q
    b.close()
    t.close()


def test_c4_full_join_40k(ctx, c4_points):
    """Join-count with 40k Voronoi polygons (4-40 vertices) over the 200M table."""
    x, y = c4_points
    N = x.size
    tess = gen.voronoi_jitter(40_000, 4, 40, seed=9, L=L)
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    b = ctx.batch(tess, [0, 40_000])
    counts = ctx.batch_join_count(b, t).cpu().numpy().astype(np.int64)
    assert counts.sum() == N
    plain = ctx.join_count(dx, dy, tess).cpu().numpy().astype(np.int64)
    assert np.array_equal(plain, counts)
    pt, pg = ctx.join_pairs(dx, dy, tess)
    pt = pt.cpu().numpy().astype(np.int64)
    pg = pg.cpu().numpy().astype(np.int64)
    assert pt.size == N and np.array_equal(pt, np.arange(N))
    assert np.array_equal(np.bincount(pg, minlength=40_000), counts)
    idx = _sample(N, 8)
    opt, opg = oracle.join_pairs(x[idx], y[idx], tess)
    assert np.array_equal(opt, np.arange(idx.size))
    assert np.array_equal(pg[idx], opg.astype(np.int64))
    b.close()
    t.close()
