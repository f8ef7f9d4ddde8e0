"""GPU parity of the distance join with lines (join types (1) and (2) with
lines as the constraint dataset) against the exact CPU oracle: pairs and
per-line counts, per-line distances, point lines against the disk join,
the capacity protocol and invalid input."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import buffer as B
from paper_2203_14362_amd import spade
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _i64(t):
    return t.cpu().numpy().astype(np.int64)


@pytest.fixture(scope="module")
def pts():
    return gen.mixture_points(200_000, seed=51, L=L)


@pytest.fixture(scope="module")
def roads():
    return gen.road_lines(40, 50, 300.0, seed=52, L=L)


@pytest.mark.parametrize("r", [0.0, 60.0, 700.0])
def test_type1_pairs_and_counts(ctx, pts, roads, r):
    x, y = pts
    pt, pl = ctx.distance_join_lines(_dev(x), _dev(y), roads, r)
    wp, wl = B.distance_join_lines(x, y, roads, r)
    assert np.array_equal(_i64(pt), wp) and np.array_equal(_i64(pl), wl)
    c = ctx.distance_join_lines_count(_dev(x), _dev(y), roads, r)
    assert np.array_equal(c.cpu().numpy().astype(np.uint64), B.distance_join_lines_count(x, y, roads, r))
    if r > 0:
        assert wp.size > 1000


def test_type2_per_line_distances(ctx, pts, roads):
    x, y = pts
    rng = np.random.default_rng(53)
    rad = rng.uniform(0.0, 400.0, roads["n_polys"])
    rad[3] = 0.0
    pt, pl = ctx.distance_join_lines(_dev(x), _dev(y), roads, rad)
    wp, wl = B.distance_join_lines(x, y, roads, rad)
    assert np.array_equal(_i64(pt), wp) and np.array_equal(_i64(pl), wl)
    c = ctx.distance_join_lines_count(_dev(x), _dev(y), roads, rad)
    assert np.array_equal(c.cpu().numpy().astype(np.uint64), np.bincount(wl, minlength=roads["n_polys"]))


def test_point_lines_equal_the_disk_join(ctx, pts):
    x, y = pts
    rng = np.random.default_rng(54)
    k = rng.choice(x.size, 50, replace=False)
    cx, cy = np.round(x[k]), np.round(y[k])
    lines = gen.polys_from_rings([[np.array([[a, b]])] for a, b in zip(cx, cy)])
    rad = rng.uniform(50.0, 800.0, 50)
    pt, pl = ctx.distance_join_lines(_dev(x), _dev(y), lines, rad)
    dp, dd = ctx.distance_join(_dev(x), _dev(y), cx, cy, rad)
    assert torch.equal(pt.cpu().to(torch.int64), dp.cpu().to(torch.int64))
    assert torch.equal(pl.cpu().to(torch.int64), dd.cpu().to(torch.int64))


def test_capacity_and_invalid(ctx, pts, roads):
    from paper_2203_14362_amd import SpadeError
    x, y = pts
    dx, dy = _dev(x), _dev(y)
    wp, wl = B.distance_join_lines(x, y, roads, 150.0)
    cap = wp.size // 2
    lib = ctx.lib
    P = spade._Points(dx.numel(), dx.data_ptr(), dy.data_ptr())
    dl = ctx.polys(roads)
    bpt = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    bpl = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    ctx._sync_stream()
    rc = lib.spade_distance_join_lines_pairs(ctx.handle, ctypes.byref(P), ctypes.byref(dl.cstruct()), None, 150.0,
                                             ctypes.c_void_p(bpt.data_ptr()), ctypes.c_void_p(bpl.data_ptr()), cap,
                                             ctypes.byref(n))
    assert rc == spade.SPADE_E_CAPACITY and n.value == wp.size
    assert np.array_equal(bpt.cpu().numpy().astype(np.int64), wp[:cap])
    assert np.array_equal(bpl.cpu().numpy().astype(np.int64), wl[:cap])
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    pt, pl = ctx.distance_join_lines(e, e, roads, 10.0)
    assert pt.numel() == 0 and pl.numel() == 0
    assert int(ctx.distance_join_lines_count(e, e, roads, 10.0).sum()) == 0
    with pytest.raises(SpadeError):
        ctx.distance_join_lines(dx, dy, roads, -1.0)
    bad_r = np.full(roads["n_polys"], 5.0)
    bad_r[7] = np.nan
    with pytest.raises(SpadeError):
        ctx.distance_join_lines(dx, dy, roads, bad_r)
    bad = dict(roads)
    bad["vy"] = roads["vy"].copy()
    bad["vy"][11] = np.inf
    with pytest.raises(SpadeError):
        ctx.distance_join_lines_count(dx, dy, bad, 5.0)
