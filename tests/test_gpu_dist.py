"""Distance joins (types (1) and (2)) and kNN selection on the GPU against the
CPU oracle (oracle/disk.py): pairs, per-disk counts and nearest-first ids,
bit-exact, including points exactly on circles and ties in distance."""
import numpy as np
import pytest
import torch

from oracle import disk
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _u32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


@pytest.fixture(scope="module")
def clustered():
    return gen.mixture_points(400_000, seed=81, L=L)


@pytest.mark.parametrize("kind", ["type1", "type2", "type2_wide", "one_disk", "zero_radius"])
def test_distance_join_matches_oracle(ctx, clustered, kind):
    x, y = clustered
    rng = np.random.default_rng(82)
    nd = {"type1": 1500, "type2": 1500, "type2_wide": 60, "one_disk": 1, "zero_radius": 50}[kind]
    cx, cy = gen.mixture_points(nd, seed=83, L=L)
    if kind == "type1":
        r = 400.0
    elif kind == "type2":
        r = np.exp(rng.uniform(np.log(20.0), np.log(2000.0), nd))
    elif kind == "type2_wide":
        r = rng.uniform(2000.0, 15000.0, nd)
    elif kind == "one_disk":
        r = 5000.0
    else:
        r = 0.0
        cx, cy = x[:nd].copy(), y[:nd].copy()    # disks of radius 0 at data points
    pt, pd = ctx.distance_join(_dev(x), _dev(y), cx, cy, r)
    opt, opd = disk.distance_join(x, y, cx, cy, r)
    assert np.array_equal(_u32(pt), opt.astype(np.uint32))
    assert np.array_equal(_u32(pd), opd.astype(np.uint32))
    cnt = ctx.distance_join_count(_dev(x), _dev(y), cx, cy, r).cpu().numpy().astype(np.uint64)
    assert np.array_equal(cnt, np.bincount(opd, minlength=nd).astype(np.uint64))
    if kind == "zero_radius":
        assert opt.size >= nd


def test_distance_join_lattice_points_on_circles(ctx):
    """Integer lattice, integer radii: many points lie exactly on circles."""
    g = np.arange(-40, 41, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    cx = np.array([0.0, 3.0, -5.0, 7.0, 0.5, 20.0])
    cy = np.array([0.0, -2.0, 4.0, 7.0, 0.5, -20.0])
    r = np.array([5.0, 25.0, 0.0, 13.0, 10.5, 30.0])
    pt, pd = ctx.distance_join(_dev(x), _dev(y), cx, cy, r)
    want = sorted((i, j) for j in range(cx.size) for i in range(x.size)
                  if (x[i] - cx[j]) ** 2 + (y[i] - cy[j]) ** 2 <= r[j] ** 2)   # exact: small dyadic values
    assert list(zip(_u32(pt).tolist(), _u32(pd).tolist())) == want


def test_distance_join_capacity_and_invalid(ctx, clustered):
    from paper_2203_14362_amd import SpadeError
    x, y = clustered
    cx, cy = gen.mixture_points(100, seed=84, L=L)
    full_pt, full_pd = ctx.distance_join(_dev(x), _dev(y), cx, cy, 800.0)
    pt, pd = ctx.distance_join(_dev(x), _dev(y), cx, cy, 800.0, cap=7)   # retried at the reported size
    assert torch.equal(pt, full_pt) and torch.equal(pd, full_pd)
    for bad in [(cx, cy, -1.0), (np.array([np.nan]), np.array([0.0]), 1.0),
                (cx, cy, np.full(cx.size, np.inf))]:
        with pytest.raises(SpadeError):
            ctx.distance_join(_dev(x), _dev(y), *bad)
    e_pt, e_pd = ctx.distance_join(_dev(x), _dev(y), np.zeros(0), np.zeros(0), 1.0)
    assert e_pt.numel() == 0


@pytest.mark.parametrize("k", [1, 10, 1000, 50_000])
def test_knn_matches_oracle(ctx, clustered, k):
    x, y = clustered
    dx, dy = _dev(x), _dev(y)
    for (px, py) in [(L / 2, L / 2), (x[123], y[123]), (-5000.0, 70000.0), (31234.5, 1.0)]:
        got = ctx.knn(dx, dy, px, py, k).cpu().numpy().astype(np.int64)
        assert np.array_equal(got, disk.knn(x, y, px, py, k)), (px, py, k)


def test_knn_ties_and_edges(ctx):
    g = np.arange(-30, 31, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel().copy(), Y.ravel().copy()
    x[::97] = np.nan                          # points that can never be chosen
    dx, dy = _dev(x), _dev(y)
    for (px, py, k) in [(0.0, 0.0, 1), (0.0, 0.0, 45), (3.0, -7.0, 500), (30.0, 30.0, 10_000)]:
        got = ctx.knn(dx, dy, px, py, k).cpu().numpy().astype(np.int64)
        assert np.array_equal(got, disk.knn(x, y, px, py, k)), (px, py, k)
    assert ctx.knn(dx, dy, 0.0, 0.0, 0).numel() == 0
    assert ctx.knn(dx[:0], dy[:0], 0.0, 0.0, 5).numel() == 0


def test_knn_beyond_power_of_two_circles(ctx):
    """Points farther than 2^511 (6.7e153) from the query lie outside every
    power-of-two circle: a k that needs them takes the circles r_max / 2^i
    from the points' bounding box.  Squared distances stay below the FP64
    maximum, inside the exact predicate's range."""
    g = np.arange(-5, 6, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    far_x = np.array([9e153, 0.0, -6e153, 5e153, 3.0])
    far_y = np.array([0.0, 8e153, -6e153, 0.0, 7e153])
    x = np.concatenate([X.ravel(), far_x])
    y = np.concatenate([Y.ravel(), far_y])
    dx, dy = _dev(x), _dev(y)
    for k in (5, 121, 122, 123, 124, 200):
        got = ctx.knn(dx, dy, 0.5, 0.25, k).cpu().numpy().astype(np.int64)
        assert np.array_equal(got, disk.knn(x, y, 0.5, 0.25, k)), k
