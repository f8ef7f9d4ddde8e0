"""GPU parity at small sizes: the HIP path vs the CPU oracle, element by element.

Inputs are seeded synthetic stand-ins (workloads.gen); expected values come
from the oracle only.  Sizes span many canvas tiles, ragged tails and every
canvas resolution class (1x1 = pure brute force up to 4096^2).
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _u32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


@pytest.fixture(scope="module")
def c1():
    x, y = gen.uniform_points(100_000, seed=1)
    polys = gen.voronoi_jitter(64, 8, 64, seed=1, L=1.0)
    return x, y, polys


def test_orient_matches_oracle(ctx):
    rng = np.random.default_rng(7)
    n = 20000
    a = rng.uniform(-1, 1, (n, 2))
    b = rng.uniform(-1, 1, (n, 2))
    t = rng.integers(-8, 9, n)[:, None] / 8.0
    c = a + t * (b - a)                     # near-collinear (rounded)
    c[: n // 4] = rng.uniform(-1, 1, (n // 4, 2))
    # exactly collinear dyadic triples
    a[n // 2:n // 2 + 1000] = rng.integers(-1000, 1000, (1000, 2)) / 64.0
    b[n // 2:n // 2 + 1000] = a[n // 2:n // 2 + 1000] + rng.integers(-50, 50, (1000, 2)) / 64.0
    c[n // 2:n // 2 + 1000] = a[n // 2:n // 2 + 1000] + 2 * (b[n // 2:n // 2 + 1000] - a[n // 2:n // 2 + 1000])
    # one-ulp perturbations
    c[n - 1000:] = np.nextafter(c[n - 1000:], np.inf)
    got = ctx.orient(torch.from_numpy(a), torch.from_numpy(b), torch.from_numpy(c)).cpu().numpy()
    want = np.array([oracle.orient_sign(*a[i], *b[i], *c[i]) for i in range(n)], dtype=np.int32)
    assert np.array_equal(got, want)
    assert (want == 0).sum() >= 1000


def test_c1_join_count(ctx, c1):
    x, y, polys = c1
    got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64)
    want = oracle.join_count(x, y, polys)
    assert np.array_equal(got, want)
    assert int(want.sum()) == x.size          # tessellation of [0,1)^2


def test_c1_join_pairs(ctx, c1):
    x, y, polys = c1
    pt, pg = ctx.join_pairs(_dev(x), _dev(y), polys)
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(_u32(pt), opt)
    assert np.array_equal(_u32(pg), opg)


@pytest.mark.parametrize("wh", [(1, 1), (2, 3), (17, 13), (64, 64), (333, 517), (1024, 1024), (4096, 4096), (8192, 1)])
def test_resolution_invariance(ctx, c1, wh):
    x, y, polys = c1
    ctx.set_canvas_size(*wh)
    try:
        got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64)
    finally:
        ctx.set_canvas_size(0, 0)
    assert np.array_equal(got, oracle.join_count(x, y, polys))


@pytest.mark.parametrize("wh", [(512, 1), (300, 2), (4096, 3)])
def test_long_runs_in_few_rows(ctx, wh):
    """Few canvas rows put whole polygons into one row: long runs of entries
    (processed by whole waves) and more of them than the per-row wave queue
    holds (the rest processed serially)."""
    x, y = gen.uniform_points(50_000, seed=31)
    polys = gen.voronoi_jitter(100, 30, 90, seed=31, L=1.0)
    ctx.set_canvas_size(*wh)
    try:
        got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64)
        pt, pg = ctx.join_pairs(_dev(x), _dev(y), polys)
    finally:
        ctx.set_canvas_size(0, 0)
    assert np.array_equal(got, oracle.join_count(x, y, polys))
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg)


def test_lattice_rectangles_gpu(ctx):
    h = 2.0 ** -6
    x, y = gen.lattice_points(130, 130, h, x0=-h, y0=-h)
    polys = gen.rect_grid(4, 4, 0.0, 0.0, 0.5, 0.5)   # corners on lattice lines
    for wh in [(0, 0), (8, 8), (7, 9), (512, 512)]:
        ctx.set_canvas_size(*wh)
        got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy()
        ctx.set_canvas_size(0, 0)
        assert got.tolist() == [32 * 32] * 16


def test_select_star(ctx):
    x, y = gen.mixture_points(300_000, seed=3, L=60000.0)
    poly = gen.star_polygon(1000, 0.15, (30000.0, 30000.0), L=60000.0, seed=3)
    got = _u32(ctx.select(_dev(x), _dev(y), poly))
    want = oracle.select(x, y, poly)
    assert np.array_equal(got, want)
    assert want.size > 0


def _mixed_polys():
    """Overlapping stars, a polygon with a hole, a duplicated polygon,
    axis-aligned (horizontal-edge) rectangles, a two-ring multi-polygon and
    degenerate polygons, over [0,1]^2."""
    star = lambda V, f, c, s: np.stack([gen.star_polygon(V, f, c, L=1.0, seed=s)["vx"],
                                        gen.star_polygon(V, f, c, L=1.0, seed=s)["vy"]], 1)
    outer = np.array([[0.05, 0.05], [0.6, 0.05], [0.6, 0.6], [0.05, 0.6]])
    hole = star(30, 0.03, (0.3, 0.3), 11)
    rect = np.array([[0.125, 0.5], [0.875, 0.5], [0.875, 0.75], [0.125, 0.75]])
    rings = [
        [star(200, 0.2, (0.5, 0.5), 1)],
        [star(50, 0.1, (0.45, 0.55), 2)],
        [outer, hole],
        [star(50, 0.1, (0.45, 0.55), 2)],          # duplicate of polygon 1
        [rect],
        [np.array([[0.7, 0.7], [0.9, 0.7], [0.9, 0.9]]), np.array([[0.1, 0.8], [0.2, 0.8], [0.15, 0.95]])],
        [np.array([[0.2, 0.2], [0.4, 0.4]])],      # two vertices
        [np.array([[0.1, 0.3], [0.5, 0.3], [0.9, 0.3]])],   # horizontal, zero area
    ]
    return gen.polys_from_rings(rings)


@pytest.mark.parametrize("wh", [(0, 0), (1, 1), (7, 5), (256, 256), (2048, 2048), (8192, 1)])
def test_overlaps_holes_multirings(ctx, wh):
    polys = _mixed_polys()
    x, y = gen.uniform_points(60_000, seed=21)
    x = np.concatenate([x, polys["vx"], (polys["vx"] + np.roll(polys["vx"], 1)) / 2])
    y = np.concatenate([y, polys["vy"], (polys["vy"] + np.roll(polys["vy"], 1)) / 2])
    ctx.set_canvas_size(*wh)
    try:
        got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64)
        pt, pg = ctx.join_pairs(_dev(x), _dev(y), polys)
    finally:
        ctx.set_canvas_size(0, 0)
    assert np.array_equal(got, oracle.join_count(x, y, polys))
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg)
    assert got[1] == got[3] and got[6] == 0 and got[7] == 0


def test_empty_and_degenerate_inputs(ctx):
    polys = gen.voronoi_jitter(8, 5, 12, seed=3, L=1.0)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert ctx.join_count(e, e, polys).cpu().tolist() == [0] * 8
    pt, pg = ctx.join_pairs(e, e, polys)
    assert pt.numel() == 0 and pg.numel() == 0
    empty = {"n_polys": 0, "poly_ring_off": np.zeros(1, np.int64), "ring_vtx_off": np.zeros(1, np.int64),
             "vx": np.zeros(0), "vy": np.zeros(0)}
    x, y = gen.uniform_points(1000, seed=4)
    assert ctx.join_count(_dev(x), _dev(y), empty).numel() == 0
    # NaN / inf / far-away points lie in no polygon
    xs = np.array([np.nan, 0.5, np.inf, -np.inf, 5.0, 0.5])
    ys = np.array([0.5, np.nan, 0.5, 0.5, 0.5, 0.5])
    got = ctx.join_count(_dev(xs), _dev(ys), polys).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, oracle.join_count(xs, ys, polys)) and int(got.sum()) == 1


def test_capacity_protocol(ctx):
    from paper_2203_14362_amd import SPADE_E_CAPACITY, SpadeError
    import ctypes
    x, y = gen.uniform_points(50_000, seed=6)
    poly = gen.star_polygon(100, 0.3, (0.5, 0.5), L=1.0, seed=6)
    want = oracle.select(x, y, poly)
    # a small explicit capacity: the wrapper retries with the reported size
    got = _u32(ctx.select(_dev(x), _dev(y), poly, cap=10))
    assert np.array_equal(got, want)
    pt, pg = ctx.join_pairs(_dev(x), _dev(y), poly, cap=3)
    assert np.array_equal(_u32(pt), want) and np.all(_u32(pg) == 0)


def test_invalid_polygon_sets(ctx):
    from paper_2203_14362_amd import SpadeError
    x, y = gen.uniform_points(100, seed=7)
    bad = {"n_polys": 1, "poly_ring_off": np.array([0, 1], np.int64),
           "ring_vtx_off": np.array([0, 3], np.int64),
           "vx": np.array([0.0, np.nan, 1.0]), "vy": np.array([0.0, 1.0, 0.0])}
    with pytest.raises(SpadeError):
        ctx.join_count(_dev(x), _dev(y), bad)
    bad2 = {"n_polys": 2, "poly_ring_off": np.array([0, 2, 1], np.int64),
            "ring_vtx_off": np.array([0, 3, 6], np.int64),
            "vx": np.zeros(6), "vy": np.zeros(6)}
    with pytest.raises(SpadeError):
        ctx.join_count(_dev(x), _dev(y), bad2)
    # the context still works afterwards
    polys = gen.voronoi_jitter(8, 5, 12, seed=3, L=1.0)
    assert np.array_equal(ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64),
                          oracle.join_count(x, y, polys))


@pytest.mark.parametrize("wh", [(0, 0), (700, 700), (2048, 2048)])
def test_byte_coarse_large_labels(ctx, wh):
    """More than 253 polygons in one canvas: byte-sized coarse words cannot
    hold the larger labels, whose uniform blocks are then read from the full
    canvas."""
    x, y = gen.uniform_points(200_000, seed=61)
    polys = gen.voronoi_jitter(400, 5, 20, seed=61, L=1.0)
    ctx.set_canvas_size(*wh)
    try:
        got = ctx.join_count(_dev(x), _dev(y), polys).cpu().numpy().astype(np.uint64)
        pt, pg = ctx.join_pairs(_dev(x), _dev(y), polys)
    finally:
        ctx.set_canvas_size(0, 0)
    assert np.array_equal(got, oracle.join_count(x, y, polys))
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg)
