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
