"""The caller's bounding box: canvases sized without waiting for the device.

A polygon set built from host arrays carries their bounding box, so the
library sizes the canvas at once and checks on the device, before anything
reads the polygon arrays, that the offsets are valid and that every vertex
lies inside the box.  A box that is too large only changes the canvas (the
results stay exact); one that misses a vertex, like invalid offsets, fails
the call and leaves the context usable.  The plain calls also read the
build's counters only at the probe's own synchronisation; a build whose row
pass ran out of room is redone and probed again.
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


def _counts(ctx, x, y, p):
    return ctx.join_count(_dev(x), _dev(y), p).cpu().numpy().astype(np.uint64)


def test_box_is_taken_from_host_arrays(ctx):
    polys = gen.voronoi_jitter(20, 5, 30, seed=51, L=1.0)
    dp = ctx.polys(polys)
    want = [polys["vx"].min(), polys["vx"].max(), polys["vy"].min(), polys["vy"].max()]
    assert dp.bbox is not None and np.array_equal(dp.bbox, want)
    x, y = gen.uniform_points(100_000, seed=51)
    assert np.array_equal(_counts(ctx, x, y, dp), oracle.join_count(x, y, polys))


def test_larger_box_gives_the_same_results(ctx):
    polys = gen.voronoi_jitter(30, 5, 40, seed=52, L=1.0)
    x, y = gen.uniform_points(100_000, seed=52)
    x = x * 1.4 - 0.2
    y = y * 1.4 - 0.2
    dp = ctx.polys(polys)
    dp.bbox = dp.bbox + np.array([-0.3, 0.25, -0.1, 0.4])
    assert np.array_equal(_counts(ctx, x, y, dp), oracle.join_count(x, y, polys))
    pt, pg = ctx.join_pairs(_dev(x), _dev(y), dp)
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg)
    cv = ctx.canvas(dp)
    try:
        assert cv.info()["n_polys"] == 30
    finally:
        cv.close()


@pytest.mark.parametrize("side", [0, 1, 2, 3])
def test_box_missing_a_vertex_fails(ctx, side):
    from paper_2203_14362_amd import SpadeError
    polys = gen.voronoi_jitter(12, 5, 20, seed=53, L=1.0)
    x, y = gen.uniform_points(10_000, seed=53)
    dp = ctx.polys(polys)
    shrink = np.zeros(4)
    shrink[side] = 1e-9 if side in (0, 2) else -1e-9
    dp.bbox = dp.bbox + shrink
    with pytest.raises(SpadeError, match="bounding box"):
        ctx.join_count(_dev(x), _dev(y), dp)
    with pytest.raises(SpadeError, match="bounding box"):
        ctx.join_pairs(_dev(x), _dev(y), dp)
    with pytest.raises(SpadeError, match="bounding box"):
        ctx.canvas(dp)
    # the context still works, with and without the box
    assert np.array_equal(_counts(ctx, x, y, polys), oracle.join_count(x, y, polys))
    dp.bbox = None
    assert np.array_equal(_counts(ctx, x, y, dp), oracle.join_count(x, y, polys))


def test_invalid_offsets_with_box_fail(ctx):
    from paper_2203_14362_amd import SpadeError
    x, y = gen.uniform_points(1000, seed=54)
    # decreasing ring offsets, finite vertices (so the box is known)
    bad = {"n_polys": 2, "poly_ring_off": None, "ring_vtx_off": np.array([0, 5, 3], np.int64),
           "vx": np.linspace(0.1, 0.9, 5), "vy": np.array([0.1, 0.8, 0.3, 0.9, 0.2])}
    with pytest.raises(SpadeError, match="ring_vtx_off"):
        ctx.join_count(_dev(x), _dev(y), bad)
    # vertex count of the arrays differs from the offsets
    bad2 = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, 4], np.int64),
            "vx": np.array([0.1, 0.9, 0.9, 0.1, 0.5, 0.5]), "vy": np.array([0.1, 0.1, 0.9, 0.9, 0.5, 0.5])}
    with pytest.raises(SpadeError, match="n_vertices"):
        ctx.join_count(_dev(x), _dev(y), bad2)
    with pytest.raises(SpadeError, match="n_vertices"):
        ctx.select(_dev(x), _dev(y), bad2)
    polys = gen.voronoi_jitter(8, 5, 12, seed=3, L=1.0)
    assert np.array_equal(_counts(ctx, x, y, polys), oracle.join_count(x, y, polys))


def test_overflowing_row_pass_is_redone(ctx):
    """Overlapping stars overflow the single row pass's first guess; the
    plain call probes, sees the flag at its synchronisation, rebuilds and
    probes again.  A fresh context each time, so the guess starts small."""
    from paper_2203_14362_amd import Context
    rings = []
    for k in range(16):
        s = gen.star_polygon(60, 0.25, (0.45 + 0.007 * k, 0.5), L=1.0, seed=100 + k)
        rings.append([np.stack([s["vx"], s["vy"]], 1)])
    polys = gen.polys_from_rings(rings)
    x, y = gen.uniform_points(100_000, seed=55)
    want = oracle.join_count(x, y, polys)
    opt, opg = oracle.join_pairs(x, y, polys)
    for call in ("count", "pairs"):
        c = Context(0)
        try:
            if call == "count":
                assert np.array_equal(_counts(c, x, y, polys), want)
            else:
                pt, pg = c.join_pairs(_dev(x), _dev(y), polys)
                assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg)
        finally:
            c.close()
