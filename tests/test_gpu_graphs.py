"""Repeated canvas builds replayed from captured HIP graphs.

The second build of a canvas with unchanged launch parameters captures its
launches into a graph and later builds replay it.  Every replay must equal
the eager result and the oracle, also with other device work (other
queries, torch kernels) between the replays, after the parameters change
(a new capture) and when the single row pass overflows its capacity and the
exact path follows the replayed launches.
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


def test_replays_equal_eager_and_oracle(ctx):
    x, y = gen.uniform_points(200_000, seed=41)
    polys = gen.voronoi_jitter(64, 8, 64, seed=41, L=1.0)
    other = gen.voronoi_jitter(30, 5, 20, seed=42, L=1.0)
    dx, dy = _dev(x), _dev(y)
    from paper_2203_14362_amd import Context
    ctx2 = Context(0)
    want = oracle.join_count(x, y, polys)
    opt, opg = oracle.join_pairs(x, y, polys)
    ctx.set_graphs(False)
    eager = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
    ctx.set_graphs(True)
    assert np.array_equal(eager, want)
    for k in range(6):
        got = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, want), k
        pt, pg = ctx.join_pairs(dx, dy, polys)
        assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg), k
        # device work in between: another context's query, a torch kernel
        assert int(ctx2.join_count(dx, dy, other).sum().item()) == x.size
        (dx * 2.0).sum().item()
    caps, reps = ctx.graph_stats()
    assert caps >= 1 and reps >= 8, (caps, reps)
    # new parameters (another resolution): eager, capture, replays again
    ctx.set_canvas_size(300, 200)
    try:
        for k in range(4):
            got = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, want), k
    finally:
        ctx.set_canvas_size(0, 0)
    caps2, reps2 = ctx.graph_stats()
    assert caps2 == caps + 1 and reps2 >= reps + 2, (caps2, reps2)
    ctx2.close()


def test_replays_with_overflowing_row_pass(ctx):
    """Heavily overlapping polygons: the single row pass runs out of record
    capacity on the first builds and the exact path completes them."""
    rings = [[np.stack([gen.star_polygon(40, 0.2, (0.5 + 0.01 * k, 0.5), L=1.0, seed=k)["vx"],
                        gen.star_polygon(40, 0.2, (0.5 + 0.01 * k, 0.5), L=1.0, seed=k)["vy"]], 1)]
             for k in range(12)]
    polys = gen.polys_from_rings(rings)
    x, y = gen.uniform_points(100_000, seed=43)
    dx, dy = _dev(x), _dev(y)
    want = oracle.join_count(x, y, polys)
    opt, opg = oracle.join_pairs(x, y, polys)
    cv = ctx.canvas(polys)          # a resident canvas of its own
    cv.close()
    for k in range(5):
        got = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, want), k
        pt, pg = ctx.join_pairs(dx, dy, polys)
        assert np.array_equal(_u32(pt), opt) and np.array_equal(_u32(pg), opg), k
