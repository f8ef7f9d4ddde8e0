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


def test_batch_join_count_graph_replays(ctx):
    """The batch join-count's launches are captured on the second call with
    the same set and table memory and replayed afterwards, each replay
    reading the rebuilt set's descriptors: every replay equals the oracle,
    with other device work between replays."""
    import oracle
    from workloads import gen
    L = gen.EXTENT_M
    x, y = gen.mixture_points(500_000, seed=95, L=L)
    t = ctx.table(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    cap0, rep0 = ctx.graph_stats()
    b = None
    base, _ = gen.query_stars(16, 8, 300, seed=96, L=L, area=(1e-3, 3e-2), data_seed=95)
    for k in range(6):
        # the same queries moved a little each time: same sizes, new descriptors
        stars = dict(base)
        stars["vx"] = base["vx"] + 256.0 * k
        stars["vy"] = base["vy"] - 128.0 * k
        qb = np.arange(17)
        b = ctx.batch(stars, qb, into=b)
        got = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, oracle.join_count(x, y, stars)), k
        torch.randn(1 << 20, device="cuda").sum().item()      # other work between replays
    cap1, rep1 = ctx.graph_stats()
    assert cap1 - cap0 >= 1 and rep1 - rep0 >= 2
    b.close()
    t.close()
