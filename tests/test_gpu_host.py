"""Out-of-core tables: points kept in host memory, filtered by the clustered
grid index and streamed to the device in double-buffered chunks.  Results
equal the oracle on the original arrays."""
import numpy as np
import pytest

import oracle
from workloads import configs, gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


@pytest.fixture(scope="module")
def host_table(ctx):
    # more points than one staging buffer holds (2^24), with NaN points
    x, y = gen.mixture_points(40_000_000, seed=91, L=L)
    x[::1_000_003] = np.nan
    t = ctx.host_table(x, y)
    yield x, y, t
    t.close()


def test_host_join_count(ctx, host_table):
    x, y, t = host_table
    polys = configs.c2_polys()
    got = ctx.host_join_count(t, polys).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, oracle.join_count(x, y, polys))
    assert t.last_streamed == np.isfinite(x).sum()        # the tessellation covers every cell


def test_host_select_filters_cells(ctx, host_table):
    x, y, t = host_table
    for (V, area, cx, cy) in [(10_000, 0.15, L / 2, L / 2), (300, 0.002, 0.3 * L, 0.6 * L), (50, 1e-4, 5.0, 5.0)]:
        star = gen.star_polygon(V, area, (cx, cy), L=L, seed=92)
        got = ctx.host_select(t, star).cpu().numpy().astype(np.int64).astype(np.uint32)
        assert np.array_equal(got, oracle.select(x, y, star))
        assert t.last_streamed < x.size                    # the index filtered cells out


def test_host_small_and_empty(ctx):
    x, y = gen.uniform_points(1000, seed=93)
    t = ctx.host_table(x, y)
    polys = gen.voronoi_jitter(9, 8, 20, seed=93, L=1.0)
    assert np.array_equal(ctx.host_join_count(t, polys).cpu().numpy().astype(np.uint64),
                          oracle.join_count(x, y, polys))
    t.close()
    e = ctx.host_table(np.zeros(0), np.zeros(0))
    assert int(ctx.host_join_count(e, polys).sum()) == 0
    e.close()
