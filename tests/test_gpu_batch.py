"""GPU parity of resident tables and query batches against the CPU oracle.

A batch rasterises many queries into one canvas set and probes a resident,
grid-clustered point table once per (chunk, query) overlap.  Every query's
result must equal the oracle's for that query alone, and the result of a
query must not depend on the other queries of its batch.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _u32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


def _subset(polys, ks):
    """Polygons ks of a one-ring-per-polygon set, as a new set."""
    rvo = polys["ring_vtx_off"]
    rings = [[np.stack([polys["vx"][rvo[k]:rvo[k + 1]], polys["vy"][rvo[k]:rvo[k + 1]]], 1)] for k in ks]
    return gen.polys_from_rings(rings)


@pytest.fixture(scope="module")
def table_pts():
    x, y = gen.mixture_points(400_000, seed=3, L=L)
    # non-finite points, duplicates and the extent's corners
    x = np.concatenate([x, [np.nan, np.inf, 0.0, L, x[5], x[5]], x[:1000]])
    y = np.concatenate([y, [1.0, 2.0, 0.0, L, y[5], y[5]], y[:1000]])
    return x, y


@pytest.fixture(scope="module")
def stars():
    return gen.query_stars(48, 8, 3000, seed=11, L=L, area=(1e-4, 2e-2), data_seed=3)


def test_table_info(ctx, table_pts):
    x, y = table_pts
    t = ctx.table(_dev(x), _dev(y))
    info = t.info()
    assert info["n_points"] == x.size
    assert info["grid"] >= 1 and info["chunks"] == (x.size - 2 + 4095) // 4096
    t.close()


def test_batch_select_matches_oracle(ctx, table_pts, stars):
    x, y = table_pts
    polys, qb = stars
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    ids = _u32(ids)
    assert off[0] == 0 and off[-1] == ids.size
    nonempty = 0
    for q in range(polys["n_polys"]):
        want = oracle.select(x, y, polys, q)
        got = ids[off[q]:off[q + 1]]
        assert np.array_equal(got, want), "query %d" % q
        nonempty += want.size > 0
    assert nonempty >= polys["n_polys"] // 2
    b.close()
    t.close()


def test_batch_alone_equals_mix(ctx, table_pts, stars):
    x, y = table_pts
    polys, qb = stars
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    ids = _u32(ids)
    for q in (0, 7, 23, 47):
        one = _subset(polys, [q])
        b1 = ctx.batch(one, [0, 1])
        got1, off1 = ctx.batch_select(b1, t)
        assert np.array_equal(_u32(got1), ids[off[q]:off[q + 1]])
        # and the plain single-query call on the original arrays
        assert np.array_equal(_u32(ctx.select(_dev(x), _dev(y), one)), ids[off[q]:off[q + 1]])
        b1.close()
    b.close()
    t.close()


def test_batch_join_count(ctx):
    x, y = gen.uniform_points(300_000, seed=12)
    x = np.concatenate([x, [np.nan, 0.5]])
    y = np.concatenate([y, [0.5, np.inf]])
    v1 = gen.voronoi_jitter(64, 8, 64, seed=1, L=1.0)
    v2 = gen.voronoi_jitter(300, 4, 40, seed=2, L=1.0)
    star = gen.star_polygon(500, 0.2, (0.5, 0.5), L=1.0, seed=4)
    # queries: tessellation, empty query, tessellation, one star, overlapping mix
    allp = gen.concat_polys(gen.concat_polys(v1, v2), gen.concat_polys(star, star))
    qb = np.array([0, 64, 64, 364, 365, 366], dtype=np.int64)
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(allp, qb)
    got = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
    want = oracle.join_count(x, y, allp)
    assert np.array_equal(got, want)
    n_in = 300_000                          # the finite points, all in [0,1)^2
    assert int(want[:64].sum()) == n_in and int(want[64:364].sum()) == n_in
    # the same counts from the plain call, query by query
    assert np.array_equal(ctx.join_count(_dev(x), _dev(y), v1).cpu().numpy().astype(np.uint64), got[:64])
    b.close()
    t.close()


@pytest.mark.parametrize("case", ["one_tess", "three_tess_and_star", "large_tess_and_small"])
def test_batch_join_count_full_extent_canvases(ctx, case):
    """Canvases over most of the table's box (counted over the whole table)
    beside canvases probed chunk by chunk: every count equals the oracle's."""
    x, y = gen.uniform_points(60_000, seed=15)
    star = gen.star_polygon(300, 0.15, (0.4, 0.6), L=1.0, seed=5)
    if case == "one_tess":
        parts = [gen.voronoi_jitter(500, 4, 30, seed=6, L=1.0)]
    elif case == "three_tess_and_star":
        parts = [gen.voronoi_jitter(m, 4, 20, seed=7 + m, L=1.0) for m in (40, 200, 900)] + [star]
    else:
        # more polygons than the count probe's LDS histogram holds, beside a small tessellation
        parts = [gen.voronoi_jitter(9000, 4, 8, seed=9, L=1.0), gen.voronoi_jitter(30, 4, 20, seed=10, L=1.0), star]
    allp = parts[0]
    for p_ in parts[1:]:
        allp = gen.concat_polys(allp, p_)
    qb = np.cumsum([0] + [p_["n_polys"] for p_ in parts]).astype(np.int64)
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(allp, qb)
    for rep in range(2):
        got = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
        want = oracle.join_count(x, y, allp)
        assert np.array_equal(got, want), rep
    for q, p_ in enumerate(parts):
        if p_ is not star:
            assert int(got[qb[q]:qb[q + 1]].sum()) == x.size
    b.close()
    t.close()


def test_batch_select_capacity_and_retry(ctx, table_pts, stars):
    from paper_2203_14362_amd import SPADE_E_CAPACITY
    x, y = table_pts
    polys, qb = stars
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(polys, qb)
    full, off = ctx.batch_select(b, t)
    small, off2 = ctx.batch_select(b, t, cap=5)     # retried with the reported total
    assert np.array_equal(off, off2)
    assert np.array_equal(_u32(full), _u32(small))
    b.close()
    t.close()


def test_batch_degenerate(ctx):
    polys, qb = gen.query_stars(6, 8, 50, seed=13, L=1.0, area=(1e-3, 1e-2), data_seed=3)
    # empty table
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    t = ctx.table(e, e)
    assert t.info()["chunks"] == 0
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    assert ids.numel() == 0 and off.tolist() == [0] * 7
    assert ctx.batch_join_count(b, t).cpu().tolist() == [0] * 6
    t.close()
    # a table far away from every query, and one of only non-finite points
    for xs, ys in ((np.full(5000, 7.0), np.linspace(5, 6, 5000)), (np.full(100, np.nan), np.zeros(100))):
        t = ctx.table(_dev(xs), _dev(ys))
        ids, off = ctx.batch_select(b, t)
        assert ids.numel() == 0
        assert ctx.batch_join_count(b, t).cpu().tolist() == [0] * 6
        t.close()
    b.close()


def test_batch_invalid(ctx, table_pts):
    from paper_2203_14362_amd import SpadeError
    x, y = gen.uniform_points(1000, seed=14)
    t = ctx.table(_dev(x), _dev(y))
    v = gen.voronoi_jitter(8, 5, 12, seed=3, L=1.0)
    with pytest.raises(SpadeError):
        ctx.batch(v, [0, 5, 4, 8])          # decreasing bounds
    with pytest.raises(SpadeError):
        ctx.batch(v, [0, 4])                # does not end at n_polys
    b = ctx.batch(v, [0, 4, 8])
    with pytest.raises(SpadeError):
        ctx.batch_select(b, t)              # selection needs one polygon per query
    with pytest.raises(SpadeError):
        ctx.join_count(_dev(x), _dev(y), b)  # a set is not a single canvas
    got = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, oracle.join_count(x, y, v))
    b.close()
    t.close()


def test_batch_select_many_runs(ctx):
    """Point ids above 2^27 (28 bits): a run of the selection's sort holds
    at most 16 queries (32-bit keys), so 97 queries make seven runs, the
    last of one query; the finite points sit at spread ids among non-finite
    ones.  Also with a capacity that ends inside the fifth run."""
    rng = np.random.default_rng(41)
    n = (1 << 27) + 5
    xf, yf = gen.mixture_points(200_000, seed=42, L=L)
    pos = np.sort(rng.choice(n, xf.size, replace=False))
    pos[-1] = n - 1
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    x[torch.from_numpy(pos).cuda()] = _dev(xf)
    y[torch.from_numpy(pos).cuda()] = _dev(yf)
    polys, qb = gen.query_stars(97, 8, 1500, seed=43, L=L, area=(1e-3, 3e-2), data_seed=42)
    t = ctx.table(x, y)
    del x, y
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    ids = ids.cpu().numpy().astype(np.int64)
    for q in range(97):
        want = pos[oracle.select(xf, yf, polys, q).astype(np.int64)]
        assert np.array_equal(ids[off[q]:off[q + 1]], want), "query %d" % q
    # first-cap semantics with the cap inside the fifth run (queries 64..79)
    cap = int((off[70] + off[71]) // 2)
    if cap > 0:
        buf = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        off2 = np.zeros(98, dtype=np.int64)
        ctx._sync_stream()
        rc = ctx.lib.spade_batch_select(ctx.handle, b.handle, t.handle, ctypes.c_void_p(buf.data_ptr()), cap,
                                        off2.ctypes.data_as(ctypes.c_void_p))
        from paper_2203_14362_amd import SPADE_E_CAPACITY
        assert rc == SPADE_E_CAPACITY and np.array_equal(off2, off)
        assert np.array_equal(buf.cpu().numpy().astype(np.int64), ids[:cap])
    b.close()
    t.close()


def test_batch_select_without_hit_masks(ctx, table_pts, stars, monkeypatch):
    """The write pass that probes again (match masks over their limit) gives
    the same ids, also for a capacity that ends inside the batch."""
    x, y = table_pts
    polys, qb = stars
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    monkeypatch.setenv("SPADE_HIT_MASK_LIMIT", "0")
    ids2, off2 = ctx.batch_select(b, t)
    assert np.array_equal(off, off2) and torch.equal(ids, ids2)
    cap = int(off[-1]) // 2
    buf = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    off3 = np.zeros(off.size, dtype=np.int64)
    ctx._sync_stream()
    rc = ctx.lib.spade_batch_select(ctx.handle, b.handle, t.handle, ctypes.c_void_p(buf.data_ptr()), cap,
                                    off3.ctypes.data_as(ctypes.c_void_p))
    from paper_2203_14362_amd import SPADE_E_CAPACITY
    assert rc == SPADE_E_CAPACITY and np.array_equal(off3, off)
    assert torch.equal(buf[:cap], ids[:cap])
    monkeypatch.delenv("SPADE_HIT_MASK_LIMIT")
    for q in (0, 11, 47):
        assert np.array_equal(_u32(ids2)[off[q]:off[q + 1]], oracle.select(x, y, polys, q)), q
    b.close()
    t.close()


@pytest.mark.parametrize("n", [1, 7, 33, 70])
def test_batch_select_tiny_tables(ctx, n):
    """Id spaces of a few bits: the ordering bitmap is a single word."""
    rng = np.random.default_rng(50 + n)
    x = rng.uniform(0.2, 0.8, n)
    y = rng.uniform(0.2, 0.8, n)
    polys, qb = gen.query_stars(5, 8, 40, seed=51, L=1.0, area=(0.05, 0.4), data_seed=3)
    t = ctx.table(_dev(x), _dev(y))
    b = ctx.batch(polys, qb)
    ids, off = ctx.batch_select(b, t)
    ids = _u32(ids)
    for q in range(5):
        assert np.array_equal(ids[off[q]:off[q + 1]], oracle.select(x, y, polys, q)), q
    b.close()
    t.close()
