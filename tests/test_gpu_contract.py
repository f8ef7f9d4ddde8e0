"""The C ABI's contract, called through raw ctypes: results complete when a
plain call returns (also on the path that rebuilds an overflowing canvas),
the first cap results written on SPADE_E_CAPACITY, memory facts."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from oracle import disk as odisk
from paper_2203_14362_amd import spade
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _pts(dx, dy):
    return spade._Points(dx.numel(), dx.data_ptr(), dy.data_ptr())


def _overlapping_squares(k=40):
    """k large squares that overlap almost everywhere: at a fixed canvas every
    interior pixel is claimed by many polygons, far more candidate records
    than the first row pass is sized for."""
    rings = []
    for i in range(k):
        a = 0.01 + 0.002 * i
        b = 0.99 - 0.0015 * i
        rings.append([np.array([[a, a], [b, a], [b, b], [a, b]])])
    return gen.polys_from_rings(rings)


def test_join_count_rebuild_path_complete_on_return():
    """spade_join_count on its own stream, results read on another stream
    right after it returns, on a fresh context whose first build overflows."""
    lib = spade.load_library()
    polys = _overlapping_squares()
    x, y = gen.uniform_points(200_000, seed=31)
    dx, dy = _dev(x), _dev(y)
    own = torch.cuda.Stream()
    other = torch.cuda.Stream()
    h = ctypes.c_void_p()
    assert lib.spade_ctx_create(0, ctypes.c_void_p(own.cuda_stream), ctypes.byref(h)) == 0
    try:
        assert lib.spade_ctx_set_canvas_size(h, 256, 256) == 0
        dp = spade.DevicePolys(polys, torch.device("cuda", 0))
        torch.cuda.synchronize()
        out = torch.full((polys["n_polys"],), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        P = _pts(dx, dy)
        rc = lib.spade_join_count(h, ctypes.byref(P), ctypes.byref(dp.cstruct()), ctypes.c_void_p(out.data_ptr()))
        assert rc == 0, lib.spade_last_error(h)
        with torch.cuda.stream(other):
            got = out.to("cpu").numpy().astype(np.uint64)
        b, r = ctypes.c_int64(), ctypes.c_int64()
        lib.spade_ctx_build_stats(h, ctypes.byref(b), ctypes.byref(r))
        assert b.value >= 2 and r.value == 1       # the first build was redone
    finally:
        lib.spade_ctx_destroy(h)
    assert np.array_equal(got, oracle.join_count(x, y, polys))


def test_capacity_writes_first_cap_results(ctx):
    lib = ctx.lib
    x, y = gen.uniform_points(60_000, seed=32)
    dx, dy = _dev(x), _dev(y)
    P = _pts(dx, dy)
    star = gen.star_polygon(300, 0.3, (0.5, 0.5), L=1.0, seed=33)
    want = oracle.select(x, y, star)
    cap = want.size // 2
    dp = ctx.polys(star)
    buf = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    ctx._sync_stream()
    rc = lib.spade_select(ctx.handle, ctypes.byref(P), ctypes.byref(dp.cstruct()), ctypes.c_void_p(buf.data_ptr()),
                          cap, ctypes.byref(n))
    assert rc == spade.SPADE_E_CAPACITY and n.value == want.size
    assert np.array_equal(buf.cpu().numpy().astype(np.uint32), want[:cap])

    # distance selection
    wd = odisk.select_disk(x, y, 0.4, 0.55, 0.21)
    capd = wd.size // 3
    buf = torch.full((capd,), -1, dtype=torch.int32, device="cuda")
    rc = lib.spade_select_disk(ctx.handle, ctypes.byref(P), 0.4, 0.55, 0.21, ctypes.c_void_p(buf.data_ptr()), capd,
                               ctypes.byref(n))
    assert rc == spade.SPADE_E_CAPACITY and n.value == wd.size
    assert np.array_equal(buf.cpu().numpy().astype(np.uint32), wd[:capd])

    # join pairs
    polys = gen.voronoi_jitter(16, 8, 64, seed=34, L=1.0)
    opt, opg = oracle.join_pairs(x, y, polys)
    capp = opt.size - 777
    dpp = ctx.polys(polys)
    bpt = torch.full((capp,), -1, dtype=torch.int32, device="cuda")
    bpg = torch.full((capp,), -1, dtype=torch.int32, device="cuda")
    rc = lib.spade_join_pairs(ctx.handle, ctypes.byref(P), ctypes.byref(dpp.cstruct()),
                              ctypes.c_void_p(bpt.data_ptr()), ctypes.c_void_p(bpg.data_ptr()), capp, ctypes.byref(n))
    assert rc == spade.SPADE_E_CAPACITY and n.value == opt.size
    assert np.array_equal(bpt.cpu().numpy().astype(np.uint32), opt[:capp])
    assert np.array_equal(bpg.cpu().numpy().astype(np.uint32), opg[:capp])

    # join pairs with overlapping polygons: caps that cut through the
    # entries of a point in several polygons keep its smallest polygons
    stars, _ = gen.query_stars(40, 8, 64, seed=35, L=1.0, area=(0.02, 0.2), data_seed=2)
    opt, opg = oracle.join_pairs(x, y, stars)
    runs = np.nonzero((opt[1:-1] == opt[:-2]) & (opt[1:-1] == opt[2:]))[0] + 1
    assert runs.size > 100
    dps = ctx.polys(stars)
    for capp in (int(runs[0]), int(runs[runs.size // 2]), int(runs[-1]) + 1, opt.size - 1):
        bpt = torch.full((capp,), -1, dtype=torch.int32, device="cuda")
        bpg = torch.full((capp,), -1, dtype=torch.int32, device="cuda")
        rc = lib.spade_join_pairs(ctx.handle, ctypes.byref(P), ctypes.byref(dps.cstruct()),
                                  ctypes.c_void_p(bpt.data_ptr()), ctypes.c_void_p(bpg.data_ptr()), capp,
                                  ctypes.byref(n))
        assert rc == spade.SPADE_E_CAPACITY and n.value == opt.size
        assert np.array_equal(bpt.cpu().numpy().astype(np.uint32), opt[:capp]), capp
        assert np.array_equal(bpg.cpu().numpy().astype(np.uint32), opg[:capp]), capp
    full_pt, full_pg = ctx.join_pairs(_dev(x), _dev(y), stars)
    assert np.array_equal(full_pt.cpu().numpy(), opt) and np.array_equal(full_pg.cpu().numpy(), opg)

    # distance selections from lines and from a polygon
    from oracle import buffer as obuf
    lines = gen.polys_from_rings([[np.array([[0.1, 0.1], [0.5, 0.7], [0.9, 0.2]])],
                                  [np.array([[0.2, 0.9], [0.8, 0.85]])]])
    for fn, geom, r, want_fn in ((lib.spade_select_near_lines, lines, 0.05, obuf.select_near_lines),
                                 (lib.spade_select_within_polygon, star, 0.03, obuf.select_within_polygon)):
        wl = want_fn(x, y, geom, r)
        capl = wl.size // 2
        dg = ctx.polys(geom)
        buf = torch.full((capl,), -1, dtype=torch.int32, device="cuda")
        rc = fn(ctx.handle, ctypes.byref(P), ctypes.byref(dg.cstruct()), r, ctypes.c_void_p(buf.data_ptr()), capl,
                ctypes.byref(n))
        assert rc == spade.SPADE_E_CAPACITY and n.value == wl.size
        assert np.array_equal(buf.cpu().numpy().astype(np.uint32), wl[:capl])


def test_batch_select_capacity_writes_first_cap(ctx):
    L = gen.EXTENT_M
    x, y = gen.mixture_points(300_000, seed=4, L=L)
    stars, qb = gen.query_stars(24, 8, 2000, seed=35, L=L, area=(1e-3, 5e-2), data_seed=4)
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    b = ctx.batch(stars, qb)
    full, off = ctx.batch_select(b, t)
    full = full.cpu().numpy().astype(np.uint32)
    for q in range(24):
        assert np.array_equal(full[off[q]:off[q + 1]], oracle.select(x, y, stars, q)), q
    cap = int(off[-1]) * 2 // 3
    buf = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    off2 = np.zeros(25, dtype=np.int64)
    ctx._sync_stream()
    rc = ctx.lib.spade_batch_select(ctx.handle, b.handle, t.handle, ctypes.c_void_p(buf.data_ptr()), cap,
                                    off2.ctypes.data_as(ctypes.c_void_p))
    assert rc == spade.SPADE_E_CAPACITY
    assert np.array_equal(off2, off)
    assert np.array_equal(buf.cpu().numpy().astype(np.uint32), full[:cap])
    b.close()
    t.close()


def test_mem_info(ctx):
    m = ctx.mem_info()
    assert 0 < m["free"] <= m["total"]
    assert m["ctx"] >= 0
    f, t = torch.cuda.mem_get_info()
    assert m["total"] == t
