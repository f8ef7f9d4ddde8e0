"""Layer index and layered joins on the GPU.

* The layer assignment equals an independent emulation of the paper's
  two-pass iteration (Sec. 5.5) on pixel-centre coverage computed by the
  CPU oracle's exact containment test.
* Joins over layered canvas sets (one canvas per layer, probed through the
  canvas-set path over a resident table) equal the oracle: counts and pairs,
  for overlapping stars mixed with a tessellation, at several index and
  canvas resolutions.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _grid(polys, res):
    vx, vy = polys["vx"], polys["vy"]
    x0, x1, y0, y1 = vx.min(), vx.max(), vy.min(), vy.max()
    w, h = x1 - x0, y1 - y0
    if w >= h:
        W, H = res, max(1, min(res, int(np.ceil(res * h / w))))
    else:
        H, W = res, max(1, min(res, int(np.ceil(res * w / h))))
    return x0, y0, W / w, H / h, W, H


def _emulated_layers(polys, res):
    """The paper's iteration on pixel-centre coverage from the oracle."""
    X0, Y0, sx, sy, W, H = _grid(polys, res)
    pp = dict(polys)
    pp["vx"] = (polys["vx"] - X0) * sx
    pp["vy"] = (polys["vy"] - Y0) * sy
    cy, cx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    pt, pg = oracle.join_pairs(cx.ravel(), cy.ravel(), pp)
    pt, pg = pt.astype(np.int64), pg.astype(np.int64)
    M = polys["n_polys"]
    layer = np.full(M, -1)
    it = 0
    while (layer < 0).any():
        rem = layer[pg] < 0
        cmax = np.full(W * H, -1)
        np.maximum.at(cmax, pt[rem], pg[rem])
        cropped = np.zeros(M, bool)
        bad = rem & (cmax[pt] != pg)
        cropped[pg[bad]] = True
        layer[(layer < 0) & ~cropped] = it
        it += 1
    return layer, it


def _overlap_set(seed, L=1.0, nstars=60):
    tess = gen.voronoi_jitter(30, 8, 40, seed=seed, L=L)
    stars, _ = gen.query_stars(nstars, 8, 400, seed=seed + 1, L=L, area=(2e-3, 8e-2), data_seed=seed)
    return gen.concat_polys(stars, tess)


@pytest.mark.parametrize("res", [1, 7, 128, 333])
def test_layer_index_matches_emulation(ctx, res):
    polys = _overlap_set(61)
    layer, n = ctx.layer_index(polys, res)
    want, wn = _emulated_layers(polys, res)
    assert n == wn
    assert np.array_equal(layer.cpu().numpy(), want)


def test_tessellation_is_one_layer(ctx):
    tess = gen.voronoi_jitter(400, 8, 64, seed=62, L=gen.EXTENT_M)
    layer, n = ctx.layer_index(tess, 2048)
    assert n == 1 and int(layer.max()) == 0


@pytest.fixture(scope="module")
def table_pts(ctx):
    x, y = gen.uniform_points(400_000, seed=63)
    t = ctx.table(_dev(x), _dev(y))
    yield x, y, t
    t.close()


@pytest.mark.parametrize("res,ppv", [(0, 0), (16, 64), (1024, 512), (4096, 16)])
def test_layered_join_matches_oracle(ctx, table_pts, res, ppv):
    x, y, t = table_pts
    polys = _overlap_set(64)
    if ppv:
        ctx.set_pixels_per_vertex(ppv)
    try:
        b = ctx.layered(polys, res)
    finally:
        ctx.set_pixels_per_vertex(256)
    assert b.n_layers > 1
    counts = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
    assert np.array_equal(counts, oracle.join_count(x, y, polys))
    pt, pg = ctx.batch_join_pairs(b, t)
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(pt.cpu().numpy().astype(np.uint32), opt)
    assert np.array_equal(pg.cpu().numpy().astype(np.uint32), opg)
    b.close()


def test_batch_join_pairs_on_a_plain_batch(ctx, table_pts):
    """Pairs over a batch canvas set (several queries, overlapping polygons)
    report positions in the concatenated polygon set."""
    x, y, t = table_pts
    polys = _overlap_set(65, nstars=20)
    M = polys["n_polys"]
    b = ctx.batch(polys, [0, 7, 20, M])
    pt, pg = ctx.batch_join_pairs(b, t)
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(pt.cpu().numpy().astype(np.uint32), opt)
    assert np.array_equal(pg.cpu().numpy().astype(np.uint32), opg)
    b.close()


def test_layered_degenerate(ctx, table_pts):
    x, y, t = table_pts
    empty = {"n_polys": 0, "poly_ring_off": None, "ring_vtx_off": np.zeros(1, np.int64),
             "vx": np.zeros(0), "vy": np.zeros(0)}
    layer, n = ctx.layer_index(empty)
    assert n == 0 and layer.numel() == 0
    tiny = gen.polys_from_rings([[np.array([[0.5, 0.5], [0.5 + 1e-9, 0.5], [0.5, 0.5 + 1e-9]])],
                                 [np.array([[0.1, 0.1], [0.9, 0.1], [0.9, 0.9], [0.1, 0.9]])]])
    layer, n = ctx.layer_index(tiny, 64)
    assert n == 1                          # the tiny one covers no pixel centre
    b = ctx.layered(tiny)
    counts = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
    assert np.array_equal(counts, oracle.join_count(x, y, tiny))
    b.close()


def test_batch_join_pairs_capacity_writes_first_cap(ctx, table_pts):
    """A capacity below the total: the first cap pairs of the (point,
    polygon) order are written and the total reported; with room for all of
    them every pair is written."""
    import ctypes
    from paper_2203_14362_amd import spade
    x, y, t = table_pts
    polys = _overlap_set(66, nstars=30)
    b = ctx.layered(polys)
    opt, opg = oracle.join_pairs(x, y, polys)
    for cap in (opt.size, opt.size + 7, opt.size // 3):
        bpt = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
        bpg = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
        n = ctypes.c_int64()
        ctx._sync_stream()
        rc = ctx.lib.spade_batch_join_pairs(ctx.handle, b.handle, t.handle, ctypes.c_void_p(bpt.data_ptr()),
                                            ctypes.c_void_p(bpg.data_ptr()), cap, ctypes.byref(n))
        assert n.value == opt.size
        assert rc == (spade.SPADE_OK if cap >= opt.size else spade.SPADE_E_CAPACITY)
        m = min(cap, opt.size)
        assert np.array_equal(bpt[:m].cpu().numpy().astype(np.uint32), opt[:m]), cap
        assert np.array_equal(bpg[:m].cpu().numpy().astype(np.uint32), opg[:m]), cap
    b.close()
