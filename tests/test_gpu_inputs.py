"""GPU parity on inputs that stress the pixel map and the exact predicate:
the Web-Mercator-like offset frame at the full 100M-point size, canvases up
to 8192^2 in that frame, and the metamorphic transforms of the polygon set
(ring reversal, start-vertex rotation, polygon permutation, dyadic
translation and scaling), each compared with the oracle on the same
transformed inputs."""
import numpy as np
import pytest
import torch

import oracle
from workloads import configs, gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def offset_c2():
    x, y = configs.c2_points()
    polys = configs.c2_polys()
    return gen.offset_frame(x, y, polys)


def test_offset_frame_c2_counts_and_pairs_full(ctx, offset_c2):
    """100M clustered points and the 260 cells moved to (-8.27e6, 4.94e6):
    counts and every pair equal the oracle's."""
    x, y, polys = offset_c2
    dx, dy = _dev(x), _dev(y)
    got = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
    want = oracle.join_count(x, y, polys)
    assert np.array_equal(got, want) and int(want.sum()) == x.size
    pt, pg = ctx.join_pairs(dx, dy, polys)
    assert pt.numel() == x.size
    assert torch.equal(pt.to(torch.int64), torch.arange(x.size, device="cuda"))
    hist = torch.bincount(pg.to(torch.int64), minlength=260).cpu().numpy().astype(np.uint64)
    assert np.array_equal(hist, want)
    # every point's polygon: the oracle's pairs in full (one per point here)
    opt, opg = oracle.join_pairs(x, y, polys)
    assert np.array_equal(opt, np.arange(x.size, dtype=np.uint32))
    assert np.array_equal(pg.cpu().numpy().astype(np.uint32), opg)


@pytest.mark.parametrize("wh", [(1024, 1024), (4096, 4096), (8192, 8192), (8192, 1), (3, 8192)])
def test_offset_frame_resolutions(ctx, offset_c2, wh):
    x, y, polys = offset_c2
    n = 3_000_000
    xs, ys = x[:n], y[:n]
    want_pt, want_pg = oracle.join_pairs(xs, ys, polys)
    ctx.set_canvas_size(*wh)
    try:
        pt, pg = ctx.join_pairs(_dev(xs), _dev(ys), polys)
        cnt = ctx.join_count(_dev(xs), _dev(ys), polys).cpu().numpy().astype(np.uint64)
    finally:
        ctx.set_canvas_size(0, 0)
    assert np.array_equal(pt.cpu().numpy().astype(np.uint32), want_pt)
    assert np.array_equal(pg.cpu().numpy().astype(np.uint32), want_pg)
    assert np.array_equal(cnt, np.bincount(want_pg.astype(np.int64), minlength=260).astype(np.uint64))


def _ring_slices(polys):
    rvo = polys["ring_vtx_off"]
    return [(int(rvo[r]), int(rvo[r + 1])) for r in range(rvo.size - 1)]


def _map_rings(polys, fn):
    vx, vy = polys["vx"].copy(), polys["vy"].copy()
    for a, b in _ring_slices(polys):
        ix = fn(np.arange(a, b))
        vx[a:b], vy[a:b] = polys["vx"][ix], polys["vy"][ix]
    out = dict(polys)
    out["vx"], out["vy"] = vx, vy
    return out


def _permute(polys, perm):
    """Polygon set whose polygon k is the input's polygon perm[k] (one ring each)."""
    rvo = polys["ring_vtx_off"]
    rings = [[np.stack([polys["vx"][rvo[p]:rvo[p + 1]], polys["vy"][rvo[p]:rvo[p + 1]]], 1)] for p in perm]
    return gen.polys_from_rings(rings)


@pytest.fixture(scope="module")
def overl():
    """Overlapping stars plus a tessellation: points in several polygons."""
    x, y = gen.uniform_points(150_000, seed=41)
    tess = gen.voronoi_jitter(48, 8, 64, seed=41, L=1.0)
    stars, _ = gen.query_stars(40, 8, 300, seed=42, L=1.0, area=(1e-3, 5e-2), data_seed=41)
    polys = gen.concat_polys(tess, stars)
    # every coordinate on the 2^-30 grid, so that translating by 2^10 is exact
    q = 2.0 ** 30
    polys["vx"], polys["vy"] = np.round(polys["vx"] * q) / q, np.round(polys["vy"] * q) / q
    return np.round(x * q) / q, np.round(y * q) / q, polys


@pytest.mark.parametrize("kind", ["reverse", "rotate", "permute", "translate", "scale_up", "scale_down"])
def test_metamorphic_transforms(ctx, overl, kind):
    x, y, polys = overl
    M = polys["n_polys"]
    base_pt, base_pg = oracle.join_pairs(x, y, polys)
    if kind == "reverse":
        tp, tx, ty, perm = _map_rings(polys, lambda ix: ix[::-1]), x, y, np.arange(M)
    elif kind == "rotate":
        tp, tx, ty, perm = _map_rings(polys, lambda ix: np.roll(ix, 3)), x, y, np.arange(M)
    elif kind == "permute":
        perm = np.random.default_rng(43).permutation(M)
        tp, tx, ty = _permute(polys, perm), x, y
    else:
        s, d = {"translate": (1.0, 2.0 ** 10), "scale_up": (2.0 ** 20, 0.0), "scale_down": (2.0 ** -30, 0.0)}[kind]
        tp = dict(polys)
        tp["vx"], tp["vy"] = polys["vx"] * s + d, polys["vy"] * s - d
        tx, ty, perm = x * s + d, y * s - d, np.arange(M)
    # the oracle on the transformed inputs equals the original up to the permutation
    opt, opg = oracle.join_pairs(tx, ty, tp)
    inv = np.empty(M, np.int64)
    inv[perm] = np.arange(M)
    mapped = sorted(zip(base_pt.tolist(), inv[base_pg.astype(np.int64)].tolist()))
    assert list(zip(opt.tolist(), opg.tolist())) == mapped
    # and the GPU equals the oracle on the transformed inputs
    pt, pg = ctx.join_pairs(_dev(tx), _dev(ty), tp)
    assert np.array_equal(pt.cpu().numpy().astype(np.uint32), opt)
    assert np.array_equal(pg.cpu().numpy().astype(np.uint32), opg)
    cnt = ctx.join_count(_dev(tx), _dev(ty), tp).cpu().numpy().astype(np.uint64)
    assert np.array_equal(cnt, oracle.join_count(tx, ty, tp))
