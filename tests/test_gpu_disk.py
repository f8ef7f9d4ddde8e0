"""Distance selection from a point on the GPU against the CPU oracle: the
closed disk, decided exactly, ids ascending.  Inputs are seeded synthetic
stand-ins; expected values come from ``oracle.disk`` only."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import disk
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _ids(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32).astype(np.int64)


@pytest.mark.parametrize("cx,cy,r", [(0.5, 0.5, 0.25), (0.1, 0.9, 0.05), (0.5, 0.5, 2.0), (5.0, 5.0, 0.5),
                                     (0.3, 0.3, 0.0), (0.0, 0.0, 1e-3)])
def test_uniform_points_match_oracle(ctx, cx, cy, r):
    # 200,001 points: 49 chunks of 4096 and a ragged tail
    x, y = gen.uniform_points(200_001, seed=71)
    got = _ids(ctx.select_disk(_dev(x), _dev(y), cx, cy, r))
    assert np.array_equal(got, disk.select_disk(x, y, cx, cy, r))


def test_points_on_and_around_the_circle(ctx):
    rng = np.random.default_rng(72)
    cx, cy, r = 0.1, -0.7, 0.3
    th = rng.uniform(0, 2 * np.pi, 30_000)
    x = cx + r * np.cos(th)
    y = cy + r * np.sin(th)
    x = np.concatenate([x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf), [cx + r, cx, np.nan, np.inf]])
    y = np.concatenate([y, y, y, [cy, cy - r, 0.0, cy]])
    got = _ids(ctx.select_disk(_dev(x), _dev(y), cx, cy, r))
    want = disk.select_disk(x, y, cx, cy, r)
    assert np.array_equal(got, want)
    assert 0 < want.size < x.size


def test_integer_lattice_on_the_circle(ctx):
    g = np.arange(-300, 301, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    for r in (5.0, 25.0, 65.0, 0.0, 300.0):
        got = _ids(ctx.select_disk(_dev(x), _dev(y), 0.0, 0.0, r))
        assert np.array_equal(got, disk.select_disk(x, y, 0.0, 0.0, r)), r


def test_clustered_points_full_size(ctx):
    """100M taxi-like clustered points, one disk around a cluster: every id."""
    L = gen.EXTENT_M
    x, y = gen.mixture_points(100_000_000, seed=2, L=L)
    cx, cy, r = float(np.median(x[:100_000])), float(np.median(y[:100_000])), 0.08 * L
    got = ctx.select_disk(_dev(x), _dev(y), cx, cy, r)
    want = disk.select_disk(x, y, cx, cy, r)
    assert got.numel() == want.size and want.size > 100_000
    assert np.array_equal(_ids(got), want)


def test_empty_input_capacity_and_invalid_arguments(ctx):
    from paper_2203_14362_amd import SpadeError
    from paper_2203_14362_amd.spade import SPADE_E_CAPACITY, SPADE_E_INVALID, _points
    x, y = gen.uniform_points(50_000, seed=73)
    dx, dy = _dev(x), _dev(y)
    assert ctx.select_disk(dx[:0], dy[:0], 0.5, 0.5, 0.3).numel() == 0
    want = disk.select_disk(x, y, 0.5, 0.5, 0.3)
    # too small a buffer: the call reports the size and writes the first
    # cap ids (two-step Map); the binding retries with the size
    P = _points(dx, dy)
    buf = torch.full((11,), -1, dtype=torch.int32, device="cuda")
    nout = ctypes.c_int64()
    rc = ctx.lib.spade_select_disk(ctx.handle, ctypes.byref(P), 0.5, 0.5, 0.3, ctypes.c_void_p(buf.data_ptr()),
                                   10, ctypes.byref(nout))
    torch.cuda.synchronize()
    assert rc == SPADE_E_CAPACITY and nout.value == want.size
    got = buf.cpu().numpy()
    assert np.array_equal(got[:10].astype(np.uint32), want[:10]) and got[10] == -1
    assert np.array_equal(_ids(ctx.select_disk(dx, dy, 0.5, 0.5, 0.3, cap=10)), want)
    for bad in [(0.5, 0.5, -1.0), (np.nan, 0.5, 0.1), (0.5, np.inf, 0.1), (0.5, 0.5, np.inf)]:
        with pytest.raises(SpadeError):
            ctx.select_disk(dx, dy, *bad)
    rc = ctx.lib.spade_select_disk(ctx.handle, ctypes.byref(P), 0.5, 0.5, 0.3, None, 10, ctypes.byref(nout))
    assert rc == SPADE_E_INVALID
    # the context still works
    assert np.array_equal(_ids(ctx.select_disk(dx, dy, 0.5, 0.5, 0.3)), want)
