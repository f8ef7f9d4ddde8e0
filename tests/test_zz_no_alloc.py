"""spade_canvas_join_count_noalloc through the C ABI: the same counts as
spade_canvas_join_count on the same canvas and points, on two calls in a
row (the second with a smaller input), also after other work has used the
device, and its limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2203_14362_amd import spade
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _counts(lib, h, cv, dx, dy, fn, M):
    P = spade._Points(dx.numel(), dx.data_ptr(), dy.data_ptr())
    out = torch.full((M,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    rc = fn(h, cv, ctypes.byref(P), ctypes.c_void_p(out.data_ptr()))
    assert rc == 0, lib.spade_last_error(h)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("M", [300, 9000])     # LDS histogram and global-atomic probes
def test_noalloc_matches_allocating_call(M):
    lib = spade.load_library()
    h = ctypes.c_void_p()
    assert lib.spade_ctx_create(0, None, ctypes.byref(h)) == 0
    cv = ctypes.c_void_p()
    try:
        L = gen.EXTENT_M
        polys = gen.voronoi_jitter(M, 4, 40, seed=51 + M, L=L)
        dp = spade.DevicePolys(polys, torch.device("cuda", 0))
        torch.cuda.synchronize()
        assert lib.spade_canvas_build(h, ctypes.byref(dp.cstruct()), ctypes.byref(cv)) == 0, lib.spade_last_error(h)
        x, y = gen.mixture_points(3_000_000, seed=52, L=L)
        for n in (3_000_000, 777_777):                       # second call: smaller input
            dx, dy = _dev(x[:n]), _dev(y[:n])
            a = _counts(lib, h, cv, dx, dy, lib.spade_canvas_join_count_noalloc, M)
            b = _counts(lib, h, cv, dx, dy, lib.spade_canvas_join_count, M)
            assert np.array_equal(a, b), n
            assert int(a.sum()) == n
        assert np.array_equal(a, oracle.join_count(x[:777_777], y[:777_777], polys))
    finally:
        lib.spade_canvas_destroy(cv)
        lib.spade_ctx_destroy(h)


def test_noalloc_limit():
    lib = spade.load_library()
    h = ctypes.c_void_p()
    assert lib.spade_ctx_create(0, None, ctypes.byref(h)) == 0
    cv = ctypes.c_void_p()
    try:
        rings = [[np.array([[i, 0.0], [i + 1.0, 0.0], [i + 1.0, 1.0], [i, 1.0]])] for i in range(65537)]
        polys = gen.polys_from_rings(rings)
        dp = spade.DevicePolys(polys, torch.device("cuda", 0))
        torch.cuda.synchronize()
        assert lib.spade_canvas_build(h, ctypes.byref(dp.cstruct()), ctypes.byref(cv)) == 0, lib.spade_last_error(h)
        dx, dy = _dev(np.array([0.5])), _dev(np.array([0.5]))
        P = spade._Points(1, dx.data_ptr(), dy.data_ptr())
        out = torch.empty(65537, dtype=torch.int64, device="cuda")
        rc = lib.spade_canvas_join_count_noalloc(h, cv, ctypes.byref(P), ctypes.c_void_p(out.data_ptr()))
        assert rc == spade.SPADE_E_UNSUPPORTED
        assert b"65536" in lib.spade_last_error(h)
    finally:
        lib.spade_canvas_destroy(cv)
        lib.spade_ctx_destroy(h)
