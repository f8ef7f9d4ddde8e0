"""CPU oracle for point-in-polygon selection, join pairs and join-count.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this; the product path never does.

The arithmetic lives in ``oracle.c`` (plain brute force, exact orientation
sign, OpenMP over points).  This module only compiles it with gcc and
marshals numpy arrays through ctypes.  ``micro.py`` holds an independent
exact-rational version for tiny inputs.

Polygon sets use the CSR layout shared by every caller in this repository:
``poly_ring_off`` [M+1] (or None: ring i is polygon i), ``ring_vtx_off``
[R+1], vertex coordinates ``vx``, ``vy`` (float64); rings are implicitly
closed and polygons combine their rings by even-odd parity.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    p = ctypes.c_void_p
    lib.orc_orient_sign.argtypes = [d] * 6
    lib.orc_orient_sign.restype = i32
    lib.orc_set_filter.argtypes = [i32]
    lib.orc_set_filter.restype = None
    lib.orc_set_grid.argtypes = [i32]
    lib.orc_set_grid.restype = None
    lib.orc_filter_grid.argtypes = [i64, p, p, p, p]
    lib.orc_filter_grid.restype = i32
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = i32
    lib.orc_inside.argtypes = [d, d, i64, p, p, p, p, i64]
    lib.orc_inside.restype = i32
    lib.orc_join_count.argtypes = [i64, p, p, i64, p, p, p, p, p]
    lib.orc_join_count.restype = None
    lib.orc_point_nmatch.argtypes = [i64, p, p, i64, p, p, p, p, p]
    lib.orc_point_nmatch.restype = None
    lib.orc_join_pairs.argtypes = [i64, p, p, i64, p, p, p, p, i64, p, p]
    lib.orc_join_pairs.restype = i64
    lib.orc_select.argtypes = [i64, p, p, i64, p, p, p, p, i64, i64, p]
    lib.orc_select.restype = i64
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Polys:
    """Keeps contiguous copies alive for the duration of a call."""

    def __init__(self, polys):
        self.M = int(polys["n_polys"])
        pro = polys.get("poly_ring_off")
        self.pro = None if pro is None else _i64(pro)
        self.rvo = _i64(polys["ring_vtx_off"])
        self.vx = _f64(polys["vx"])
        self.vy = _f64(polys["vy"])

    def args(self):
        return (self.M, _ptr(self.pro), _ptr(self.rvo), _ptr(self.vx), _ptr(self.vy))


def orient_sign(ax, ay, bx, by, cx, cy) -> int:
    """Exact sign of (b-a) x (c-a)."""
    return int(_load().orc_orient_sign(ax, ay, bx, by, cx, cy))


def set_filter(on: bool) -> None:
    """Test hook: False sends every orientation through the big-integer path."""
    _load().orc_set_filter(1 if on else 0)


def set_grid(on: bool) -> None:
    """Test hook: False replaces the uniform-grid candidate filter by one
    cell that lists every polygon (bounding-box rejects only)."""
    _load().orc_set_grid(1 if on else 0)


def filter_grid(polys) -> int:
    """Side of the candidate grid the oracle builds for a polygon set."""
    P = _Polys(polys)
    return int(_load().orc_filter_grid(*P.args()))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def inside(px, py, polys, k) -> bool:
    P = _Polys(polys)
    return bool(_load().orc_inside(float(px), float(py), *P.args(), int(k)))


def join_count(x, y, polys) -> np.ndarray:
    """Per-polygon counts (uint64[M])."""
    x, y = _f64(x), _f64(y)
    P = _Polys(polys)
    out = np.zeros(max(P.M, 1), dtype=np.uint64)
    _load().orc_join_count(x.size, _ptr(x), _ptr(y), *P.args(), _ptr(out))
    return out[:P.M]


def point_nmatch(x, y, polys) -> np.ndarray:
    """Number of polygons containing each point (int32[N])."""
    x, y = _f64(x), _f64(y)
    P = _Polys(polys)
    out = np.zeros(max(x.size, 1), dtype=np.int32)
    _load().orc_point_nmatch(x.size, _ptr(x), _ptr(y), *P.args(), _ptr(out))
    return out[:x.size]


def join_pairs(x, y, polys):
    """(pt uint32[], poly uint32[]) ascending by (pt, poly)."""
    x, y = _f64(x), _f64(y)
    P = _Polys(polys)
    lib = _load()
    total = lib.orc_join_pairs(x.size, _ptr(x), _ptr(y), *P.args(), 0, None, None)
    pt = np.zeros(max(total, 1), dtype=np.uint32)
    pg = np.zeros(max(total, 1), dtype=np.uint32)
    lib.orc_join_pairs(x.size, _ptr(x), _ptr(y), *P.args(), total, _ptr(pt), _ptr(pg))
    return pt[:total], pg[:total]


def select(x, y, polys, k: int = 0) -> np.ndarray:
    """Ascending ids of the points inside polygon k (uint32[])."""
    x, y = _f64(x), _f64(y)
    P = _Polys(polys)
    lib = _load()
    total = lib.orc_select(x.size, _ptr(x), _ptr(y), *P.args(), int(k), 0, None)
    out = np.zeros(max(total, 1), dtype=np.uint32)
    lib.orc_select(x.size, _ptr(x), _ptr(y), *P.args(), int(k), total, _ptr(out))
    return out[:total]
