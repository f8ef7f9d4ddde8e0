"""Python binding of libspade.so: argument marshalling only.

Every step of a query (rasterisation, probing, exact tests, counting,
ordered compaction) runs in the library's HIP kernels.  torch supplies device
memory and the current stream.  The binding refuses to run without the
compiled library: there is no fallback implementation.

Polygon sets are dicts in CSR layout (see ``workloads.gen``) with host numpy
arrays or device tensors: ``n_polys``, ``poly_ring_off`` (or None),
``ring_vtx_off``, ``vx``, ``vy``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspade.so")

SPADE_OK = 0
SPADE_E_INVALID = -1
SPADE_E_CAPACITY = -2
SPADE_E_NOMEM = -3
SPADE_E_HIP = -4
SPADE_E_UNSUPPORTED = -5
SPADE_E_TOO_LARGE = -6

EXPORTS = [
    "spade_ctx_create", "spade_ctx_destroy", "spade_ctx_set_stream", "spade_last_error",
    "spade_ctx_set_canvas_size", "spade_select", "spade_join_count", "spade_join_pairs",
    "spade_canvas_build", "spade_canvas_destroy", "spade_canvas_info", "spade_canvas_select",
    "spade_canvas_join_count", "spade_canvas_join_count_async", "spade_canvas_join_pairs",
    "spade_orient_batch", "spade_ctx_set_timing", "spade_ctx_last_timing",
    "spade_table_create", "spade_table_destroy", "spade_table_info", "spade_batch_build",
    "spade_batch_select", "spade_batch_join_count", "spade_ctx_set_pixels_per_vertex",
    "spade_batch_rebuild", "spade_ctx_set_graphs", "spade_ctx_graph_stats", "spade_select_disk",
    "spade_ctx_build_stats", "spade_ctx_batch_stats", "spade_mem_info", "spade_canvas_join_count_noalloc",
    "spade_stream_read", "spade_batch_join_pairs", "spade_layer_index",
    "spade_layered_build", "spade_distance_join_pairs", "spade_distance_join_count", "spade_knn_select",
    "spade_host_table_create", "spade_host_table_destroy", "spade_host_table_info", "spade_host_join_count",
    "spade_host_select", "spade_batch_submit", "spade_batch_wait", "spade_job_query", "spade_job_free",
    "spade_select_near_lines", "spade_select_within_polygon", "spade_distance_join_lines_pairs",
    "spade_distance_join_lines_count",
]

JOB_SELECT, JOB_COUNT, JOB_PAIRS = 1, 2, 3


class SpadeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("spade error %d: %s" % (code, msg))
        self.code = code


class _Points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class _Disks(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cx", ctypes.c_void_p), ("cy", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("r_all", ctypes.c_double)]


class _JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_out", ctypes.c_int64), ("out0", ctypes.c_void_p),
                ("out1", ctypes.c_void_p), ("off", ctypes.POINTER(ctypes.c_int64)), ("n_off", ctypes.c_int64)]


class _DevArray:
    """A device array the library owns, seen by torch without a copy."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr or 0), False),
                                         "version": 2}


class _Polys(ctypes.Structure):
    _fields_ = [("n_polys", ctypes.c_int64), ("n_rings", ctypes.c_int64),
                ("poly_ring_off", ctypes.c_void_p), ("ring_vtx_off", ctypes.c_void_p),
                ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p), ("n_vertices", ctypes.c_int64),
                ("bbox", ctypes.c_void_p)]


_lib = None


def load_library():
    """Load libspade.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libspade.so is missing: build it with paper_2203_14362_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.spade_ctx_create.argtypes = [ctypes.c_int, vp, P(vp)]
    lib.spade_ctx_destroy.argtypes = [vp]
    lib.spade_ctx_destroy.restype = None
    lib.spade_ctx_set_stream.argtypes = [vp, vp]
    lib.spade_last_error.argtypes = [vp]
    lib.spade_last_error.restype = ctypes.c_char_p
    lib.spade_ctx_set_canvas_size.argtypes = [vp, i32, i32]
    lib.spade_select.argtypes = [vp, P(_Points), P(_Polys), vp, i64, P(i64)]
    lib.spade_select_disk.argtypes = [vp, P(_Points), ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, i64,
                                      P(i64)]
    lib.spade_select_near_lines.argtypes = [vp, P(_Points), P(_Polys), ctypes.c_double, vp, i64, P(i64)]
    lib.spade_select_within_polygon.argtypes = [vp, P(_Points), P(_Polys), ctypes.c_double, vp, i64, P(i64)]
    lib.spade_distance_join_lines_pairs.argtypes = [vp, P(_Points), P(_Polys), vp, ctypes.c_double, vp, vp, i64,
                                                    P(i64)]
    lib.spade_distance_join_lines_count.argtypes = [vp, P(_Points), P(_Polys), vp, ctypes.c_double, vp]
    lib.spade_join_count.argtypes = [vp, P(_Points), P(_Polys), vp]
    lib.spade_join_pairs.argtypes = [vp, P(_Points), P(_Polys), vp, vp, i64, P(i64)]
    lib.spade_canvas_build.argtypes = [vp, P(_Polys), P(vp)]
    lib.spade_canvas_destroy.argtypes = [vp]
    lib.spade_canvas_destroy.restype = None
    lib.spade_canvas_info.argtypes = [vp, P(i32), P(i32), P(i64), P(i64), P(i64)]
    lib.spade_canvas_select.argtypes = [vp, vp, P(_Points), vp, i64, P(i64)]
    lib.spade_canvas_join_count.argtypes = [vp, vp, P(_Points), vp]
    lib.spade_canvas_join_count_async.argtypes = [vp, vp, P(_Points), vp]
    lib.spade_canvas_join_count_noalloc.argtypes = [vp, vp, P(_Points), vp]
    lib.spade_canvas_join_pairs.argtypes = [vp, vp, P(_Points), vp, vp, i64, P(i64)]
    lib.spade_orient_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.spade_ctx_set_timing.argtypes = [vp, ctypes.c_int]
    lib.spade_ctx_last_timing.argtypes = [vp, P(ctypes.c_float), P(ctypes.c_float)]
    lib.spade_table_create.argtypes = [vp, P(_Points), P(vp)]
    lib.spade_table_destroy.argtypes = [vp]
    lib.spade_table_destroy.restype = None
    lib.spade_table_info.argtypes = [vp, P(i64), P(i32), P(i64), P(i64)]
    lib.spade_batch_build.argtypes = [vp, P(_Polys), i32, vp, P(vp)]
    lib.spade_batch_rebuild.argtypes = [vp, P(_Polys), i32, vp, vp]
    lib.spade_batch_select.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.spade_batch_join_count.argtypes = [vp, vp, vp, vp]
    lib.spade_ctx_set_pixels_per_vertex.argtypes = [vp, ctypes.c_double]
    lib.spade_ctx_set_graphs.argtypes = [vp, ctypes.c_int]
    lib.spade_ctx_graph_stats.argtypes = [vp, P(i64), P(i64)]
    lib.spade_ctx_build_stats.argtypes = [vp, P(i64), P(i64)]
    lib.spade_ctx_batch_stats.argtypes = [vp, P(i64)]
    lib.spade_batch_join_pairs.argtypes = [vp, vp, vp, vp, vp, i64, P(i64)]
    lib.spade_distance_join_pairs.argtypes = [vp, P(_Points), P(_Disks), vp, vp, i64, P(i64)]
    lib.spade_distance_join_count.argtypes = [vp, P(_Points), P(_Disks), vp]
    lib.spade_knn_select.argtypes = [vp, P(_Points), ctypes.c_double, ctypes.c_double, i64, vp, P(i64)]
    lib.spade_host_table_create.argtypes = [vp, vp, vp, i64, P(vp)]
    lib.spade_batch_submit.argtypes = [vp, vp, P(_Polys), i32, vp, vp, ctypes.c_int, P(vp)]
    lib.spade_batch_wait.argtypes = [vp, P(_JobResult)]
    lib.spade_job_query.argtypes = [vp]
    lib.spade_job_free.argtypes = [vp]
    lib.spade_job_free.restype = None
    lib.spade_host_table_destroy.argtypes = [vp]
    lib.spade_host_table_destroy.restype = None
    lib.spade_host_table_info.argtypes = [vp, P(i64), P(i32), P(i64)]
    lib.spade_host_join_count.argtypes = [vp, vp, P(_Polys), vp, P(i64)]
    lib.spade_host_select.argtypes = [vp, vp, P(_Polys), vp, i64, P(i64), P(i64)]
    lib.spade_layer_index.argtypes = [vp, P(_Polys), i32, vp, P(i32)]
    lib.spade_layered_build.argtypes = [vp, P(_Polys), i32, P(vp), P(i32)]
    lib.spade_stream_read.argtypes = [vp, P(_Points), ctypes.c_int, vp]
    lib.spade_mem_info.argtypes = [vp, P(ctypes.c_size_t), P(ctypes.c_size_t), P(ctypes.c_size_t)]
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int:
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return t.contiguous()


def _dev_i64(a, device):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.int64)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(device)
    return t.contiguous()


class DevicePolys:
    """A polygon set resident on the device, in the C ABI's CSR layout."""

    def __init__(self, polys, device):
        self.n_polys = int(polys["n_polys"])
        pro = polys.get("poly_ring_off")
        self.ring_vtx_off = _dev_i64(polys["ring_vtx_off"], device)
        self.n_rings = int(self.ring_vtx_off.numel()) - 1
        self.poly_ring_off = None if pro is None else _dev_i64(pro, device)
        self.vx = _dev_f64(polys["vx"], device)
        self.vy = _dev_f64(polys["vy"], device)
        # bounding box of host vertex arrays (the library checks it on the
        # device); device arrays are left to the library
        self._cs = None
        self.bbox = None
        hx, hy = polys["vx"], polys["vy"]
        if not isinstance(hx, torch.Tensor) and not isinstance(hy, torch.Tensor):
            hx = np.asarray(hx, dtype=np.float64)
            hy = np.asarray(hy, dtype=np.float64)
            if hx.size and hx.size == hy.size and np.all(np.isfinite(hx)) and np.all(np.isfinite(hy)):
                self.bbox = np.array([hx.min(), hx.max(), hy.min(), hy.max()], dtype=np.float64)

    @property
    def bbox(self):
        return self._bbox

    @bbox.setter
    def bbox(self, b):
        self._bbox = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        self._cs = None

    def cstruct(self):
        if self._cs is None:
            self._cs = _Polys(self.n_polys, self.n_rings,
                              0 if self.poly_ring_off is None else self.poly_ring_off.data_ptr(),
                              self.ring_vtx_off.data_ptr() if self.ring_vtx_off.numel() else 0,
                              self.vx.data_ptr() if self.vx.numel() else 0,
                              self.vy.data_ptr() if self.vy.numel() else 0,
                              int(self.vx.numel()),
                              None if self._bbox is None else self._bbox.ctypes.data)
        return self._cs


def _compact(buf, m):
    """The first m elements of an output buffer; copied out when they fill
    less than half of it, so a result never pins a much larger buffer."""
    return buf[:m] if 2 * m >= buf.numel() else buf[:m].clone()


def _ids(t, n):
    """Point ids come back as uint32; tensors of more than 2^31 - 1 points
    return them widened to int64 so that no id reads as negative."""
    if n <= 0x7FFFFFFF:
        return t
    return t.to(torch.int64) & 0xFFFFFFFF


def _points(x, y):
    if x.dtype != torch.float64 or y.dtype != torch.float64:
        raise TypeError("points must be float64 tensors")
    if x.shape != y.shape or x.dim() != 1:
        raise ValueError("x and y must be 1-D tensors of equal length")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("point arrays must be contiguous")
    n = x.numel()
    return _Points(n, x.data_ptr() if n else 0, y.data_ptr() if n else 0)


class Canvas:
    """A rasterised polygon set resident on the device."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle

    def info(self):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        m, nb, by = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.ctx.lib.spade_canvas_info(self.handle, ctypes.byref(w), ctypes.byref(h), ctypes.byref(m),
                                       ctypes.byref(nb), ctypes.byref(by))
        return {"width": w.value, "height": h.value, "n_polys": m.value,
                "boundary_pixels": nb.value, "device_bytes": by.value}

    def close(self):
        if self.handle:
            self.ctx.lib.spade_canvas_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Table:
    """Device-resident point table clustered by a grid (the library's copy)."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle

    def info(self):
        n, g, c, by = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        self.ctx.lib.spade_table_info(self.handle, ctypes.byref(n), ctypes.byref(g), ctypes.byref(c),
                                      ctypes.byref(by))
        return {"n_points": n.value, "grid": g.value, "chunks": c.value, "device_bytes": by.value}

    def close(self):
        if self.handle:
            self.ctx.lib.spade_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostTable:
    """Out-of-core point table: a clustered copy in pinned host memory,
    streamed to the device per query."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle
        self.last_streamed = 0

    def info(self):
        n, g, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        self.ctx.lib.spade_host_table_info(self.handle, ctypes.byref(n), ctypes.byref(g), ctypes.byref(b))
        return {"n_points": n.value, "grid": g.value, "host_bytes": b.value}

    def close(self):
        if self.handle:
            self.ctx.lib.spade_host_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Job:
    """An asynchronous batch job (spade_batch_submit).  ``wait`` returns
    tensors that own their memory: select -> (ids int32, offsets int64
    numpy), count -> int64 counts, pairs -> (point ids, polygon ids)."""

    def __init__(self, ctx: "Context", handle, kind, keep):
        self.ctx = ctx
        self.handle = handle
        self.kind = kind
        self._keep = keep            # polygon arrays, canvas set and table the job reads
        self._res = None

    def done(self) -> bool:
        return self._res is not None or self.ctx.lib.spade_job_query(self.handle) == 1

    def __del__(self):
        # a job dropped without wait: free the handle (after the job is done)
        # so its result buffer goes back to the context
        h = getattr(self, "handle", None)
        if h is not None and getattr(self.ctx, "handle", None) is not None:
            self.ctx.lib.spade_job_free(h)
            self.handle = None

    def wait(self):
        if self._res is not None:
            return self._res
        r = _JobResult()
        rc = self.ctx.lib.spade_batch_wait(self.handle, ctypes.byref(r))
        try:
            if rc != SPADE_OK:
                raise SpadeError(rc, self.ctx.lib.spade_last_error(self.ctx.handle).decode())
            dev = self.ctx.device
            n = int(r.n_out)
            # copies of the results first: the offsets live in the job handle,
            # the arrays in a buffer the context lends the job until it is freed
            with torch.cuda.device(dev):
                if self.kind == JOB_COUNT:
                    out = torch.as_tensor(_DevArray(r.out0, n, "<i8"), device=dev).clone()
                elif self.kind == JOB_SELECT:
                    off = np.ctypeslib.as_array(r.off, shape=(int(r.n_off),)).copy()
                    out = (torch.as_tensor(_DevArray(r.out0, n, "<i4"), device=dev).clone(), off)
                else:
                    out = (torch.as_tensor(_DevArray(r.out0, n, "<i4"), device=dev).clone(),
                           torch.as_tensor(_DevArray(r.out1, n, "<i4"), device=dev).clone())
                torch.cuda.current_stream(dev).synchronize()
        finally:
            self.ctx.lib.spade_job_free(self.handle)
            self.handle = None
            self._keep = None
        self._res = out
        return out


class Batch(Canvas):
    """A batch of queries rasterised as one canvas set."""

    def __init__(self, ctx: "Context", handle, qbound):
        super().__init__(ctx, handle)
        self.qbound = qbound
        self.n_queries = len(qbound) - 1
        self.n_polys = int(qbound[-1])
        self.last_total = None       # results of the last selection or join pairs over this set


class Context:
    """One spade_ctx bound to a device; calls run on torch's current stream."""

    def __init__(self, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        h = ctypes.c_void_p()
        rc = self.lib.spade_ctx_create(self.device.index, None, ctypes.byref(h))
        if rc != SPADE_OK:
            raise SpadeError(rc, "spade_ctx_create failed")
        self.handle = h
        self.timing_enabled = False
        self._select_cap = 1 << 20
        self._pairs_hint = {}        # id of a join's constraint set -> pairs of its last join (first capacity tried)

    # -- helpers
    def _check(self, rc):
        if rc != SPADE_OK:
            raise SpadeError(rc, self.lib.spade_last_error(self.handle).decode())

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device)
        self.lib.spade_ctx_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream))

    def set_canvas_size(self, width: int = 0, height: int = 0):
        self._check(self.lib.spade_ctx_set_canvas_size(self.handle, int(width), int(height)))

    def set_timing(self, on: bool = True):
        self._check(self.lib.spade_ctx_set_timing(self.handle, 1 if on else 0))
        self.timing_enabled = bool(on)

    def last_timing(self):
        """(raster_ms, probe_ms) of the last query (HIP events on its stream)."""
        r, p = ctypes.c_float(), ctypes.c_float()
        self._check(self.lib.spade_ctx_last_timing(self.handle, ctypes.byref(r), ctypes.byref(p)))
        return float(r.value), float(p.value)

    def set_graphs(self, on: bool = True):
        self._check(self.lib.spade_ctx_set_graphs(self.handle, 1 if on else 0))

    def graph_stats(self):
        """(graphs captured, replays launched) on this context."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.spade_ctx_graph_stats(self.handle, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def stream_read(self, x, y, shape: int = 0):
        """Sum of all coordinates via one plain read of the points (bandwidth
        reference; time it with the phase timer)."""
        self._sync_stream()
        P = _points(x, y)
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.spade_stream_read(self.handle, ctypes.byref(P), int(shape),
                                               ctypes.c_void_p(out.data_ptr())))
        return out

    def build_stats(self):
        """(plain-call canvas builds, builds redone for record capacity)."""
        b, r = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.spade_ctx_build_stats(self.handle, ctypes.byref(b), ctypes.byref(r)))
        return b.value, r.value

    def batch_stats(self) -> int:
        """(table chunk, query) overlaps of the last batch selection or join
        pairs on this context."""
        o = ctypes.c_int64()
        self._check(self.lib.spade_ctx_batch_stats(self.handle, ctypes.byref(o)))
        return o.value

    def mem_info(self):
        """{'free', 'total', 'ctx'}: device bytes free and in total, and the
        scratch bytes this context holds."""
        f, t, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.spade_mem_info(self.handle, ctypes.byref(f), ctypes.byref(t), ctypes.byref(c)))
        return {"free": f.value, "total": t.value, "ctx": c.value}

    def set_pixels_per_vertex(self, ppv: float):
        self._check(self.lib.spade_ctx_set_pixels_per_vertex(self.handle, float(ppv)))
        self._ppv = float(ppv)

    def pixels_per_vertex(self) -> float:
        """The automatic canvas sizing's pixels per polygon vertex."""
        return getattr(self, "_ppv", 256.0)

    def polys(self, polys):
        return polys if isinstance(polys, DevicePolys) else DevicePolys(polys, self.device)

    # -- resident tables and batches
    def table(self, x, y) -> Table:
        self._sync_stream()
        P = _points(x, y)
        h = ctypes.c_void_p()
        self._check(self.lib.spade_table_create(self.handle, ctypes.byref(P), ctypes.byref(h)))
        return Table(self, h)

    def batch(self, polys, qbound, into: "Batch" = None) -> Batch:
        """Rasterise queries [qbound[q], qbound[q+1]) of ``polys`` as one canvas
        set (into the memory of an existing set ``into`` when given)."""
        self._sync_stream()
        dp = self.polys(polys)
        qb = np.ascontiguousarray(qbound, dtype=np.int64)
        if into is not None:
            rc = self.lib.spade_batch_rebuild(self.handle, ctypes.byref(dp.cstruct()), int(qb.size - 1),
                                              qb.ctypes.data_as(ctypes.c_void_p), into.handle)
            if rc != SPADE_OK:
                into.close()
                self._check(rc)
            into.qbound, into.n_queries, into.n_polys = qb, int(qb.size - 1), int(qb[-1])
            return into
        h = ctypes.c_void_p()
        self._check(self.lib.spade_batch_build(self.handle, ctypes.byref(dp.cstruct()), int(qb.size - 1),
                                               qb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        return Batch(self, h, qb)

    def batch_select(self, batch: Batch, table: Table, cap=None):
        """(ids int32 tensor, offsets int64 numpy [nq + 1]): query q's ascending
        point ids are ids[off[q]:off[q+1]].  Without an explicit capacity the
        first attempt uses this set's last total (a rebuilt batch often
        selects as many), else the largest total seen on this context (at
        least 2^20, at most 2^28), and retries once at the reported total."""
        off = np.zeros(batch.n_queries + 1, dtype=np.int64)
        if cap is None:
            cap = getattr(batch, "last_total", None) or min(self._select_cap, 1 << 28)
        while True:
            ids = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            self._sync_stream()
            rc = self.lib.spade_batch_select(self.handle, batch.handle, table.handle,
                                             ctypes.c_void_p(ids.data_ptr()), cap,
                                             off.ctypes.data_as(ctypes.c_void_p))
            if rc == SPADE_E_CAPACITY:
                cap = int(off[-1])
                self._select_cap = max(self._select_cap, cap)
                continue
            self._check(rc)
            batch.last_total = int(off[-1])
            return _compact(ids, int(off[-1])), off

    def submit(self, batch: "Batch", polys, qbound, table: Table, kind: int) -> Job:
        """Asynchronous batch job on this context's worker thread: rebuild
        ``batch`` from ``polys`` / ``qbound`` and evaluate it over ``table``
        (``polys`` None: evaluate ``batch`` as last built).  The result
        tensors are copies made on the current stream at wait."""
        self._sync_stream()
        h = ctypes.c_void_p()
        if polys is None:
            self._check(self.lib.spade_batch_submit(self.handle, batch.handle, None, 0, None, table.handle,
                                                    int(kind), ctypes.byref(h)))
            return Job(self, h, kind, (None, batch, table))
        dp = self.polys(polys)
        qb = np.ascontiguousarray(qbound, dtype=np.int64)
        self._check(self.lib.spade_batch_submit(self.handle, batch.handle, ctypes.byref(dp.cstruct()),
                                                int(qb.size - 1), qb.ctypes.data_as(ctypes.c_void_p),
                                                table.handle, int(kind), ctypes.byref(h)))
        batch.qbound, batch.n_queries, batch.n_polys = qb, int(qb.size - 1), int(qb[-1])
        return Job(self, h, kind, (dp, batch, table))

    def host_table(self, x, y) -> HostTable:
        """Out-of-core table from host float64 arrays."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        if x.shape != y.shape or x.ndim != 1:
            raise ValueError("x and y must be 1-D arrays of equal length")
        h = ctypes.c_void_p()
        self._sync_stream()
        self._check(self.lib.spade_host_table_create(self.handle, x.ctypes.data_as(ctypes.c_void_p),
                                                     y.ctypes.data_as(ctypes.c_void_p), x.size, ctypes.byref(h)))
        return HostTable(self, h)

    def host_join_count(self, table: HostTable, polys):
        dp = self.polys(polys)
        out = torch.empty(max(dp.n_polys, 1), dtype=torch.int64, device=self.device)
        st = ctypes.c_int64()
        self._sync_stream()
        self._check(self.lib.spade_host_join_count(self.handle, table.handle, ctypes.byref(dp.cstruct()),
                                                   ctypes.c_void_p(out.data_ptr()), ctypes.byref(st)))
        table.last_streamed = st.value
        return out[:dp.n_polys]

    def host_select(self, table: HostTable, poly, cap=None):
        """Ids of the table's points inside one polygon, ascending.  The
        default capacity is the table's point count, so that the points are
        streamed once (a capacity shortfall would stream them again)."""
        dp = self.polys(poly)
        n = table.info()["n_points"]
        if cap is None:
            cap = max(1, n)
        while True:
            out = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout, st = ctypes.c_int64(), ctypes.c_int64()
            self._sync_stream()
            rc = self.lib.spade_host_select(self.handle, table.handle, ctypes.byref(dp.cstruct()),
                                            ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(nout), ctypes.byref(st))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            table.last_streamed = st.value
            return _ids(_compact(out, int(nout.value)), n)

    def batch_join_pairs(self, batch: Batch, table: Table, cap=None):
        """(point ids, polygon ids) int32 tensors of every pair of a table
        point inside a polygon of the canvas set, ascending by (point,
        polygon); polygon ids of a layered set are the caller's.  The first
        capacity tried is chosen as in batch_select."""
        if cap is None:
            cap = getattr(batch, "last_total", None) or min(self._select_cap, 1 << 28)
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            pg = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout = ctypes.c_int64()
            self._sync_stream()
            rc = self.lib.spade_batch_join_pairs(self.handle, batch.handle, table.handle,
                                                 ctypes.c_void_p(pt.data_ptr()), ctypes.c_void_p(pg.data_ptr()),
                                                 cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                self._select_cap = max(self._select_cap, cap)
                continue
            self._check(rc)
            m = int(nout.value)
            batch.last_total = m
            return _compact(pt, m), _compact(pg, m)

    def layer_index(self, polys, res: int = 0):
        """(layer of each polygon as an int32 tensor, number of layers)."""
        self._sync_stream()
        dp = self.polys(polys)
        out = torch.empty(max(dp.n_polys, 1), dtype=torch.int32, device=self.device)
        n = ctypes.c_int32()
        self._check(self.lib.spade_layer_index(self.handle, ctypes.byref(dp.cstruct()), int(res),
                                               ctypes.c_void_p(out.data_ptr()), ctypes.byref(n)))
        return out[:dp.n_polys], int(n.value)

    def layered(self, polys, res: int = 0) -> "Batch":
        """A canvas set with one canvas per layer of the polygon set, for the
        batch join calls over a table."""
        self._sync_stream()
        dp = self.polys(polys)
        h = ctypes.c_void_p()
        n = ctypes.c_int32()
        self._check(self.lib.spade_layered_build(self.handle, ctypes.byref(dp.cstruct()), int(res), ctypes.byref(h),
                                                 ctypes.byref(n)))
        b = Batch(self, h, np.array([0, dp.n_polys], dtype=np.int64))
        b.n_layers = int(n.value)
        return b

    def batch_join_count(self, batch: Batch, table: Table, out=None):
        """Per-polygon counts of the batch's polygon set (int64 tensor)."""
        self._sync_stream()
        if out is None:
            out = torch.empty(batch.n_polys, dtype=torch.int64, device=self.device)
        self._check(self.lib.spade_batch_join_count(self.handle, batch.handle, table.handle,
                                                    ctypes.c_void_p(out.data_ptr() if batch.n_polys else 0)))
        return out

    # -- canvases
    def canvas(self, polys) -> Canvas:
        self._sync_stream()
        dp = self.polys(polys)
        h = ctypes.c_void_p()
        self._check(self.lib.spade_canvas_build(self.handle, ctypes.byref(dp.cstruct()), ctypes.byref(h)))
        return Canvas(self, h)

    # -- queries
    def join_count(self, x, y, polys_or_canvas, out=None, sync=True):
        """Per-polygon counts as an int64 tensor (values are the uint64 counts)."""
        self._sync_stream()
        P = _points(x, y)
        if isinstance(polys_or_canvas, Canvas):
            M = polys_or_canvas.info()["n_polys"]
        else:
            dp = self.polys(polys_or_canvas)
            M = dp.n_polys
        if out is None:
            out = torch.empty(M, dtype=torch.int64, device=self.device)
        optr = out.data_ptr() if M else 0
        if isinstance(polys_or_canvas, Canvas):
            fn = self.lib.spade_canvas_join_count if sync else self.lib.spade_canvas_join_count_async
            self._check(fn(self.handle, polys_or_canvas.handle, ctypes.byref(P), ctypes.c_void_p(optr)))
        else:
            self._check(self.lib.spade_join_count(self.handle, ctypes.byref(P),
                                                  ctypes.byref(dp.cstruct()), ctypes.c_void_p(optr)))
        return out

    def _hint_cap(self, n, key):
        """First capacity of a join: the point count or the last join's
        total with the same constraint set, whichever is larger."""
        return max(n, 1, self._pairs_hint.get(key, 0))

    def _remember_pairs(self, key, m):
        if len(self._pairs_hint) >= 64 and key not in self._pairs_hint:
            self._pairs_hint.pop(next(iter(self._pairs_hint)))
        self._pairs_hint[key] = m

    def _emit(self, x, y, target, pairs, cap):
        P = _points(x, y)
        n = P.n
        if cap is None:
            # a selection has at most n results; join pairs can have more
            # (overlapping polygons): the last join with the same polygons
            # gives the first capacity tried, so that repeated joins run once
            cap = max(n, 1)
            if pairs:
                cap = max(cap, getattr(target, "last_pairs", 0)) if isinstance(target, Canvas) else \
                    self._hint_cap(n, id(target))
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            pg = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device) if pairs else None
            nout = ctypes.c_int64()
            self._sync_stream()
            if isinstance(target, Canvas):
                if pairs:
                    rc = self.lib.spade_canvas_join_pairs(self.handle, target.handle, ctypes.byref(P),
                                                          ctypes.c_void_p(pt.data_ptr()),
                                                          ctypes.c_void_p(pg.data_ptr()), cap,
                                                          ctypes.byref(nout))
                else:
                    rc = self.lib.spade_canvas_select(self.handle, target.handle, ctypes.byref(P),
                                                      ctypes.c_void_p(pt.data_ptr()), cap, ctypes.byref(nout))
            else:
                dp = self.polys(target)
                if pairs:
                    rc = self.lib.spade_join_pairs(self.handle, ctypes.byref(P), ctypes.byref(dp.cstruct()),
                                                   ctypes.c_void_p(pt.data_ptr()), ctypes.c_void_p(pg.data_ptr()),
                                                   cap, ctypes.byref(nout))
                else:
                    rc = self.lib.spade_select(self.handle, ctypes.byref(P), ctypes.byref(dp.cstruct()),
                                               ctypes.c_void_p(pt.data_ptr()), cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            m = int(nout.value)
            if pairs:
                if isinstance(target, Canvas):
                    target.last_pairs = m
                else:
                    self._remember_pairs(id(target), m)
            return (_ids(_compact(pt, m), n), _compact(pg, m)) if pairs else _ids(_compact(pt, m), n)

    def select(self, x, y, poly_or_canvas, cap=None):
        """Ascending ids of the points inside the one polygon (int32 tensor;
        int64 when there are more than 2^31 - 1 points)."""
        return self._emit(x, y, poly_or_canvas, False, cap)

    def select_disk(self, x, y, cx, cy, r, cap=None):
        """Ascending ids (int32 tensor) of the points within distance r of
        (cx, cy), closed disk, decided exactly."""
        P = _points(x, y)
        if cap is None:
            cap = max(P.n, 1)
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout = ctypes.c_int64()
            self._sync_stream()
            rc = self.lib.spade_select_disk(self.handle, ctypes.byref(P), float(cx), float(cy), float(r),
                                            ctypes.c_void_p(pt.data_ptr()), cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            return _ids(_compact(pt, int(nout.value)), P.n)

    def _select_dist(self, fn, x, y, polys, r, cap):
        P = _points(x, y)
        dp = self.polys(polys)
        if cap is None:
            cap = max(P.n, 1)
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout = ctypes.c_int64()
            self._sync_stream()
            rc = fn(self.handle, ctypes.byref(P), ctypes.byref(dp.cstruct()), float(r),
                    ctypes.c_void_p(pt.data_ptr()), cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            return _ids(_compact(pt, int(nout.value)), P.n)

    def select_near_lines(self, x, y, lines, r, cap=None):
        """Ascending ids of the points within closed distance r of a segment
        of `lines` (every ring of the CSR set an open polyline), decided
        exactly."""
        return self._select_dist(self.lib.spade_select_near_lines, x, y, lines, r, cap)

    def _line_radii(self, r):
        if np.ndim(r) == 0 and not isinstance(r, torch.Tensor):
            return None, float(r)
        return _dev_f64(r, self.device), 0.0

    def distance_join_lines(self, x, y, lines, r, cap=None):
        """(point ids, line ids) int32 tensors, ascending by (point, line), of
        every point within r (a scalar, or one distance per line) of each ring
        of `lines` taken as an open polyline, decided exactly."""
        P = _points(x, y)
        dl = self.polys(lines)
        rr, r_all = self._line_radii(r)
        key = (id(lines), id(r))
        if cap is None:
            cap = self._hint_cap(P.n, key)
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            pl = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout = ctypes.c_int64()
            self._sync_stream()
            rc = self.lib.spade_distance_join_lines_pairs(
                self.handle, ctypes.byref(P), ctypes.byref(dl.cstruct()),
                None if rr is None else ctypes.c_void_p(rr.data_ptr()), r_all, ctypes.c_void_p(pt.data_ptr()),
                ctypes.c_void_p(pl.data_ptr()), cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            m = int(nout.value)
            self._remember_pairs(key, m)
            return _ids(_compact(pt, m), P.n), _compact(pl, m)

    def distance_join_lines_count(self, x, y, lines, r):
        """Per-line counts (int64) of the points within each line's distance."""
        P = _points(x, y)
        dl = self.polys(lines)
        rr, r_all = self._line_radii(r)
        out = torch.empty(max(dl.n_rings, 1), dtype=torch.int64, device=self.device)
        self._sync_stream()
        self._check(self.lib.spade_distance_join_lines_count(
            self.handle, ctypes.byref(P), ctypes.byref(dl.cstruct()),
            None if rr is None else ctypes.c_void_p(rr.data_ptr()), r_all, ctypes.c_void_p(out.data_ptr())))
        return out[:dl.n_rings]

    def select_within(self, x, y, poly, r, cap=None):
        """Ascending ids of the points inside the one polygon or within
        closed distance r of one of its edges, decided exactly."""
        return self._select_dist(self.lib.spade_select_within_polygon, x, y, poly, r, cap)

    def _disks(self, cx, cy, r):
        cx = _dev_f64(cx, self.device)
        cy = _dev_f64(cy, self.device)
        if np.ndim(r) == 0 and not isinstance(r, torch.Tensor):
            rr, r_all = None, float(r)
        else:
            rr, r_all = _dev_f64(r, self.device), 0.0
        keep = (cx, cy, rr)
        n = cx.numel()
        D = _Disks(n, cx.data_ptr() if n else 0, cy.data_ptr() if n else 0,
                   None if rr is None else (rr.data_ptr() if n else 0), r_all)
        return D, keep

    def distance_join(self, x, y, cx, cy, r, cap=None):
        """(point ids, disk ids) of every point within distance r (a scalar:
        type (1); one radius per disk: type (2)) of a disk centre, ascending
        by (point, disk); closed disks, decided exactly."""
        P = _points(x, y)
        D, keep = self._disks(cx, cy, r)
        key = (id(cx), id(cy), id(r))
        if cap is None:
            cap = self._hint_cap(P.n, key)
        while True:
            pt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            pd = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            nout = ctypes.c_int64()
            self._sync_stream()
            rc = self.lib.spade_distance_join_pairs(self.handle, ctypes.byref(P), ctypes.byref(D),
                                                    ctypes.c_void_p(pt.data_ptr()), ctypes.c_void_p(pd.data_ptr()),
                                                    cap, ctypes.byref(nout))
            if rc == SPADE_E_CAPACITY:
                cap = int(nout.value)
                continue
            self._check(rc)
            m = int(nout.value)
            self._remember_pairs(key, m)
            return _ids(_compact(pt, m), P.n), _compact(pd, m)

    def distance_join_count(self, x, y, cx, cy, r):
        """Points within each disk (int64 tensor [number of disks])."""
        P = _points(x, y)
        D, keep = self._disks(cx, cy, r)
        out = torch.empty(max(D.n, 1), dtype=torch.int64, device=self.device)
        self._sync_stream()
        self._check(self.lib.spade_distance_join_count(self.handle, ctypes.byref(P), ctypes.byref(D),
                                                       ctypes.c_void_p(out.data_ptr())))
        return out[:D.n]

    def knn(self, x, y, px, py, k):
        """Ids of the k points nearest to (px, py), nearest first (equal
        distances by ascending id); exact."""
        P = _points(x, y)
        out = torch.empty(max(int(k), 1), dtype=torch.int32, device=self.device)
        nout = ctypes.c_int64()
        self._sync_stream()
        self._check(self.lib.spade_knn_select(self.handle, ctypes.byref(P), float(px), float(py), int(k),
                                              ctypes.c_void_p(out.data_ptr()), ctypes.byref(nout)))
        return _ids(out[:int(nout.value)], P.n)

    def join_pairs(self, x, y, polys_or_canvas, cap=None):
        """(point ids, polygon ids) int32 tensors, ascending by (point, polygon)."""
        return self._emit(x, y, polys_or_canvas, True, cap)

    def orient(self, a, b, c):
        """Device exact orientation signs for (n,2) float64 tensors a, b, c."""
        self._sync_stream()
        a = a.to(self.device, torch.float64).contiguous()
        b = b.to(self.device, torch.float64).contiguous()
        c = c.to(self.device, torch.float64).contiguous()
        cols = [t[:, i].contiguous() for t in (a, b, c) for i in (0, 1)]
        n = a.shape[0]
        out = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._check(self.lib.spade_orient_batch(self.handle, n, *[ctypes.c_void_p(t.data_ptr()) for t in cols],
                                                ctypes.c_void_p(out.data_ptr())))
        return out[:n]

    def close(self):
        if getattr(self, "handle", None):
            self.lib.spade_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
