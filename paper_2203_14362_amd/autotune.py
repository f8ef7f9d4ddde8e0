"""Canvas-resolution autotuner.

The canvas resolution trades rasterisation against probing: a finer canvas
costs more rows to rasterise and more canvas words to write, a coarser one
sends more points to the exact boundary test.  The best point depends on
the polygons (vertex count, shape) and on the points (how many, where), so
it is measured instead of modelled: a few micro-trials of the real query at
candidate resolutions (pixels per polygon vertex), timed with the library's
own phase events, pick the fastest.  Results never depend on the choice
(every resolution is exact); only the time does.

Choices are cached per workload signature (polygon count, vertex count and
point count, each rounded to a power of two) in memory and, optionally, in
a JSON file, so a workload is tuned once.  A read-only preset table of
choices measured on MI355X ships with the package (``tuned_mi355x.json``);
entries of the writable cache take precedence over it, and ``force``
re-measures either.
"""
from __future__ import annotations

import json
import math
import os
import threading

DEFAULT_CANDIDATES = (32.0, 40.0, 48.0, 56.0, 64.0, 80.0, 96.0, 112.0, 128.0, 160.0, 192.0, 384.0)
PRESET_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def _bucket(n: int) -> int:
    return 0 if n <= 0 else int(round(math.log2(n)))


def signature(kind: str, n_polys: int, n_vertices: int, n_points: int) -> str:
    return "%s/p%d/v%d/n%d" % (kind, _bucket(n_polys), _bucket(n_vertices), _bucket(n_points))


class Autotuner:
    def __init__(self, path: str = None, candidates=DEFAULT_CANDIDATES, repeats: int = 3,
                 preset: str = PRESET_PATH):
        self.path = path
        self.candidates = tuple(float(c) for c in candidates)
        self.repeats = repeats
        self._lock = threading.Lock()
        self.table = {}
        self.preset = {}
        self.last_source = None
        if path and os.path.exists(path):
            with open(path) as fh:
                self.table = json.load(fh)
        if preset and os.path.exists(preset):
            with open(preset) as fh:
                self.preset = json.load(fh)

    def _save(self):
        if not self.path:
            return
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, key: str):
        with self._lock:
            e = self.table.get(key, self.preset.get(key))
        return None if e is None else float(e["ppv"])

    def tune(self, key: str, trial, force: bool = False):
        """Pick the fastest pixels-per-vertex for `key`.  ``trial(ppv)``
        runs the query once at that setting and returns its device time in
        milliseconds.  Returns (ppv, {ppv: best ms})."""
        if not force:
            with self._lock:
                self.last_source = "cache" if key in self.table else "preset" if key in self.preset else None
            hit = self.lookup(key)
            if hit is not None:
                return hit, {}
        times = {}
        for ppv in self.candidates:
            trial(ppv)                                   # warm: allocations, caches
            times[ppv] = min(trial(ppv) for _ in range(self.repeats))
        best = min(times, key=times.get)
        with self._lock:
            self.last_source = "measured"
            self.table[key] = {"ppv": best, "ms": {str(k): round(v, 4) for k, v in times.items()}}
            self._save()
        return best, times


def tune_join_count(ctx, x, y, polys, tuner: Autotuner = None, force: bool = False):
    """Tune and set ctx's pixels-per-vertex for join-counts of `polys` over
    the points (x, y): each trial is a whole join-count (rasterisation plus
    probe) timed by the library's events.  Returns (ppv, times)."""
    tuner = tuner or Autotuner()
    dp = ctx.polys(polys)
    nv = int(dp.ring_vtx_off[-1].item()) if dp.ring_vtx_off.numel() else 0
    key = signature("count", dp.n_polys, nv, int(x.numel()))
    was = ctx.timing_enabled

    def trial(ppv):
        ctx.set_pixels_per_vertex(ppv)
        ctx.join_count(x, y, dp)
        r, p = ctx.last_timing()
        return r + p

    ctx.set_timing(True)
    try:
        ppv, times = tuner.tune(key, trial, force=force)
    finally:
        ctx.set_timing(was)
    ctx.set_pixels_per_vertex(ppv)
    return ppv, times


SELECT_CANDIDATES = (96.0, 192.0, 384.0, 768.0, 1600.0)


def tune_select(ctx, x, y, poly, tuner: Autotuner = None, force: bool = False):
    """Tune and set ctx's pixels-per-vertex for selections with the one
    polygon `poly` over the points (x, y): each trial is a whole selection
    (rasterisation plus both probe passes) timed by the library's events.
    Returns (ppv, times)."""
    tuner = tuner or Autotuner(candidates=SELECT_CANDIDATES)
    dp = ctx.polys(poly)
    nv = int(dp.ring_vtx_off[-1].item()) if dp.ring_vtx_off.numel() else 0
    key = signature("select", dp.n_polys, nv, int(x.numel()))
    was = ctx.timing_enabled

    def trial(ppv):
        ctx.set_pixels_per_vertex(ppv)
        ctx.select(x, y, dp)
        r, p = ctx.last_timing()
        return r + p

    ctx.set_timing(True)
    try:
        ppv, times = tuner.tune(key, trial, force=force)
    finally:
        ctx.set_timing(was)
    ctx.set_pixels_per_vertex(ppv)
    return ppv, times


BATCH_SELECT_CANDIDATES = (12.0, 24.0, 48.0, 96.0)


def tune_batch_select(ctx, polys, qbound, table, tuner: Autotuner = None, force: bool = False):
    """Tune and set ctx's pixels-per-vertex for batch selections of the
    queries [qbound[q], qbound[q+1]) of `polys` over `table`: each trial
    rebuilds the batch's canvas set and selects, timed on the host around a
    device synchronisation (rasterisation, count pass, write pass and
    ordering).  Returns (ppv, times)."""
    import time
    import numpy as np
    import torch
    tuner = tuner or Autotuner(candidates=BATCH_SELECT_CANDIDATES, repeats=2)
    qb = np.asarray(qbound, dtype=np.int64)
    nv = int(np.asarray(polys["ring_vtx_off"])[-1]) if len(polys["ring_vtx_off"]) else 0
    key = signature("batch_select/q%d" % (qb.size - 1), int(polys["n_polys"]), nv, int(table.info()["n_points"]))
    state = {"b": None}

    def trial(ppv):
        ctx.set_pixels_per_vertex(ppv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        state["b"] = ctx.batch(polys, qb, into=state["b"])
        ids, off = ctx.batch_select(state["b"], table)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3
        del ids
        return dt

    try:
        ppv, times = tuner.tune(key, trial, force=force)
    finally:
        if state["b"] is not None:
            state["b"].close()
    ctx.set_pixels_per_vertex(ppv)
    return ppv, times
