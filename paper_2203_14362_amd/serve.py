"""Continuous-batching query server over a device-resident point table.

Requests (a selection with one polygon, or a join-count with a polygon set)
arrive at any time.  A dispatcher admits them in arrival order while their
estimated device memory fits the budget left by the requests in flight, and
hands each admitted group to the next free worker as one batch; requests
that arrive while batches are running join the next batch (continuous
batching).  Each worker owns a library context on its own HIP stream, so
the batches of different workers overlap on the device.  Every request
records its arrival, admission and completion times; ``latency_stats``
reports p50 / p99 from arrival to result-ready.

The scheduling logic is independent of the device: ``Server`` drives any
executor with ``n_workers`` and ``estimate(req)`` that either runs a batch
synchronously (``run(worker, reqs)``, one host thread per worker) or
submits it asynchronously (``submit(worker, reqs)`` returning a token,
``poll(token)``, ``collect(token)``): then the dispatcher submits and one
completion thread collects, and no host thread blocks in a device call.
``SpadeExecutor`` is the device executor: one canvas set per worker and
kind, evaluated by the library's asynchronous batch jobs over the shared
resident table.  Requests may carry a ``key`` naming their polygon set (equal
keys, equal polygons): a batch holding one keyed request keeps its canvas set
in a small per-worker cache, and a later such batch with the same key is
evaluated on it without rasterising again.

Admission counts device memory three ways against one budget: the estimates
of the requests in flight, the bytes of finished results the caller still
holds (released when the result tensor is garbage-collected), and what the
executor keeps resident (canvas sets, scratch, result buffers; asked after
every batch).
"""
from __future__ import annotations

import collections
import threading
import time
import weakref
from dataclasses import dataclass
from typing import Any, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    kind: str                      # "select" (one polygon) or "count"
    polys: dict                    # host CSR polygon set
    arrival: Optional[float] = None
    admitted: Optional[float] = None
    done: Optional[float] = None
    batch: Optional[int] = None
    worker: Optional[int] = None
    est_bytes: int = 0
    result: Any = None             # select: int32 ids; count: int64 counts
    error: Optional[str] = None
    result_size: Optional[int] = None   # when the server does not keep results
    key: Any = None                # names the polygon set (equal keys, equal polygons); None: not cached

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None or self.arrival is None else self.done - self.arrival


def n_vertices(polys) -> int:
    return int(np.asarray(polys["ring_vtx_off"])[-1])


def concat_sets(sets):
    """One CSR polygon set holding `sets` one after another, and the
    polygon offsets of each input set ([len(sets) + 1])."""
    pro, rvo, vx, vy = [np.zeros(1, np.int64)], [np.zeros(1, np.int64)], [], []
    bounds = [0]
    nr = nv = npoly = 0
    for p in sets:
        r = np.asarray(p["ring_vtx_off"], dtype=np.int64)
        m = int(p["n_polys"])
        pr = p.get("poly_ring_off")
        pr = np.arange(m + 1, dtype=np.int64) if pr is None else np.asarray(pr, dtype=np.int64)
        pro.append(pr[1:] + nr)
        rvo.append(r[1:] + nv)
        vx.append(np.asarray(p["vx"], dtype=np.float64))
        vy.append(np.asarray(p["vy"], dtype=np.float64))
        nr += r.size - 1
        nv += int(r[-1])
        npoly += m
        bounds.append(npoly)
    out = {"n_polys": npoly, "poly_ring_off": np.concatenate(pro), "ring_vtx_off": np.concatenate(rvo),
           "vx": np.concatenate(vx) if vx else np.zeros(0), "vy": np.concatenate(vy) if vy else np.zeros(0)}
    return out, np.asarray(bounds, dtype=np.int64)


class Server:
    """Arrival-ordered admission by memory budget + continuous batching."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 1024,
                 max_batch_vertices: int = 8_000_000, clock=time.perf_counter, keep_results: bool = True):
        self.ex = executor
        self.keep_results = keep_results  # False: record result sizes, drop the results
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_batch_vertices = max_batch_vertices
        self.clock = clock
        self._cv = threading.Condition()
        self._pending = collections.deque()
        self._free = list(range(executor.n_workers))
        self._reserved = 0
        self._peak_reserved = 0
        self._inflight = 0
        self._stop = False
        self._nbatch = 0
        self._work = [collections.deque() for _ in range(executor.n_workers)]
        self.done: List[Request] = []
        self.batches: List[List[int]] = []
        self._threads = []
        self._async = hasattr(executor, "submit")
        self._inflight_jobs = []          # async mode: (worker, batch, extra, token)
        self._held = 0                    # bytes of finished results still referenced
        self._resident = int(getattr(executor, "resident_bytes", lambda: 0)())
        self.peak_accounted = 0
        self.mem_trace = []               # (time, reserved, held, resident) after every batch

    # -- public
    def start(self):
        self._threads = [threading.Thread(target=self._dispatch, daemon=True)]
        if self._async:
            self._threads.append(threading.Thread(target=self._reaper, daemon=True))
        else:
            self._threads += [threading.Thread(target=self._worker, args=(w,), daemon=True)
                              for w in range(self.ex.n_workers)]
        for t in self._threads:
            t.start()
        return self

    def submit(self, req: Request):
        if req.arrival is None:
            req.arrival = self.clock()
        req.est_bytes = int(self.ex.estimate(req))
        with self._cv:
            self._pending.append(req)
            self._cv.notify_all()

    def drain(self, timeout: float = None):
        """Wait until every submitted request has completed."""
        t_end = None if timeout is None else time.monotonic() + timeout
        with self._cv:
            while self._pending or self._inflight:
                left = None if t_end is None else t_end - time.monotonic()
                if left is not None and left <= 0:
                    raise TimeoutError("requests still pending")
                self._cv.wait(left)

    def stop(self):
        """Finish every submitted request, then end the threads."""
        self.drain()
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    @property
    def peak_reserved(self) -> int:
        return self._peak_reserved

    @property
    def held_bytes(self) -> int:
        return self._held

    def accounted(self) -> int:
        """Device bytes admission counts now: in flight + held results +
        executor-resident (caller holds the lock or reads a snapshot)."""
        return self._reserved + self._held + self._resident

    # -- internals
    def _take_batch(self):
        """Requests admitted now, in arrival order (caller holds the lock)."""
        batch, verts, extra = [], 0, 0
        while self._pending and len(batch) < self.max_batch:
            r = self._pending[0]
            if r.est_bytes > self.budget:
                self._pending.popleft()
                r.error = "request needs about %d device bytes, above the budget of %d" % (r.est_bytes, self.budget)
                r.done = self.clock()
                self.done.append(r)
                continue
            v = n_vertices(r.polys)
            if self.accounted() + extra + r.est_bytes > self.budget:
                if not batch and self._inflight == 0:
                    # nothing in flight will free memory: only results the
                    # caller still holds stand in the way
                    self._pending.popleft()
                    r.error = ("device memory budget exhausted: %d bytes of results still held, %d resident"
                               % (self._held, self._resident))
                    r.done = self.clock()
                    self.done.append(r)
                    continue
                break                      # head waits for memory: no overtaking
            if batch and verts + v > self.max_batch_vertices:
                break
            self._pending.popleft()
            batch.append(r)
            verts += v
            extra += r.est_bytes
        return batch, extra

    def _dispatch(self):
        with self._cv:
            while True:
                if self._free and self._pending:
                    batch, extra = self._take_batch()
                    self._cv.notify_all()      # rejected requests may complete a drain
                    if batch:
                        self._launch(batch, extra)
                        continue
                    # the head waits for memory held by batches in flight (with
                    # nothing in flight the head always fits: its estimate was
                    # checked against the whole budget)
                if self._stop and not self._pending:
                    return
                self._cv.wait()

    def _launch(self, batch, extra):
        w = self._free.pop(0)
        now = self.clock()
        bid = self._nbatch
        self._nbatch += 1
        for r in batch:
            r.admitted, r.batch, r.worker = now, bid, w
        self._reserved += extra
        self._peak_reserved = max(self._peak_reserved, self._reserved)
        self._inflight += len(batch)
        self.batches.append([r.rid for r in batch])
        self.peak_accounted = max(self.peak_accounted, self.accounted())
        if self._async:
            try:
                token = self.ex.submit(w, batch)
            except Exception as e:          # nothing was queued: fail the batch at once
                token = ("error", e)
            self._inflight_jobs.append((w, batch, extra, token))
        else:
            self._work[w].append((batch, extra))
        self._cv.notify_all()

    def _worker(self, w):
        while True:
            with self._cv:
                while not self._work[w] and not self._stop:
                    self._cv.wait()
                if not self._work[w]:
                    return
                batch, extra = self._work[w].popleft()
            try:
                self.ex.run(w, batch)
            except Exception as e:
                # one bad request must not fail its batch: run them one by one
                for r in batch:
                    try:
                        if len(batch) == 1:
                            raise e
                        self.ex.run(w, [r])
                    except Exception as e1:
                        r.error = "%s: %s" % (type(e1).__name__, e1)
                        r.result = None
            self._finish(w, batch, extra)

    def _track(self, r):
        """Count a finished result as held until the caller drops it."""
        res = r.result
        parts = res if isinstance(res, tuple) else (res,)
        for t in parts:
            nb = int(getattr(t, "nbytes", 0) or 0)
            if nb <= 0:
                continue
            try:
                weakref.finalize(t, self._release, nb)
            except TypeError:
                continue
            self._held += nb

    def _release(self, nb):
        with self._cv:
            self._held -= nb
            self._cv.notify_all()

    def _finish(self, w, batch, extra):
        t = self.clock()
        resident = int(getattr(self.ex, "resident_bytes", lambda: 0)())
        with self._cv:
            for r in batch:
                r.done = t
                self.done.append(r)
                if r.error is None and r.result is not None:
                    if self.keep_results:
                        self._track(r)
                    else:
                        r.result_size = int(r.result.numel()) if hasattr(r.result, "numel") else 1
                        r.result = None
            self._reserved -= extra
            self._inflight -= len(batch)
            self._resident = resident
            self._free.append(w)
            self.mem_trace.append((t, self._reserved, self._held, self._resident))
            self._cv.notify_all()

    def _reaper(self):
        """Async mode: collects finished jobs in completion order."""
        idle = 1e-4
        while True:
            with self._cv:
                if self._stop and not self._inflight_jobs and not self._pending:
                    return
                jobs = list(self._inflight_jobs)
            ready = [j for j in jobs if not (isinstance(j[3], tuple) and j[3] and j[3][0] == "error") and
                     self.ex.poll(j[3])]
            failed = [j for j in jobs if isinstance(j[3], tuple) and j[3] and j[3][0] == "error"]
            if not ready and not failed:
                time.sleep(idle)
                continue
            for j in failed + ready:
                w, batch, extra, token = j
                with self._cv:
                    self._inflight_jobs.remove(j)
                try:
                    if j in failed:
                        raise token[1]
                    self.ex.collect(token, batch)
                except Exception as e:
                    # one bad request must not fail its batch: run them one by one
                    for r in batch:
                        try:
                            if len(batch) == 1:
                                raise e
                            self.ex.collect(self.ex.submit(w, [r]), [r])
                        except Exception as e1:
                            r.error = "%s: %s" % (type(e1).__name__, e1)
                            r.result = None
                self._finish(w, batch, extra)


def replay(server: Server, requests, arrivals, clock=time.perf_counter, sleep=time.sleep):
    """Submit requests at their arrival offsets (seconds from now), then wait
    for all of them.  Returns the wall time from the first arrival to the
    last completion."""
    t0 = clock()
    for r, a in zip(requests, arrivals):
        dt = t0 + a - clock()
        if dt > 0:
            sleep(dt)
        r.arrival = t0 + a
        server.submit(r)
    server.drain()
    return max(r.done for r in requests) - t0


def latency_stats(requests):
    lat = np.array([r.latency for r in requests if r.latency is not None and r.error is None])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}


class SpadeExecutor:
    """Device executor: workers with their own context and stream over one
    resident table.  A batch becomes at most two canvas sets (its selections,
    its join-counts) evaluated with the library's batch calls."""

    def __init__(self, x, y, n_workers: int = 2, device: int = 0, pixels_per_vertex: float = None,
                 cached_sets: int = 8):
        import torch
        from .spade import Context
        self.torch = torch
        self.n_workers = n_workers
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_workers)]
        self.ctxs = []
        for s in self.streams:
            with torch.cuda.stream(s):
                c = Context(device)
                if pixels_per_vertex:
                    c.set_pixels_per_vertex(pixels_per_vertex)
                self.ctxs.append(c)
        self.ppv = pixels_per_vertex or 256.0
        self._sets = [[None, None] for _ in range(n_workers)]
        # per worker: canvas sets of keyed batches, least recently used first
        self.cached_sets = int(cached_sets)
        self._cache = [collections.OrderedDict() for _ in range(n_workers)]
        self.cache_hits = 0
        self.cache_builds = 0
        self._resident_w = [0] * n_workers
        with torch.cuda.stream(self.streams[0]):
            self.table = self.ctxs[0].table(x, y)
        self.streams[0].synchronize()
        # coarse point histogram for output-size estimates
        self.n_points = int(x.numel())
        fin = torch.isfinite(x) & torch.isfinite(y)
        if self.n_points and bool(fin.any()):
            xf, yf = x[fin], y[fin]
            self.ext = (float(xf.min()), float(xf.max()), float(yf.min()), float(yf.max()))
            G = 128
            gx = ((xf - self.ext[0]) / max(self.ext[1] - self.ext[0], 1e-300) * G).clamp(0, G - 1).long()
            gy = ((yf - self.ext[2]) / max(self.ext[3] - self.ext[2], 1e-300) * G).clamp(0, G - 1).long()
            h = torch.bincount(gy * G + gx, minlength=G * G).reshape(G, G).cpu().numpy()
            self.hist = np.cumsum(np.cumsum(h, 0), 1)   # 2-D prefix sums
            self.G = G
        else:
            self.hist = None
        torch.cuda.synchronize(self.device)

    def _points_in_box(self, x0, x1, y0, y1) -> int:
        if self.hist is None:
            return 0
        X0, X1, Y0, Y1 = self.ext
        G = self.G
        c0 = int(np.clip(np.floor((x0 - X0) / max(X1 - X0, 1e-300) * G), 0, G - 1))
        c1 = int(np.clip(np.floor((x1 - X0) / max(X1 - X0, 1e-300) * G), 0, G - 1))
        r0 = int(np.clip(np.floor((y0 - Y0) / max(Y1 - Y0, 1e-300) * G), 0, G - 1))
        r1 = int(np.clip(np.floor((y1 - Y0) / max(Y1 - Y0, 1e-300) * G), 0, G - 1))
        H = self.hist
        tot = H[r1, c1]
        if r0 > 0:
            tot -= H[r0 - 1, c1]
        if c0 > 0:
            tot -= H[r1, c0 - 1]
        if r0 > 0 and c0 > 0:
            tot += H[r0 - 1, c0 - 1]
        return int(tot)

    def estimate(self, req: Request) -> int:
        """Device bytes a request holds while in flight (upper estimate):
        canvas words and coarse level (about three words per pixel), edges,
        their row entries and the boundary index sized from them (64-byte
        records), outputs."""
        V = n_vertices(req.polys)
        px = min(max(self.ppv * V, 64 * 64), 4096 * 4096)
        b = 12 * px + 1024 * V + (1 << 20)
        if req.kind == "select":
            if V:
                vx, vy = np.asarray(req.polys["vx"]), np.asarray(req.polys["vy"])
                b += 4 * self._points_in_box(vx.min(), vx.max(), vy.min(), vy.max())
        else:
            b += 8 * int(req.polys["n_polys"])
        return int(b)

    def submit(self, w: int, reqs: List[Request]):
        """Queues the batch's selections and join-counts as asynchronous jobs
        on worker w's context (its own stream and worker thread)."""
        from .spade import JOB_COUNT, JOB_SELECT
        torch = self.torch
        ctx, s = self.ctxs[w], self.streams[w]
        jobs = []
        with torch.cuda.stream(s):
            work = []
            for kind, code, slot in (("select", JOB_SELECT, 0), ("count", JOB_COUNT, 1)):
                rs = [r for r in reqs if r.kind == kind]
                if rs:
                    polys, qb = concat_sets([r.polys for r in rs])
                    # a batch of one keyed request keeps its set: combinations
                    # of several requests rarely come back
                    key = (kind, rs[0].key) if len(rs) == 1 and rs[0].key is not None else None
                    work.append((kind, code, slot, rs, polys, qb, key))
            # sets this worker lacks (its reusable ones, or a keyed batch's
            # set not cached yet) are built before its first job is queued (a
            # call on a context waits for the job it is running)
            cache = self._cache[w]
            for kind, code, slot, rs, polys, qb, key in work:
                if key is not None and self.cached_sets > 0:
                    if key in cache:
                        cache.move_to_end(key)
                        self.cache_hits += 1
                    else:
                        cache[key] = ctx.batch(polys, qb)
                        self.cache_builds += 1
                        # the worker is free (its last batch was collected), so
                        # no job of its context still reads an evicted set
                        while len(cache) > self.cached_sets:
                            cache.popitem(last=False)[1].close()
                elif self._sets[w][slot] is None:
                    self._sets[w][slot] = ctx.batch(polys, qb)
            s.synchronize()
            for kind, code, slot, rs, polys, qb, key in work:
                if key is not None and self.cached_sets > 0:
                    jobs.append((kind, rs, qb, ctx.submit(cache[key], None, None, self.table, code)))
                else:
                    jobs.append((kind, rs, qb, ctx.submit(self._sets[w][slot], polys, qb, self.table, code)))
        return (w, jobs)

    def poll(self, token) -> bool:
        return all(j.done() for _, _, _, j in token[1])

    def collect(self, token, reqs: List[Request]):
        w, jobs = token
        torch = self.torch
        err = None
        with torch.cuda.stream(self.streams[w]):
            for kind, rs, qb, job in jobs:
                try:
                    res = job.wait()
                except Exception as e:      # every job is waited for, the first error raised
                    err = err or e
                    continue
                if kind == "select":
                    ids, off = res
                    for q, r in enumerate(rs):
                        r.result = ids[int(off[q]):int(off[q + 1])].clone()
                else:
                    for q, r in enumerate(rs):
                        r.result = res[int(qb[q]):int(qb[q + 1])].clone()
        self.streams[w].synchronize()
        self._measure_resident(w)
        if err is not None:
            raise err

    def _measure_resident(self, w: int):
        """Worker w's resident device bytes (its context is idle): scratch,
        job result buffers and canvas sets."""
        tot = self.ctxs[w].mem_info()["ctx"]
        for b in self._sets[w] + list(self._cache[w].values()):
            if b is not None:
                tot += b.info()["device_bytes"]
        self._resident_w[w] = int(tot)

    def resident_bytes(self) -> int:
        """Device bytes the executor keeps between batches (the table is
        counted at creation, outside the budget); each worker's share is
        measured when its last batch was collected."""
        return int(sum(self._resident_w))

    def run(self, w: int, reqs: List[Request]):
        torch = self.torch
        ctx, s = self.ctxs[w], self.streams[w]
        with torch.cuda.stream(s):
            sel = [r for r in reqs if r.kind == "select"]
            cnt = [r for r in reqs if r.kind == "count"]
            # one canvas set per worker and kind, rebuilt in place: no device
            # allocation or free (which would synchronise the device) per batch
            if sel:
                polys, qb = concat_sets([r.polys for r in sel])
                b = self._sets[w][0] = ctx.batch(polys, qb, into=self._sets[w][0])
                ids, off = ctx.batch_select(b, self.table)
                # each result owns its memory: a view would keep the whole
                # batch's id buffer alive for as long as any result lives
                for q, r in enumerate(sel):
                    r.result = ids[int(off[q]):int(off[q + 1])].clone()
            if cnt:
                polys, qb = concat_sets([r.polys for r in cnt])
                b = self._sets[w][1] = ctx.batch(polys, qb, into=self._sets[w][1])
                counts = ctx.batch_join_count(b, self.table)
                for q, r in enumerate(cnt):
                    r.result = counts[int(qb[q]):int(qb[q + 1])].clone()
        s.synchronize()

    def autotune(self, sample: List[Request], candidates=None):
        """Pick the canvas resolution (pixels per vertex) for every worker
        from timed batches of `sample` on worker 0; returns (ppv, {ppv: ms})."""
        import time as _time
        cands = tuple(candidates or (48.0, 96.0, 192.0, 384.0))
        times = {}
        for ppv in cands:
            self.ctxs[0].set_pixels_per_vertex(ppv)
            self.run(0, [Request(-1, r.kind, r.polys) for r in sample])   # warm
            best = None
            for _ in range(2):
                t0 = _time.perf_counter()
                self.run(0, [Request(-1, r.kind, r.polys) for r in sample])
                dt = (_time.perf_counter() - t0) * 1e3
                best = dt if best is None else min(best, dt)
            times[ppv] = best
        self.ppv = min(times, key=times.get)
        for c in self.ctxs:
            c.set_pixels_per_vertex(self.ppv)
        return self.ppv, times

    def close(self):
        for pair in self._sets:
            for b in pair:
                if b is not None:
                    b.close()
        for cache in self._cache:
            for b in cache.values():
                b.close()
            cache.clear()
        self.table.close()
        for c in self.ctxs:
            c.close()
