"""Scheduling of the query server, on the CPU with a stand-in executor.

The executor sleeps for a time that grows with the request size and returns
a value computed from the request alone, so every property of the
scheduler (admission by memory budget, arrival order, continuous batching,
overlap of workers, error isolation) can be checked without a device.
"""
import threading
import time

import numpy as np
import pytest

from paper_2203_14362_amd.serve import Request, Server, concat_sets, latency_stats, n_vertices, replay


def _poly(nv, seed):
    rng = np.random.default_rng(seed)
    return {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, nv], np.int64),
            "vx": rng.random(nv), "vy": rng.random(nv)}


class FakeExecutor:
    def __init__(self, n_workers=2, bytes_per_vertex=1000, fail_on=None):
        self.n_workers = n_workers
        self.bpv = bytes_per_vertex
        self.fail_on = fail_on
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.reserved_seen = []

    def estimate(self, req):
        return self.bpv * n_vertices(req.polys)

    @staticmethod
    def answer(req):
        return float(np.sum(req.polys["vx"])) + req.rid

    def run(self, w, reqs):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        try:
            if self.fail_on is not None and any(r.rid == self.fail_on for r in reqs):
                raise ValueError("planted failure")
            time.sleep(0.004 + 2e-6 * sum(n_vertices(r.polys) for r in reqs))
            for r in reqs:
                r.result = self.answer(r)
        finally:
            with self.lock:
                self.active -= 1


def _requests(n, seed=0, vmin=8, vmax=2000):
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(vmin), np.log(vmax), n)).astype(int)
    return [Request(i, "select" if i % 2 else "count", _poly(int(v), i)) for i, v in enumerate(sizes)]


def test_concat_sets_offsets():
    a = {"n_polys": 2, "poly_ring_off": np.array([0, 1, 3]), "ring_vtx_off": np.array([0, 3, 6, 10]),
         "vx": np.arange(10.0), "vy": np.arange(10.0)}
    b = _poly(4, 1)
    out, bounds = concat_sets([a, b, a])
    assert bounds.tolist() == [0, 2, 3, 5]
    assert out["poly_ring_off"].tolist() == [0, 1, 3, 4, 5, 7]
    assert out["ring_vtx_off"].tolist() == [0, 3, 6, 10, 14, 17, 20, 24]
    assert np.array_equal(out["vx"][10:14], b["vx"])


def test_all_served_with_alone_results_and_ordering():
    ex = FakeExecutor()
    reqs = _requests(60)
    srv = Server(ex, budget_bytes=10**12).start()
    arrivals = np.cumsum(np.random.default_rng(1).exponential(1 / 400.0, len(reqs)))
    replay(srv, reqs, arrivals)
    srv.stop()
    assert len(srv.done) == len(reqs)
    for r in reqs:
        assert r.error is None
        assert r.result == FakeExecutor.answer(r)          # same as alone
        assert r.arrival <= r.admitted <= r.done
    # arrival order is kept: batch ids never decrease along arrivals
    assert all(reqs[i].batch <= reqs[i + 1].batch for i in range(len(reqs) - 1))
    # continuous batching: requests that queued behind running batches share one
    assert max(len(b) for b in srv.batches) > 1
    assert ex.max_active == 2                               # both workers overlapped
    st = latency_stats(reqs)
    assert st["n"] == len(reqs) and 0 < st["p50_ms"] <= st["p99_ms"]


def test_admission_by_memory_budget():
    ex = FakeExecutor(bytes_per_vertex=1000)
    reqs = _requests(40, seed=3, vmin=500, vmax=1000)
    budget = 1000 * 2500          # about three requests in flight at a time
    srv = Server(ex, budget_bytes=budget).start()
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert srv.peak_reserved <= budget
    assert all(r.error is None for r in reqs)
    assert max(len(b) for b in srv.batches) <= 3


def test_oversized_request_is_rejected_alone():
    ex = FakeExecutor(bytes_per_vertex=1000)
    reqs = _requests(10, seed=4, vmin=10, vmax=100)
    big = Request(99, "count", _poly(5000, 99))
    srv = Server(ex, budget_bytes=1000 * 1000).start()
    for r in reqs[:5] + [big] + reqs[5:]:
        srv.submit(r)
    srv.stop()
    assert big.error is not None and "budget" in big.error
    assert all(r.error is None and r.result == FakeExecutor.answer(r) for r in reqs)


def test_executor_failure_is_isolated_to_its_request():
    ex = FakeExecutor(n_workers=1, fail_on=3)
    reqs = _requests(12, seed=5)
    srv = Server(ex, budget_bytes=10**12).start()
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert reqs[3].error is not None and "planted" in reqs[3].error
    # the others, also those batched with it, are answered
    assert all(r.error is None and r.result == FakeExecutor.answer(r) for r in reqs if r.rid != 3)


def test_vertex_cap_splits_batches():
    ex = FakeExecutor(n_workers=1)
    reqs = _requests(20, seed=6, vmin=900, vmax=1000)
    srv = Server(ex, budget_bytes=10**12, max_batch_vertices=2500).start()
    for r in reqs:
        srv.submit(r)
    srv.stop()
    for b in srv.batches:
        assert len(b) == 1 or sum(n_vertices(reqs[i].polys) for i in b) <= 2500


class FakeAsyncExecutor(FakeExecutor):
    """The same work on a timer thread: submit returns at once, poll and
    collect follow the asynchronous executor protocol."""

    def submit(self, w, reqs):
        box = {"done": False, "err": None}

        def work():
            try:
                self.run(w, reqs)
            except Exception as e:      # delivered by collect
                box["err"] = e
            box["done"] = True
        th = threading.Thread(target=work, daemon=True)
        th.start()
        return (th, box)

    def poll(self, token):
        return token[1]["done"]

    def collect(self, token, reqs):
        token[0].join()
        if token[1]["err"] is not None:
            raise token[1]["err"]


def test_async_executor_results_and_overlap():
    ex = FakeAsyncExecutor(n_workers=3)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=8).start()
    reqs = _requests(80, seed=5)
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert all(r.error is None for r in reqs)
    assert all(r.result == FakeExecutor.answer(r) for r in reqs)
    assert ex.max_active >= 2
    assert max(len(b) for b in srv.batches) > 1


def test_async_failure_isolated():
    ex = FakeAsyncExecutor(n_workers=2, fail_on=7)
    srv = Server(ex, budget_bytes=10 ** 9).start()
    reqs = _requests(20, seed=6)
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert reqs[7].error and "planted" in reqs[7].error
    assert all(r.error is None for r in reqs if r.rid != 7)


class _Held:
    """A result object with a size, like a device tensor."""

    def __init__(self, nbytes):
        self.nbytes = nbytes


class HeldExecutor(FakeExecutor):
    def run(self, w, reqs):
        for r in reqs:
            r.result = _Held(self.bpv * n_vertices(r.polys))


def test_held_results_count_against_the_budget():
    """Finished results the caller keeps count against the budget until they
    are dropped; with nothing in flight a request that cannot fit because of
    them is refused instead of waiting forever."""
    import gc
    ex = HeldExecutor(n_workers=1, bytes_per_vertex=1000)
    budget = 1000 * 3000
    srv = Server(ex, budget_bytes=budget).start()
    a = Request(0, "count", _poly(2000, 0))
    srv.submit(a)
    srv.drain()
    assert srv.held_bytes == 1000 * 2000
    b = Request(1, "count", _poly(1500, 1))          # 1.5 MB more: above the budget while a is held
    srv.submit(b)
    srv.drain()
    assert b.error and "held" in b.error
    a.result = None                                  # the caller drops a's result
    gc.collect()
    assert srv.held_bytes == 0
    c = Request(2, "count", _poly(1500, 2))
    srv.submit(c)
    srv.stop()
    assert c.error is None


def test_results_not_kept():
    ex = HeldExecutor(n_workers=2)
    srv = Server(ex, budget_bytes=10 ** 9, keep_results=False).start()
    reqs = _requests(10, seed=8)
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert all(r.result is None and r.result_size == 1 for r in reqs)
    assert srv.held_bytes == 0
