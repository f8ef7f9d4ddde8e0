"""The query server on the device: every served result equals the same
request evaluated alone (plain single-query call on the original arrays),
and a sample of them equals the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _mixed_requests(n, seed, tess):
    from paper_2203_14362_amd.serve import Request
    rng = np.random.default_rng(seed)
    stars, _ = gen.query_stars(n, 8, 2000, seed=seed, L=L, area=(1e-4, 1e-2), data_seed=3)
    rvo = stars["ring_vtx_off"]
    M = tess["n_polys"]
    trvo = tess["ring_vtx_off"]
    reqs = []
    for i in range(n):
        if i % 2 == 0:
            p = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, rvo[i + 1] - rvo[i]]),
                 "vx": stars["vx"][rvo[i]:rvo[i + 1]], "vy": stars["vy"][rvo[i]:rvo[i + 1]]}
            reqs.append(Request(i, "select", p))
        else:
            m = int(np.exp(rng.uniform(np.log(16), np.log(M))))
            ks = np.sort(rng.choice(M, m, replace=False))
            rings = [[np.stack([tess["vx"][trvo[k]:trvo[k + 1]], tess["vy"][trvo[k]:trvo[k + 1]]], 1)] for k in ks]
            reqs.append(Request(i, "count", gen.polys_from_rings(rings)))
    return reqs


def test_served_equals_alone(ctx):
    from paper_2203_14362_amd.serve import SpadeExecutor, Server, latency_stats, replay
    x, y = gen.mixture_points(2_000_000, seed=3, L=L)
    tess = gen.voronoi_jitter(600, 4, 40, seed=9, L=L)
    reqs = _mixed_requests(60, 21, tess)
    dx, dy = _dev(x), _dev(y)
    ex = SpadeExecutor(dx, dy, n_workers=2)
    free, _ = torch.cuda.mem_get_info()
    srv = Server(ex, budget_bytes=free // 2).start()
    # the first few arrive as a Poisson stream, the rest in one burst: the
    # burst queues behind the batches in flight and forms mixed batches
    arrivals = gen.poisson_arrivals(200.0, 10.0, seed=7)[:8]
    replay(srv, reqs[:8], arrivals)
    for r in reqs[8:]:
        srv.submit(r)
    srv.stop()
    assert all(r.error is None for r in reqs), [r.error for r in reqs if r.error][:3]
    kind = {r.rid: r.kind for r in reqs}
    assert max(len(b) for b in srv.batches) > 1
    assert any(len({kind[i] for i in b}) == 2 for b in srv.batches), srv.batches
    st = latency_stats(reqs)
    assert st["n"] == len(reqs)
    # results own their memory (no view pinning a batch-sized buffer)
    for r in reqs:
        assert r.result.untyped_storage().nbytes() == r.result.numel() * r.result.element_size(), r.rid
    for r in reqs:
        if r.kind == "select":
            alone = ctx.select(dx, dy, r.polys)
            assert torch.equal(r.result.cpu(), alone.cpu()), r.rid
        else:
            alone = ctx.join_count(dx, dy, r.polys)
            assert torch.equal(r.result.cpu(), alone.cpu()), r.rid
    # a sample against the oracle
    for r in reqs[:6]:
        if r.kind == "select":
            want = oracle.select(x, y, r.polys)
            assert np.array_equal(r.result.cpu().numpy().astype(np.int64).astype(np.uint32), want)
        else:
            want = oracle.join_count(x, y, r.polys)
            assert np.array_equal(r.result.cpu().numpy().astype(np.uint64), want)
    ex.close()


def test_keyed_requests_reuse_their_canvas_sets(ctx):
    """Join-counts keyed by their polygon set: later batches with the same
    keys are evaluated on the cached canvas sets (no rasterisation), with
    eviction beyond the cache size, and every result equals the plain call
    and the oracle."""
    from paper_2203_14362_amd.serve import Request, Server, SpadeExecutor
    x, y = gen.mixture_points(1_000_000, seed=5, L=L)
    dx, dy = _dev(x), _dev(y)
    sets = [gen.voronoi_jitter(m, 4, 30, seed=60 + m, L=L) for m in (40, 90, 200)]
    ex = SpadeExecutor(dx, dy, n_workers=2, cached_sets=2)
    free, _ = torch.cuda.mem_get_info()
    reqs = []
    order = [0, 1, 0, 2, 1, 0, 2, 2, 0, 1, 1, 0]
    for i, k in enumerate(order):
        # one at a time, so that every batch holds a single keyed request
        srv = Server(ex, budget_bytes=free // 2).start()
        r = Request(i, "count", sets[k], key=("tess", k))
        srv.submit(r)
        srv.stop()
        assert r.error is None, r.error
        reqs.append((k, r))
    assert ex.cache_hits > 0 and ex.cache_builds > 3   # hits, and rebuilds after evictions
    assert ex.cache_hits + ex.cache_builds == len(order)
    for k, r in reqs:
        assert torch.equal(r.result.cpu(), ctx.join_count(dx, dy, sets[k]).cpu()), r.rid
    for k in range(3):
        got = next(r for kk, r in reqs if kk == k).result.cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, oracle.join_count(x, y, sets[k]))
    ex.close()
