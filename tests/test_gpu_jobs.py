"""Asynchronous batch jobs through the C ABI: results equal the synchronous
batch calls and the oracle; a call on a context while its worker runs a job
waits for the job (no shared scratch); two jobs of one kind may be
outstanding at once; a submit / wait / free loop allocates nothing after
its first round."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_14362_amd import Context
from paper_2203_14362_amd.serve import concat_sets
from paper_2203_14362_amd.spade import JOB_COUNT, JOB_PAIRS, JOB_SELECT
from workloads import gen

pytestmark = pytest.mark.gpu

L = gen.EXTENT_M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def data():
    x, y = gen.mixture_points(1_000_000, seed=31, L=L)
    stars, qb = gen.query_stars(12, 8, 3000, seed=32, L=L, area=(1e-4, 2e-2), data_seed=31)
    tess = gen.voronoi_jitter(300, 4, 40, seed=33, L=L)
    return x, y, stars, np.asarray(qb, dtype=np.int64), tess


def _one_set(tess):
    return tess, np.array([0, tess["n_polys"]], dtype=np.int64)


def test_jobs_equal_sync_calls_and_oracle(ctx, data):
    x, y, stars, qb, tess = data
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    tp, tqb = _one_set(tess)
    bs, bc, bp = ctx.batch(stars, qb), ctx.batch(tp, tqb), ctx.batch(tp, tqb)
    js = ctx.submit(bs, stars, qb, t, JOB_SELECT)
    jc = ctx.submit(bc, tp, tqb, t, JOB_COUNT)
    jp = ctx.submit(bp, tp, tqb, t, JOB_PAIRS)
    ids, off = js.wait()
    counts = jc.wait()
    pt, pg = jp.wait()
    sids, soff = ctx.batch_select(ctx.batch(stars, qb), t)
    assert np.array_equal(off, soff) and torch.equal(ids, sids)
    assert torch.equal(counts, ctx.batch_join_count(ctx.batch(tp, tqb), t))
    spt, spg = ctx.batch_join_pairs(ctx.batch(tp, tqb), t)
    assert torch.equal(pt, spt) and torch.equal(pg, spg)
    want = oracle.join_count(x, y, tess)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint64), want)
    assert int(want.sum()) == pt.numel()
    rvo = stars["ring_vtx_off"]
    for q in (0, 5, 11):
        p = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, rvo[q + 1] - rvo[q]]),
             "vx": stars["vx"][rvo[q]:rvo[q + 1]], "vy": stars["vy"][rvo[q]:rvo[q + 1]]}
        got = ids[int(off[q]):int(off[q + 1])].cpu().numpy().astype(np.int64)
        assert np.array_equal(got, oracle.select(x, y, p).astype(np.int64)), q
    t.close()


def test_calls_while_a_job_runs_wait_for_it(data):
    """Builds and queries on the same context right after a submit (the
    executor pattern that once shared the context's scratch with the job)."""
    x, y, stars, qb, tess = data
    c = Context(0)
    dx, dy = _dev(x), _dev(y)
    t = c.table(dx, dy)
    tp, tqb = _one_set(tess)
    want_sel = c.batch_select(c.batch(stars, qb), t)
    want_cnt = oracle.join_count(x, y, tess)
    bs = c.batch(stars, qb)
    for rep in range(3):
        print("calls while a job runs, round", rep, flush=True)
        js = c.submit(bs, stars, qb, t, JOB_SELECT)
        bc = c.batch(tp, tqb)                       # waits for the select job
        cnt_plain = c.join_count(dx, dy, tp)        # plain call on the same context
        jc = c.submit(bc, tp, tqb, t, JOB_COUNT)
        ids, off = js.wait()
        counts = jc.wait()
        assert np.array_equal(off, want_sel[1]) and torch.equal(ids, want_sel[0])
        assert np.array_equal(counts.cpu().numpy().astype(np.uint64), want_cnt)
        assert np.array_equal(cnt_plain.cpu().numpy().astype(np.uint64), want_cnt)
        bc.close()
    t.close()
    c.close()


def test_two_jobs_of_one_kind_outstanding(ctx, data):
    x, y, stars, qb, tess = data
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    tp, tqb = _one_set(tess)
    sub = gen.voronoi_jitter(40, 4, 40, seed=34, L=L)
    sp, sqb = _one_set(sub)
    j1 = ctx.submit(ctx.batch(tp, tqb), tp, tqb, t, JOB_COUNT)
    j2 = ctx.submit(ctx.batch(sp, sqb), sp, sqb, t, JOB_COUNT)
    c2 = j2.wait()        # the later one first
    c1 = j1.wait()
    assert np.array_equal(c1.cpu().numpy().astype(np.uint64), oracle.join_count(x, y, tess))
    assert np.array_equal(c2.cpu().numpy().astype(np.uint64), oracle.join_count(x, y, sub))
    t.close()


def test_job_loop_allocates_nothing_after_first_round(data):
    x, y, stars, qb, tess = data
    c = Context(0)
    dx, dy = _dev(x), _dev(y)
    t = c.table(dx, dy)
    # two batches of the stars, the second a subset of the first
    polys2, qb2 = concat_sets([{"n_polys": 1, "poly_ring_off": None,
                                "ring_vtx_off": np.array([0, stars["ring_vtx_off"][q + 1] - stars["ring_vtx_off"][q]]),
                                "vx": stars["vx"][stars["ring_vtx_off"][q]:stars["ring_vtx_off"][q + 1]],
                                "vy": stars["vy"][stars["ring_vtx_off"][q]:stars["ring_vtx_off"][q + 1]]}
                               for q in range(6)])
    b = c.batch(stars, qb)
    sizes = []
    for rep in range(4):
        for polys, qbb in ((stars, qb), (polys2, qb2)):
            j = c.submit(b, polys, qbb, t, JOB_SELECT)
            j.wait()
        sizes.append(c.mem_info()["ctx"])
    assert sizes[1] == sizes[2] == sizes[3], sizes
    t.close()
    b.close()
    c.close()


def test_query_only_jobs_reuse_the_built_set(ctx, data):
    """A job submitted without polygons evaluates the set as last built: the
    same results as the job that rebuilt it, for selections and counts."""
    x, y, stars, qb, tess = data
    dx, dy = _dev(x), _dev(y)
    t = ctx.table(dx, dy)
    tp, tqb = _one_set(tess)
    bs, bc = ctx.batch(stars, qb), ctx.batch(tp, tqb)
    ids, off = ctx.submit(bs, stars, qb, t, JOB_SELECT).wait()
    counts = ctx.submit(bc, tp, tqb, t, JOB_COUNT).wait()
    for rep in range(2):
        ids2, off2 = ctx.submit(bs, None, None, t, JOB_SELECT).wait()
        counts2 = ctx.submit(bc, None, None, t, JOB_COUNT).wait()
        assert np.array_equal(off, off2) and torch.equal(ids, ids2)
        assert torch.equal(counts, counts2)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint64), oracle.join_count(x, y, tess))
    bs.close()
    bc.close()
    t.close()
