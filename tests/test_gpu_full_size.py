"""Parity at the full workload sizes against expected values the CPU oracle
wrote (tests/golden/make_golden.py, which calls only the oracle and the
workload generators): whole outputs compared through SHA-256 digests of the
canonical arrays, plus properties that hold at any size.

* C2: all 100M pairs and the 260 counts.
* C3: all ids of the 500M-point selection.
* C4: the 40k-cell join-count over the 200M-point table (batched and plain),
  all 1,024 batched selections restricted to a 2M-point subsample, and 16 of
  them over the whole table.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

from workloads import configs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")


def _golden(name):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden values not written")
    with open(GOLDEN) as fh:
        g = json.load(fh)
    if name not in g:
        pytest.skip("golden values for %s not written" % name)
    return g[name]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _digest(*arrays):
    h = hashlib.sha256()
    for a, dt in arrays:
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def _u32(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


def test_c2_full_join_pairs_and_counts(ctx):
    """100M clustered points x 260 Voronoi-jitter polygons (50-500 vertices)."""
    g = _golden("c2_pairs")
    x, y = configs.c2_points()
    polys = configs.c2_polys()
    dx, dy = _dev(x), _dev(y)
    del x, y
    counts = ctx.join_count(dx, dy, polys).cpu().numpy().astype(np.uint64)
    assert counts.tolist() == g["counts"]
    pt, pg = ctx.join_pairs(dx, dy, polys)
    assert pt.numel() == g["n_pairs"]
    assert _digest((_u32(pt), "<u4"), (_u32(pg), "<u4")) == g["pairs_sha256"]


def test_c3_full_selection(ctx):
    """500M clustered points x one 10k-vertex star (~15% of the extent)."""
    g = _golden("c3_select")
    x, y = configs.c3_points()
    dx, dy = _dev(x), _dev(y)
    del x, y
    ids = ctx.select(dx, dy, configs.c3_star())
    assert ids.numel() == g["n_ids"]
    assert _digest((_u32(ids), "<u4")) == g["ids_sha256"]


@pytest.fixture(scope="module")
def c4_table(ctx):
    x, y = configs.c4_points()
    dx, dy = _dev(x), _dev(y)
    del x, y
    t = ctx.table(dx, dy)
    yield dx, dy, t
    t.close()


def test_c4_join_40k(ctx, c4_table):
    """Join-count with 40k census-like cells (4-40 vertices) over the table,
    batched and through the plain call on the original arrays."""
    g = _golden("c4_join_40k")
    dx, dy, t = c4_table
    cells = configs.c4_census()
    b = ctx.batch(cells, [0, cells["n_polys"]])
    counts = ctx.batch_join_count(b, t).cpu().numpy().astype(np.uint64)
    b.close()
    assert int(counts.sum()) == g["sum"] == dx.numel()
    assert _digest((counts, "<u8")) == g["counts_sha256"]
    plain = ctx.join_count(dx, dy, cells).cpu().numpy().astype(np.uint64)
    assert np.array_equal(plain, counts)


def test_c4_batched_selection(ctx, c4_table):
    """1,024 star selections (8-20,000 vertices, areas 1e-4..0.15) over the
    table in one batch: every query restricted to a 2M-point subsample, and
    16 queries in full, against the oracle's digests; three queries alone
    through the plain call."""
    gs = _golden("c4_select_subsample")
    gf = _golden("c4_select_full16")
    dx, dy, t = c4_table
    N = dx.numel()
    stars, qb = configs.c4_stars()
    b = ctx.batch(stars, qb)
    ids, off = ctx.batch_select(b, t)
    b.close()
    sub = torch.from_numpy(configs.c4_subsample(N)).cuda()
    h = hashlib.sha256()
    for q in range(len(qb) - 1):
        seg = ids[int(off[q]):int(off[q + 1])].to(torch.int64)
        if seg.numel() > 1:
            assert bool((seg[1:] > seg[:-1]).all()), q
        pos = torch.searchsorted(sub, seg).clamp(max=sub.numel() - 1)
        kept = seg[sub[pos] == seg]
        assert kept.numel() == gs["per_query"][q], q
        h.update(kept.cpu().numpy().astype("<u4").tobytes())
    assert h.hexdigest() == gs["ids_sha256"]
    for q, want in gf["queries"].items():
        seg = ids[int(off[int(q)]):int(off[int(q) + 1])]
        assert seg.numel() == want["n_ids"], q
        assert _digest((_u32(seg), "<u4")) == want["ids_sha256"], q
    rvo = stars["ring_vtx_off"]
    for q in (0, 511, 1023):
        one = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, rvo[q + 1] - rvo[q]]),
               "vx": stars["vx"][rvo[q]:rvo[q + 1]], "vy": stars["vy"][rvo[q]:rvo[q + 1]]}
        alone = ctx.select(dx, dy, one)
        assert torch.equal(alone.to(torch.int64), ids[int(off[q]):int(off[q + 1])].to(torch.int64)), q
