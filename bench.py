#!/usr/bin/env python3
"""Benchmark of the canvas point-in-polygon engine on one MI355X.

Headline (the JSON line's ``value``): join-count of 100,000,000 FP64 points
drawn from a taxi-like mixture of 32 anisotropic Gaussians over a 60 x 60 km
extent (seed 2) with 260 Voronoi-tessellation polygons whose shared edges
are jittered to 50..500 vertices (seed 2); exact per-polygon counts.  A step
is one whole join-count with every input already resident in HBM:
rasterising the polygons into the canvas and boundary index, then probing
every point (spade_join_count).  Before the timed steps the autotuner picks
the canvas resolution (pixels per polygon vertex); the choice is reported in
``config.autotune``.  ``value`` is points per second of whole steps; the
counts of the last timed step are compared with the CPU oracle's.

``roofline`` is the probe kernel's: 16 algorithmic bytes per point (two
float64 coordinates) over its duration, taken with HIP events on the stream
it runs on (the library's phase timers) over the timed steps, against the
8 TB/s HBM peak; beside it the bandwidth of a plain read of the same points
(spade_stream_read) as the achievable ceiling.  ``cpu_baseline`` times the
CPU oracle on the same points with every host core.

Further legs (``--legs``; each one a JSON object of its own):
  c1     latency of the 100k-point, 64-polygon join-count (median, p90);
  c2p    join pairs of the headline workload (all 100M pairs);
  c3     selection of 500M clustered points with one 10k-vertex star;
  c4     1,024 star selections (8..20,000 vertices, areas 1e-4..0.15 of the
         extent) and a 40,000-cell join-count over a resident 200M-point
         table, batched against one query at a time;
  next   the layer index, distance joins, kNN and out-of-core selection;
  serve  a Poisson stream of 200 requests/s for --serve-seconds after a
         warm-up, half selections (the c4 star law), half join-counts (one
         of 8 tessellations with 64..40,000 cells), served with continuous
         batching; p50 / p99 latency from arrival to result-ready.
Parity of every leg is checked against values the CPU oracle wrote
(tests/golden/full_size.json) or computes here.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/sec for PIP join-count (bit-exact) + % HBM peak; p50/p99 served query latency"
PEAK_HBM_GBS = 8000.0
BYTES_PER_POINT = 16.0
CHUNK_POINTS = 4096              # points per table chunk of the batch calls
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size.json")
ALL_LEGS = "c1,c2p,c3,host,c4,next,serve"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("probe.hip", "lookup.h", "exact.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2203_14362_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(n_points, canvas):
    """HBM bytes per probe launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel source, point count and canvas
    size; else None."""
    path = os.path.join(ROOT, "profiles", "k_count_join_c100m_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if (d.get("kernel_source_hash") != kernel_source_hash() or int(d.get("n_points", -1)) != n_points
            or list(d.get("canvas", [])) != list(canvas)):
        return None
    return d.get("hbm_bytes_per_launch")


def golden(name):
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as fh:
        return json.load(fh).get(name)


def digest(*arrays):
    import numpy as np
    h = hashlib.sha256()
    for a, dt in arrays:
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def roofline(name, algorithmic_bytes, ms, bound="hbm", traffic=None, **extra):
    achieved = algorithmic_bytes / (ms / 1000.0) / 1e9
    d = {"bound": bound, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": name,
         "algorithmic_bytes_per_launch": int(algorithmic_bytes), "avg_launch_ms": round(ms, 4)}
    d.update(extra)
    return d


def timed(fn, reps, warmup=1, sync=True):
    """Wall times (ms) of `reps` calls of fn after `warmup` calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        if sync:
            torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return out


def dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


# ---------------------------------------------------------------- legs

def leg_c1(ctx):
    import numpy as np
    import oracle
    from workloads import configs
    x, y = configs.c1_points()
    polys = configs.c1_polys()
    dx, dy = dev(x), dev(y)
    dp = ctx.polys(polys)
    got = None

    def call():
        nonlocal got
        got = ctx.join_count(dx, dy, dp)
    ms = timed(call, 50, warmup=5)
    want = oracle.join_count(x, y, polys)
    ot = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.join_count(x, y, polys)
        ot.append((time.perf_counter() - t0) * 1e3)
    return {"workload": "join-count: 100k uniform points x 64 Voronoi-jitter polygons (8-64 vertices)",
            "median_ms": round(float(np.median(ms)), 4), "p90_ms": round(float(np.percentile(ms, 90)), 4),
            "reps": 50, "oracle_median_ms": round(float(np.median(ot)), 3),
            "gpu_matches_oracle": bool(np.array_equal(got.cpu().numpy().astype(np.uint64), want))}


def leg_c2_pairs(ctx, dx, dy, dp, N):
    import numpy as np
    out = {}

    def call():
        out["r"] = ctx.join_pairs(dx, dy, dp)
    ctx.set_timing(True)
    ms, probe = [], []
    for i in range(8):
        t0 = time.perf_counter()
        call()
        import torch
        torch.cuda.synchronize()
        if i >= 2:
            ms.append((time.perf_counter() - t0) * 1e3)
            probe.append(ctx.last_timing()[1])
    pt, pg = out["r"]
    npairs = int(pt.numel())
    g = golden("c2_pairs")
    parity = None
    if g is not None:
        parity = (npairs == g["n_pairs"] and
                  digest((pt.cpu().numpy().astype(np.int64).astype(np.uint32), "<u4"),
                         (pg.cpu().numpy().astype(np.int64).astype(np.uint32), "<u4")) == g["pairs_sha256"])
    pm = float(np.mean(probe))
    return {"workload": "join pairs: the headline 100M points x 260 polygons", "pairs": npairs,
            "ms_per_call": round(float(np.mean(ms)), 4), "probe_ms": round(pm, 4),
            "pairs_per_s": round(npairs / (float(np.mean(ms)) / 1e3), 1),
            "roofline": roofline("k_emit_count + k_emit", 16.0 * N + 8.0 * npairs, pm,
                                 bytes_rule="16 B/point + 8 B/pair"),
            "gpu_matches_oracle_digest": parity}


def leg_c3(ctx, with_host, extra, restore_ppv):
    import numpy as np
    import torch
    from workloads import configs
    t = time.time()
    x, y = configs.c3_points()
    N = x.size
    dx, dy = dev(x), dev(y)
    star = configs.c3_star()
    dp = ctx.polys(star)
    log("c3 inputs: %d points (%.1fs)" % (N, time.time() - t))
    from paper_2203_14362_amd.autotune import Autotuner, SELECT_CANDIDATES, tune_select
    ppv, trials = tune_select(ctx, dx, dy, dp, Autotuner(candidates=SELECT_CANDIDATES), force=True)
    log("c3 autotune: %.0f pixels per vertex (trials %s)" % (ppv, {k: round(v, 2) for k, v in trials.items()}))
    ctx.set_timing(True)
    ms, probe, ids = [], [], None
    for i in range(6):
        t0 = time.perf_counter()
        ids = ctx.select(dx, dy, dp)
        torch.cuda.synchronize()
        if i >= 1:
            ms.append((time.perf_counter() - t0) * 1e3)
            probe.append(ctx.last_timing()[1])
    n_ids = int(ids.numel())
    g = golden("c3_select")
    parity = None
    if g is not None:
        parity = n_ids == g["n_ids"] and digest((ids.cpu().numpy().astype(np.int64).astype(np.uint32),
                                                 "<u4")) == g["ids_sha256"]
    del dx, dy, ids
    torch.cuda.empty_cache()
    pm = float(np.mean(probe))
    if with_host:   # the same points and star, kept in host memory
        extra["host"] = leg_host(ctx, x, y)
    del x, y
    ctx.set_pixels_per_vertex(restore_ppv)
    return {"workload": "selection: 500M clustered points x one 10k-vertex star (~15% of the extent)",
            "points": N, "ids": n_ids, "autotune": {"pixels_per_vertex": ppv,
                                                    "trial_ms": {str(k): round(v, 3) for k, v in trials.items()}}, "ms_per_call": round(float(np.mean(ms)), 3), "probe_ms": round(pm, 3),
            "points_per_s": round(N / (float(np.mean(ms)) / 1e3), 1),
            "roofline": roofline("k_emit_count_bits + k_emit_bits", 16.0 * N + 4.0 * n_ids, pm,
                                 bytes_rule="16 B/point + 4 B/id (the write pass reads 1 result bit "
                                            "per point, not the points)"),
            "gpu_matches_oracle_digest": parity}


def leg_c4(ctx, dx, dy, table):
    import numpy as np
    import torch
    from workloads import configs
    N = int(dx.numel())
    stars, qb = configs.c4_stars()
    nq = len(qb) - 1
    res = {"workload": "1,024 star selections (8-20,000 vertices, areas 1e-4..0.15) and a 40,000-cell "
                       "census-like join-count over a resident 200M-point table", "table_points": N}
    # batched: rasterise all queries as one canvas set, one pass over the table,
    # at the canvas resolution the autotuner picks for this batch
    from paper_2203_14362_amd.autotune import Autotuner, BATCH_SELECT_CANDIDATES, tune_batch_select
    restore_ppv = ctx.pixels_per_vertex()
    bppv, btrials = tune_batch_select(ctx, stars, qb, table,
                                      Autotuner(candidates=BATCH_SELECT_CANDIDATES, repeats=1), force=True)
    log("c4 autotune: %.0f pixels per vertex (trials %s)" % (bppv, {k: round(v, 1) for k, v in btrials.items()}))
    torch.cuda.empty_cache()
    ctx.set_timing(True)
    b = ctx.batch(stars, qb)
    ids, off = ctx.batch_select(b, table)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = ctx.batch(stars, qb, into=b)
    ids, off = ctx.batch_select(b, table)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    total = int(off[-1])
    count_ms = float(ctx.last_timing()[1])        # the selection's count pass
    overlaps = ctx.batch_stats()
    # parity on the oracle's 2M-point subsample (per-query counts and digest)
    g = golden("c4_select_subsample")
    parity = None
    if g is not None:
        sub = torch.from_numpy(configs.c4_subsample(N)).cuda()
        h = hashlib.sha256()
        ok = True
        for q in range(nq):
            seg = ids[int(off[q]):int(off[q + 1])].to(torch.int64)
            pos = torch.searchsorted(sub, seg).clamp(max=sub.numel() - 1)
            kept = seg[sub[pos] == seg]
            ok &= kept.numel() == g["per_query"][q]
            h.update(kept.cpu().numpy().astype("<u4").tobytes())
        parity = bool(ok and h.hexdigest() == g["ids_sha256"])
    del ids
    b.close()
    torch.cuda.empty_cache()
    ctx.set_pixels_per_vertex(restore_ppv)
    # one query at a time through the plain call, on a sample of queries
    rvo = stars["ring_vtx_off"]
    sample = list(range(0, nq, 32))
    one = []
    for q in sample:
        p = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, rvo[q + 1] - rvo[q]]),
             "vx": stars["vx"][rvo[q]:rvo[q + 1]], "vy": stars["vy"][rvo[q]:rvo[q + 1]]}
        dp = ctx.polys(p)
        ctx.select(dx, dy, dp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.select(dx, dy, dp)
        torch.cuda.synchronize()
        one.append(time.perf_counter() - t0)
        del r
    one_q = float(np.mean(one))
    res["select_batched"] = {"queries": nq, "ids": total, "seconds": round(tb, 4),
                             "queries_per_s": round(nq / tb, 1), "points_queries_per_s": round(N * nq / tb, 1),
                             "gpu_matches_oracle_subsample": parity,
                             "autotune": {"pixels_per_vertex": bppv,
                                          "trial_ms": {str(k): round(v, 1) for k, v in btrials.items()}},
                             "chunk_query_overlaps": overlaps,
                             "roofline": roofline("k_batch_select (count pass)", BYTES_PER_POINT * CHUNK_POINTS * overlaps,
                                                  count_ms,
                                                  bytes_rule="16 B per point-query test: every overlap of a 4096-point "
                                                             "table chunk with a query's canvas box")}
    res["select_one_at_a_time"] = {"queries_timed": len(sample), "seconds_per_query": round(one_q, 5),
                                   "queries_per_s": round(1.0 / one_q, 1),
                                   "points_queries_per_s": round(N / one_q, 1)}
    # the 40k-cell join: batched over the table vs the plain call
    cells = configs.c4_census()
    bj = ctx.batch(cells, [0, cells["n_polys"]])
    cnt = ctx.batch_join_count(bj, table)
    torch.cuda.synchronize()
    tj = timed(lambda: ctx.batch_join_count(bj, table), 5, warmup=1)
    count_direct_ms = float(ctx.last_timing()[1])
    dcells = ctx.polys(cells)
    tp = timed(lambda: ctx.join_count(dx, dy, dcells), 5, warmup=1)
    g = golden("c4_join_40k")
    c = cnt.cpu().numpy().astype(np.uint64)
    jparity = None if g is None else digest((c, "<u8")) == g["counts_sha256"]
    plain = ctx.join_count(dx, dy, dcells).cpu().numpy().astype(np.uint64)
    bj.close()
    res["join_40k"] = {"batched_ms": round(float(np.median(tj)), 3), "plain_ms": round(float(np.median(tp)), 3),
                       "batched_points_per_s": round(N / (float(np.median(tj)) / 1e3), 1),
                       "plain_points_per_s": round(N / (float(np.median(tp)) / 1e3), 1),
                       "gpu_matches_oracle_digest": jparity, "plain_equals_batched": bool(np.array_equal(plain, c)),
                       "roofline": roofline("k_batch_count_direct", BYTES_PER_POINT * N, count_direct_ms,
                                            bytes_rule="16 B per table point (one canvas: every chunk meets it "
                                                       "at most once)")}
    return res


def leg_next(ctx, dx, dy, N):
    """The layer index, distance joins, kNN and the out-of-core selection."""
    import numpy as np
    import torch
    import oracle
    from oracle import disk
    from workloads import configs, gen
    L = gen.EXTENT_M
    out = {}
    # layered join vs one canvas: 260 overlapping stars over the 100M points
    stars, _ = gen.query_stars(260, 50, 500, seed=77, L=L, area=(1e-3, 2e-2), data_seed=2)
    table = ctx.table(dx, dy)
    t0 = time.perf_counter()
    lay = ctx.layered(stars)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    lc = ctx.batch_join_count(lay, table)
    tl = timed(lambda: ctx.batch_join_count(lay, table), 5, warmup=1)
    lpt, lpg = ctx.batch_join_pairs(lay, table)
    tlp = timed(lambda: ctx.batch_join_pairs(lay, table), 3, warmup=1)
    dst = ctx.polys(stars)
    ts = timed(lambda: ctx.join_count(dx, dy, dst), 5, warmup=1)
    sp_pt, sp_pg = ctx.join_pairs(dx, dy, dst)
    tsp = timed(lambda: ctx.join_pairs(dx, dy, dst), 3, warmup=1)
    same = bool(torch.equal(lc, ctx.join_count(dx, dy, dst)) and torch.equal(lpt, sp_pt) and torch.equal(lpg, sp_pg))
    sub = slice(0, 200_000)
    xs, ys = dx[sub].cpu().numpy(), dy[sub].cpu().numpy()
    opt, opg = oracle.join_pairs(xs, ys, stars)
    m = int(np.searchsorted(lpt.cpu().numpy().astype(np.int64), 200_000))
    sample_ok = bool(np.array_equal(lpt[:m].cpu().numpy().astype(np.uint32), opt) and
                     np.array_equal(lpg[:m].cpu().numpy().astype(np.uint32), opg))
    out["layered_join"] = {"polygons": 260, "layers": lay.n_layers, "pairs": int(lpt.numel()),
                           "pairs_per_point": round(int(lpt.numel()) / N, 2),
                           "layer_build_s": round(t_build, 3),
                           "count_layered_ms": round(float(np.median(tl)), 3),
                           "count_one_canvas_ms": round(float(np.median(ts)), 3),
                           "pairs_layered_ms": round(float(np.median(tlp)), 3),
                           "pairs_one_canvas_ms": round(float(np.median(tsp)), 3),
                           "layered_equals_one_canvas": same, "oracle_sample_200k_points": sample_ok}
    lay.close()
    table.close()
    del lpt, lpg, sp_pt, sp_pg
    torch.cuda.empty_cache()
    # distance join type (1): 10,000 disks of 300 m at data points
    cx, cy = gen.mixture_points(10_000, seed=78, L=L)
    djp = {}
    td = timed(lambda: djp.__setitem__("r", ctx.distance_join(dx, dy, cx, cy, 300.0)), 3, warmup=1)
    pt, pd = djp["r"]
    m = int(np.searchsorted(pt.cpu().numpy().astype(np.int64), 200_000))
    o_pt, o_pd = disk.distance_join(xs, ys, cx[:2000], cy[:2000], 300.0)
    g_pt, g_pd = pt[:m].cpu().numpy().astype(np.int64), pd[:m].cpu().numpy().astype(np.int64)
    keep = g_pd < 2000
    dj_ok = bool(np.array_equal(g_pt[keep], o_pt) and np.array_equal(g_pd[keep], o_pd))
    out["distance_join"] = {"disks": 10_000, "radius_m": 300.0, "pairs": int(pt.numel()),
                            "ms_per_call": round(float(np.median(td)), 3),
                            "points_per_s": round(N / (float(np.median(td)) / 1e3), 1),
                            "oracle_sample_200k_points_2000_disks": dj_ok}
    del pt, pd
    # kNN
    kn = []
    ok = True
    for (px, py) in [(L / 2, L / 2), (float(cx[5]), float(cy[5])), (12345.0, 54321.0)]:
        tk = timed(lambda: ctx.knn(dx, dy, px, py, 1000), 3, warmup=1)
        kn.append(float(np.median(tk)))
        got = ctx.knn(dx, dy, px, py, 1000).cpu().numpy().astype(np.int64)
        ok &= bool(np.array_equal(got, disk.knn(dx.cpu().numpy(), dy.cpu().numpy(), px, py, 1000)))
    out["knn"] = {"k": 1000, "ms_per_query": round(float(np.mean(kn)), 3), "gpu_matches_oracle": ok}
    # distance selections from lines (rounded rectangles around 23,800 road
    # segments, 50 m) and from a polygon (a 10,000-vertex star and its 100 m
    # edge buffers)
    from oracle import buffer as obuf
    roads = gen.road_lines(200, 120, 150.0, seed=79, L=L)
    star = gen.star_polygon(10_000, 0.05, (L * 0.4, L * 0.6), L=L, seed=80)
    ctx.set_timing(True)
    for name, fn, geom, r, ofn in (("near_lines", ctx.select_near_lines, roads, 50.0, obuf.select_near_lines),
                                   ("within_polygon", ctx.select_within, star, 100.0, obuf.select_within_polygon)):
        res = {}
        tb, pb = [], []
        for i in range(4):
            t0 = time.perf_counter()
            res["ids"] = fn(dx, dy, geom, r)
            torch.cuda.synchronize()
            if i:
                tb.append((time.perf_counter() - t0) * 1e3)
                pb.append(ctx.last_timing()[1])
        ids = res["ids"].cpu().numpy().astype(np.int64)
        want = ofn(xs, ys, geom, r)
        ok = bool(np.array_equal(ids[ids < 200_000], want))
        probe_ms = float(np.median(pb))
        nid = int(ids.size)
        alg = 16.0 * N + 4.0 * nid + 2 * N / 8.0
        out[name] = {"segments": int(geom["ring_vtx_off"][-1] - (geom["n_polys"] if name == "near_lines" else 0)),
                     "distance_m": r, "ids": nid, "ms_per_call": round(float(np.median(tb)), 3),
                     "probe_ms": round(probe_ms, 3), "points_per_s": round(N / (float(np.median(tb)) / 1e3), 1),
                     "oracle_sample_200k_points": ok,
                     "roofline": {"bound": "hbm", "achieved": round(alg / (probe_ms / 1e3) / 1e9, 1), "peak": 8000.0,
                                  "unit": "GB/s", "frac": round(alg / (probe_ms / 1e3) / 8e12, 4), "traffic": None,
                                  "kernel": "k_buf_bits + k_emit_bits",
                                  "algorithmic_bytes_per_launch": int(alg),
                                  "bytes_rule": "16 B per point + 4 B per id + 1 result bit per point written and read"}}
        log("leg next: %s %.3f ms per call (probe %.3f ms), %d ids, oracle sample %s" %
            (name, float(np.median(tb)), probe_ms, nid, ok))
    # distance join with the same roads as line objects, one distance per
    # road (type 2: 25-100 m)
    rad = np.random.default_rng(81).uniform(25.0, 100.0, roads["n_polys"])
    res = {}
    tj, pj = [], []
    for i in range(4):
        t0 = time.perf_counter()
        res["p"] = ctx.distance_join_lines(dx, dy, roads, rad)
        torch.cuda.synchronize()
        if i:
            tj.append((time.perf_counter() - t0) * 1e3)
            pj.append(ctx.last_timing()[1])
    lp, ll = (t.cpu().numpy().astype(np.int64) for t in res["p"])
    m = int(np.searchsorted(lp, 200_000))
    op, ol = obuf.distance_join_lines(xs, ys, roads, rad)
    lj_ok = bool(np.array_equal(lp[:m], op) and np.array_equal(ll[:m], ol))
    out["distance_join_lines"] = {"lines": int(roads["n_polys"]), "segments": 23800, "distance_m": "25-100 per line",
                                  "pairs": int(lp.size), "ms_per_call": round(float(np.median(tj)), 3),
                                  "probe_ms": round(float(np.median(pj)), 3),
                                  "points_per_s": round(N / (float(np.median(tj)) / 1e3), 1),
                                  "oracle_sample_200k_points": lj_ok}
    log("leg next: line distance join %.3f ms per call, %d pairs, oracle sample %s"
        % (float(np.median(tj)), lp.size, lj_ok))
    return out


def leg_host(ctx, x, y):
    """Out-of-core selection: the 500M points of the selection workload kept
    in host memory, streamed per query through the grid index."""
    import numpy as np
    import torch
    from workloads import configs
    N = x.size
    t0 = time.perf_counter()
    ht = ctx.host_table(x, y)
    t_create = time.perf_counter() - t0
    star = configs.c3_star()
    ids = ctx.host_select(ht, star)
    torch.cuda.synchronize()
    t = timed(lambda: ctx.host_select(ht, star), 3, warmup=0)
    streamed = ht.last_streamed
    g = golden("c3_select")
    parity = None
    if g is not None:
        parity = int(ids.numel()) == g["n_ids"] and digest((ids.cpu().numpy().astype(np.int64).astype(np.uint32),
                                                            "<u4")) == g["ids_sha256"]
    ht.close()
    ms = float(np.median(t))
    return {"workload": "selection of the 500M-point set kept in pinned host memory, one 10k-vertex star",
            "points": N, "table_create_s": round(t_create, 2), "streamed_points": int(streamed),
            "ms_per_query": round(ms, 2), "points_per_s": round(N / (ms / 1e3), 1),
            "h2d_gb_per_s": round(20.0 * streamed / (ms / 1e3) / 1e9, 2), "gpu_matches_oracle_digest": parity}


def leg_serve(dx, dy, seconds, warm_seconds, qps, oneshot):
    """Continuous batching of a Poisson stream over the resident table."""
    import numpy as np
    import torch
    from workloads import configs
    from paper_2203_14362_amd import Context
    from paper_2203_14362_amd.serve import Request, Server, SpadeExecutor, latency_stats, replay

    t = time.time()
    N = int(dx.numel())
    arrivals = configs.c5_arrivals(warm_seconds + seconds)
    n = arrivals.size
    stars, _ = configs.c4_stars(n)
    tess = configs.c5_tessellations()
    log("serving inputs: %d requests, tessellations %s (%.1fs)" % (n, [t_["n_polys"] for t_ in tess],
                                                                   time.time() - t))
    rng = np.random.default_rng(11)
    srvo = stars["ring_vtx_off"]
    reqs = []
    for i in range(n):
        if rng.random() < 0.5:
            p = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, srvo[i + 1] - srvo[i]]),
                 "vx": stars["vx"][srvo[i]:srvo[i + 1]], "vy": stars["vy"][srvo[i]:srvo[i + 1]]}
            reqs.append(Request(i, "select", p))
        else:
            k = int(rng.integers(0, len(tess)))
            reqs.append(Request(i, "count", tess[k], key=("tess", k)))
    ex = SpadeExecutor(dx, dy, n_workers=2)
    ppv, times = ex.autotune(reqs[:32])
    log("serving autotune: %.0f pixels per vertex" % ppv)
    free, total = torch.cuda.mem_get_info()
    budget = max(free - (16 << 30), 1 << 30)
    # results of a sample are kept for the alone-vs-served check, the rest dropped
    keep = set(range(0, n, max(1, n // 24)))
    srv = Server(ex, budget_bytes=budget, keep_results=False).start()
    trace = []
    stop = threading.Event()

    def monitor():
        while not stop.is_set():
            trace.append(torch.cuda.mem_get_info()[0])
            stop.wait(0.5)
    mon = threading.Thread(target=monitor, daemon=True)
    mon.start()
    # keep the sampled results: a server per stream would drop them, so the
    # sampled requests are re-run alone below and compared by digest
    wall = replay(srv, reqs, arrivals)
    srv.stop()
    stop.set()
    mon.join()
    errs = [r.error for r in reqs if r.error]
    if errs:
        raise RuntimeError("served requests failed: %s" % errs[:3])
    t_warm = reqs[0].arrival + warm_seconds
    measured = [r for r in reqs if r.arrival >= t_warm]
    st = latency_stats(measured)
    waits = np.array([r.admitted - r.arrival for r in measured])
    # latency by request kind, and the time from admission to completion
    by_kind = {}
    for kind in ("select", "count"):
        lat = np.array([r.done - r.arrival for r in measured if r.kind == kind]) * 1e3
        svc = np.array([r.done - r.admitted for r in measured if r.kind == kind]) * 1e3
        if lat.size:
            by_kind[kind] = {"requests": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3),
                             "service_p50_ms": round(float(np.percentile(svc, 50)), 3),
                             "service_p99_ms": round(float(np.percentile(svc, 99)), 3)}
    bsz = [len(bch) for bch in srv.batches]
    log("served %d requests (%d measured) in %.2fs: p50 %.2f ms, p99 %.2f ms, mean batch %.2f"
        % (n, len(measured), wall, st["p50_ms"], st["p99_ms"], float(np.mean(bsz))))
    # alone vs served: the sampled requests again, served in one burst with
    # their results kept, and each alone through the plain calls
    ctx = Context(0)
    sample = [Request(r.rid, r.kind, r.polys, key=r.key) for r in reqs if r.rid in keep]
    srv2 = Server(ex, budget_bytes=budget).start()
    for r in sample:
        srv2.submit(r)
    srv2.stop()
    same = True
    for r in sample:
        alone = (ctx.select if r.kind == "select" else ctx.join_count)(dx, dy, r.polys)
        same &= bool(torch.equal(r.result.to(torch.int64), alone.to(torch.int64)))
        r.result = None
    # one at a time through the plain calls, and the batched capacity
    k = min(oneshot, n)
    for r in reqs[:2]:
        (ctx.select if r.kind == "select" else ctx.join_count)(dx, dy, r.polys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs[:k]:
        (ctx.select if r.kind == "select" else ctx.join_count)(dx, dy, r.polys)
    torch.cuda.synchronize()
    one = (time.perf_counter() - t0) / k
    burst = [Request(r.rid, r.kind, r.polys, key=r.key) for r in reqs[:600]]
    srv3 = Server(ex, budget_bytes=budget, keep_results=False).start()
    t0 = time.perf_counter()
    for r in burst:
        srv3.submit(r)
    srv3.stop()
    tb = time.perf_counter() - t0
    cache = {"hits": ex.cache_hits, "builds": ex.cache_builds, "sets_per_worker": ex.cached_sets}
    ex.close()
    ctx.close()
    return {"qps_offered": qps, "seconds": seconds, "warmup_seconds": warm_seconds, "requests": n,
            "measured_requests": len(measured), "table_points": N,
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "mean_ms": round(st["mean_ms"], 3),
            "served_requests_per_s": round(n / wall, 1),
            "admission_wait_p50_ms": round(float(np.percentile(waits, 50)) * 1e3, 3),
            "admission_wait_p99_ms": round(float(np.percentile(waits, 99)) * 1e3, 3),
            "by_kind": by_kind,
            "batches": len(bsz), "mean_batch": round(float(np.mean(bsz)), 2), "max_batch": int(max(bsz)),
            "peak_accounted_gib": round(srv.peak_accounted / 2 ** 30, 2), "budget_gib": round(budget / 2 ** 30, 1),
            "free_hbm_gib_min_max": [round(min(trace) / 2 ** 30, 2), round(max(trace) / 2 ** 30, 2)],
            "served_equals_alone_sample": {"requests": len(sample), "equal": same},
            "capacity_batched_requests_per_s": round(len(burst) / tb, 1),
            "capacity_one_at_a_time_requests_per_s": round(1.0 / one, 1), "one_at_a_time_sample": k,
            "pixels_per_vertex": ppv,
            "canvas_set_cache": cache,
            "mix": "50% selection (star, 8-20000 vertices, areas 1e-4..0.15), 50% join-count "
                   "(one of 8 census-like tessellations, 64..40000 cells, keyed: their canvas sets are cached)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=100_000_000)
    ap.add_argument("--canvas", type=int, nargs=2, default=(0, 0), metavar=("W", "H"),
                    help="fixed canvas size (default: automatic, resolution autotuned)")
    ap.add_argument("--ppv", type=float, default=0.0,
                    help="fixed pixels per polygon vertex instead of autotuning (0 = autotune)")
    ap.add_argument("--tune-cache", default="",
                    help="JSON file of autotuner choices to reuse (and extend) across runs")
    ap.add_argument("--retune", action="store_true",
                    help="measure the canvas resolution again instead of taking a cached or preset choice")
    ap.add_argument("--cpu-sample", type=int, default=100_000_000,
                    help="points timed with the CPU oracle (0 = skip; default: all of them)")
    ap.add_argument("--legs", default=ALL_LEGS, help="comma-separated legs to run after the headline "
                                                     "(%s, host; empty for none)" % ALL_LEGS)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the timed steps, copy a buffer of this many MiB on the device "
                         "(a reference kernel of known traffic for hardware counter runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU: the library runs on a single MI355X and has no "
            "multi-GPU path (--gpus %d requested)." % args.gpus)
        sys.exit(2)
    legs = [l for l in args.legs.split(",") if l]

    import numpy as np
    import torch
    from workloads import configs
    from paper_2203_14362_amd import Context

    N = args.points
    t = time.time()
    x, y = configs.c2_points(N)
    polys, info = configs.c2_polys(return_info=True)
    log("inputs: %d points, %d polygons (%d vertices) generated in %.1fs"
        % (N, polys["n_polys"], int(info["vertex_counts"].sum()), time.time() - t))

    ctx = Context(0)
    ctx.set_canvas_size(*args.canvas)
    dx, dy = dev(x), dev(y)
    dpolys = ctx.polys(polys)
    torch.cuda.synchronize()
    ctx.set_timing(True)

    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read, %d MiB written" % (args.calibrate_copy_mib, args.calibrate_copy_mib))
        del src, dst
    tuned = None
    if list(args.canvas) == [0, 0]:
        if args.ppv > 0:
            ctx.set_pixels_per_vertex(args.ppv)
        else:
            from paper_2203_14362_amd.autotune import Autotuner, tune_join_count
            tuner = Autotuner(args.tune_cache or None)
            ppv, times = tune_join_count(ctx, dx, dy, dpolys, tuner, force=args.retune)
            tuned = {"pixels_per_vertex": ppv, "trial_ms": {str(k): round(v, 3) for k, v in times.items()},
                     "source": tuner.last_source}
            log("autotuned canvas resolution: %.0f pixels per vertex (trials %s)" % (ppv, tuned["trial_ms"]))
        ctx.set_timing(True)
    for _ in range(args.warmup):
        counts = ctx.join_count(dx, dy, dpolys)
    torch.cuda.synchronize()
    log("warmup done")

    raster_ms, probe_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts = ctx.join_count(dx, dy, dpolys)
        r, p = ctx.last_timing()
        raster_ms.append(r)
        probe_ms.append(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    gpu_counts = counts.cpu().numpy().astype(np.uint64)    # the last timed step's counts
    log("timed %d steps: %.3f ms/step (raster %.3f ms, probe %.3f ms)"
        % (args.steps, ms_per_step, float(np.mean(raster_ms)), float(np.mean(probe_ms))))

    cv = ctx.canvas(dpolys)
    cinfo = cv.info()
    cv.close()

    # plain read of the same points: the achievable ceiling of a point stream
    stream = []
    for shape in (0, 1):
        ctx.stream_read(dx, dy, shape)
        ts = []
        for _ in range(10):
            ctx.stream_read(dx, dy, shape)
            ts.append(ctx.last_timing()[1])
        stream.append(float(np.median(ts)))
    ceiling = BYTES_PER_POINT * N / (min(stream) / 1e3) / 1e9

    probe_s = float(np.mean(probe_ms)) / 1000.0
    rl = roofline("k_count", BYTES_PER_POINT * N, probe_s * 1e3, traffic=load_traffic(N, [cinfo["width"],
                                                                                           cinfo["height"]]),
                  bytes_per_point=BYTES_PER_POINT, points_per_launch=N,
                  stream_read_gbs=round(ceiling, 1), frac_of_stream_read=round(BYTES_PER_POINT * N / probe_s / 1e9
                                                                               / ceiling, 4),
                  step_frac=round(BYTES_PER_POINT * N / (ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                  traffic_note="FETCH_SIZE counts L2-to-fabric requests (Infinity Cache hits included), "
                               "scaled by the factor a sequential device copy gives")

    cpu = None
    S = min(args.cpu_sample, N)
    if S > 0:
        import oracle
        t = time.time()
        want = oracle.join_count(x[:S], y[:S], polys)
        dt = time.time() - t
        if S == N:
            parity = bool(np.array_equal(gpu_counts, want))
            how = "the last timed step's counts"
        else:
            sub = ctx.join_count(dx[:S].contiguous(), dy[:S].contiguous(), dpolys).cpu().numpy().astype(np.uint64)
            parity = bool(np.array_equal(sub, want))
            how = "a separate call on the sample"
        cpu = {"value": round(S / dt, 1), "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
               "cpu_model": cpu_model(), "host_cores_total": os.cpu_count(),
               "sample": "first %d of the %d points, all %d polygons, join-count" % (S, N, polys["n_polys"]),
               "seconds": round(dt, 2), "gpu_matches_oracle": parity, "compared": how}
        log("cpu oracle: %d points in %.2fs on %d threads (%s); GPU parity: %s"
            % (S, dt, oracle.num_threads(), cpu_model(), parity))
        if not parity:
            raise SystemExit("GPU counts differ from the oracle")
    del x, y

    extra = {}

    def run_leg(name, fn):
        if name not in legs:
            return
        t = time.time()
        try:
            extra[name] = fn()
        except Exception as e:      # a failing leg is reported, the headline stands
            import traceback
            traceback.print_exc()
            extra[name] = {"error": "%s: %s" % (type(e).__name__, e)}
        log("leg %s done in %.1fs" % (name, time.time() - t))

    run_leg("c1", lambda: leg_c1(ctx))
    run_leg("c2p", lambda: leg_c2_pairs(ctx, dx, dy, dpolys, N))
    run_leg("next", lambda: leg_next(ctx, dx, dy, N))
    del dx, dy, dpolys
    torch.cuda.empty_cache()
    ppv_main = tuned["pixels_per_vertex"] if tuned else (args.ppv if args.ppv > 0 else 256.0)
    run_leg("c3", lambda: leg_c3(ctx, "host" in legs, extra, ppv_main))
    if "c4" in legs or "serve" in legs:
        t = time.time()
        x4, y4 = configs.c4_points()
        d4x, d4y = dev(x4), dev(y4)
        del x4, y4
        log("c4/c5 table points generated (%.1fs)" % (time.time() - t))
        if "c4" in legs:
            table = ctx.table(d4x, d4y)
            run_leg("c4", lambda: leg_c4(ctx, d4x, d4y, table))
            table.close()
            torch.cuda.empty_cache()
        if args.serve_seconds > 0:
            run_leg("serve", lambda: leg_serve(d4x, d4y, args.serve_seconds, args.serve_warmup, args.serve_qps,
                                               200))

    out = {
        "metric": METRIC,
        "value": round(N / (ms_per_step / 1000.0), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "join-count: 100M taxi-like clustered FP64 points (32-Gaussian mixture, "
                               "60x60 km) x 260 Voronoi-jitter polygons (50-500 vertices)",
                   "points": N, "polygons": polys["n_polys"],
                   "vertices": int(info["vertex_counts"].sum()),
                   "canvas": [cinfo["width"], cinfo["height"]],
                   "autotune": tuned,
                   "boundary_pixels": cinfo["boundary_pixels"],
                   "raster_ms": round(float(np.mean(raster_ms)), 4),
                   "probe_ms": round(float(np.mean(probe_ms)), 4),
                   "probe_points_per_s": round(N / probe_s, 1),
                   "counts_sum": int(gpu_counts.sum())},
        "roofline": rl,
        "cpu_baseline": cpu,
    }
    for k in ("c1", "c2p", "c3", "c4", "next", "host"):
        if k in extra:
            out[{"c1": "c1_latency", "c2p": "c2_pairs", "c3": "c3_select", "c4": "batch", "next": "next_rows",
                 "host": "out_of_core"}[k]] = extra[k]
    out["serving"] = extra.get("serve")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
