#!/usr/bin/env python3
"""Benchmark of the canvas point-in-polygon join-count on one MI355X.

Workload (the headline configuration): 100,000,000 FP64 points drawn from a
taxi-like mixture of 32 anisotropic Gaussians over a 60 x 60 km extent
(seed 2) against 260 Voronoi-tessellation polygons whose shared edges are
jittered to 50..500 vertices (seed 2); output: exact per-polygon counts.

A step is one whole join-count with every input already resident in HBM:
rasterising the polygons into the canvas and boundary index, then probing
every point (spade_join_count).  Before the timed steps the autotuner picks
the canvas resolution (pixels per polygon vertex) from a few trial queries;
the choice is reported in ``config.autotune``.  ``value`` is points per second of whole
steps.  The probe kernel's duration is taken with HIP events on the stream
it runs on (the library's phase timers) over the timed steps; its roofline
entry prices 16 algorithmic bytes per point (two float64 coordinates)
against the 8 TB/s HBM peak.  ``cpu_baseline`` times the CPU oracle on a
bounded prefix of the same points with every host core.

The ``serving`` object comes from a second leg (skipped with
``--serve-seconds 0``): a resident table of 200,000,000 clustered points,
requests arriving as a Poisson stream at 200 per second for the given
number of seconds, half selections (one star of 8..20,000 vertices), half
join-counts (64..40,000 polygons of a 40,000-cell Voronoi-jitter
tessellation with 4..40 vertices each), served with continuous batching on
two workers.  It reports p50 / p99 latency from arrival to result-ready and
the served rate, beside the rate of the same requests run one at a time
with the plain single-query calls.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/sec for PIP join-count (bit-exact) + % HBM peak; p50/p99 served query latency"
PEAK_HBM_GBS = 8000.0
BYTES_PER_POINT = 16.0


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


def _mem(tag):
    import torch
    free, total = torch.cuda.mem_get_info()
    log("device memory %s: %.1f GiB free of %.1f GiB" % (tag, free / 2**30, total / 2**30))


def serving_leg(seconds, qps, n_points, oneshot_max):
    """Continuous-batching server over a resident table; one-at-a-time baseline."""
    import numpy as np
    import torch
    from workloads import gen
    from paper_2203_14362_amd import Context
    from paper_2203_14362_amd.serve import Request, Server, SpadeExecutor, latency_stats, replay

    t = time.time()
    x, y = gen.mixture_points(n_points, seed=2, L=gen.EXTENT_M)
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
    del x, y
    arrivals = gen.poisson_arrivals(qps, seconds, seed=5)
    n = arrivals.size
    stars, _ = gen.query_stars(n, 8, 20000, seed=8, L=gen.EXTENT_M, area=(1e-4, 1e-2), data_seed=2)
    tess = gen.voronoi_jitter(40000, 4, 40, seed=9, L=gen.EXTENT_M)
    log("serving inputs: %d points, %d requests, 40000-cell tessellation (%.1fs)" % (n_points, n, time.time() - t))
    rng = np.random.default_rng(11)
    srvo, trvo = stars["ring_vtx_off"], tess["ring_vtx_off"]
    reqs = []
    for i in range(n):
        if rng.random() < 0.5:
            p = {"n_polys": 1, "poly_ring_off": None, "ring_vtx_off": np.array([0, srvo[i + 1] - srvo[i]]),
                 "vx": stars["vx"][srvo[i]:srvo[i + 1]], "vy": stars["vy"][srvo[i]:srvo[i + 1]]}
            reqs.append(Request(i, "select", p))
        else:
            m = int(np.exp(rng.uniform(np.log(64), np.log(40000))))
            ks = np.sort(rng.choice(40000, m, replace=False))
            lens = trvo[ks + 1] - trvo[ks]
            idx = np.concatenate([np.arange(trvo[k], trvo[k + 1]) for k in ks])
            p = {"n_polys": m, "poly_ring_off": None,
                 "ring_vtx_off": np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
                 "vx": tess["vx"][idx], "vy": tess["vy"][idx]}
            reqs.append(Request(i, "count", p))

    _mem("before the table")
    ex = SpadeExecutor(dx, dy, n_workers=2)
    _mem("with the table")
    ppv, times = ex.autotune(reqs[:32])
    _mem("after autotuning")
    log("serving autotune: %.0f pixels per vertex (trials %s)" % (ppv, {k: round(v, 2) for k, v in times.items()}))
    free, _ = torch.cuda.mem_get_info()
    budget = max(free - (16 << 30), 1 << 30)
    # warm the workers' contexts and canvas sets
    warm = [Request(-1 - k, r.kind, r.polys) for k, r in enumerate(reqs[:4])]
    srv = Server(ex, budget_bytes=budget).start()
    for r in warm:
        srv.submit(r)
    srv.drain()
    srv.done.clear()
    srv.batches.clear()
    wall = replay(srv, reqs, arrivals)
    srv.stop()
    _mem("after the served stream")
    errs = [r.error for r in reqs if r.error]
    if errs:
        raise SystemExit("served requests failed: %s" % errs[:3])
    st = latency_stats(reqs)
    sizes = [len(b) for b in srv.batches]
    log("served %d requests in %.2fs: p50 %.2f ms, p99 %.2f ms, %d batches (mean %.1f requests)"
        % (n, wall, st["p50_ms"], st["p99_ms"], len(sizes), float(np.mean(sizes))))

    # one at a time, plain calls on the original arrays (no table, no batching)
    ctx = Context(0)
    k = min(oneshot_max, n)
    for r in reqs[:2]:
        (ctx.select if r.kind == "select" else ctx.join_count)(dx, dy, r.polys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs[:k]:
        (ctx.select if r.kind == "select" else ctx.join_count)(dx, dy, r.polys)
    torch.cuda.synchronize()
    one = (time.perf_counter() - t0) / k
    # served capacity: the same requests submitted at once (no arrival gaps)
    for r in reqs:
        r.arrival = r.admitted = r.done = r.result = None
    srv = Server(ex, budget_bytes=budget).start()
    t0 = time.perf_counter()
    for r in reqs:
        srv.submit(r)
    srv.stop()
    burst = time.perf_counter() - t0
    ex.close()
    ctx.close()
    log("capacity: batched %.1f requests/s vs one at a time %.1f requests/s" % (n / burst, 1.0 / one))
    return {"qps_offered": qps, "seconds": seconds, "requests": n, "table_points": n_points,
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "mean_ms": round(st["mean_ms"], 3), "served_requests_per_s": round(n / wall, 1),
            "batches": len(sizes), "mean_batch": round(float(np.mean(sizes)), 2),
            "capacity_batched_requests_per_s": round(n / burst, 1),
            "capacity_one_at_a_time_requests_per_s": round(1.0 / one, 1),
            "one_at_a_time_sample": k,
            "pixels_per_vertex": ppv,
            "mix": "50% selection (star, 8-20000 vertices), 50% join-count (64-40000 Voronoi cells, 4-40 vertices)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=100_000_000)
    ap.add_argument("--polygons", type=int, default=260)
    ap.add_argument("--canvas", type=int, nargs=2, default=(0, 0), metavar=("W", "H"),
                    help="fixed canvas size (default: automatic, resolution autotuned)")
    ap.add_argument("--ppv", type=float, default=0.0,
                    help="fixed pixels per polygon vertex instead of autotuning (0 = autotune)")
    ap.add_argument("--tune-cache", default="",
                    help="JSON file of autotuner choices to reuse (and extend) across runs")
    ap.add_argument("--retune", action="store_true",
                    help="measure the canvas resolution again instead of taking a cached or preset choice")
    ap.add_argument("--cpu-sample", type=int, default=100_000_000,
                    help="points of the prefix timed with the CPU oracle (0 = skip; default: all of them)")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="length of the served Poisson stream (0 = skip the serving leg)")
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-points", type=int, default=200_000_000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the timed steps, copy a buffer of this many MiB on the device "
                         "(a reference kernel of known traffic for hardware counter runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU: this build runs on a single MI355X and has no "
            "multi-GPU path (--gpus %d requested)." % args.gpus)
        sys.exit(2)

    import numpy as np
    import torch
    from workloads import gen
    from paper_2203_14362_amd import Context

    N = args.points
    t = time.time()
    x, y = gen.mixture_points(N, seed=2, L=gen.EXTENT_M)
    polys, info = gen.voronoi_jitter(args.polygons, 50, 500, seed=2, L=gen.EXTENT_M, return_info=True)
    log("inputs: %d points, %d polygons (%d vertices) generated in %.1fs"
        % (N, polys["n_polys"], int(info["vertex_counts"].sum()), time.time() - t))

    ctx = Context(0)
    ctx.set_canvas_size(*args.canvas)
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
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
    if args.canvas == (0, 0) or list(args.canvas) == [0, 0]:
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
    total = int(counts.sum().item())
    if total != N:
        raise SystemExit("counts sum to %d, expected %d (tessellation covers every point)" % (total, N))
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
    gpu_counts = counts.cpu().numpy().astype(np.uint64)
    log("timed %d steps: %.3f ms/step (raster %.3f ms, probe %.3f ms)"
        % (args.steps, ms_per_step, float(np.mean(raster_ms)), float(np.mean(probe_ms))))

    cv = ctx.canvas(dpolys)
    cinfo = cv.info()
    cv.close()

    probe_s = float(np.mean(probe_ms)) / 1000.0
    achieved = BYTES_PER_POINT * N / probe_s / 1e9
    traffic = load_traffic(N, [cinfo["width"], cinfo["height"]])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": "k_count", "bytes_per_point": BYTES_PER_POINT,
                "points_per_launch": N, "avg_launch_ms": round(probe_s * 1000.0, 4)}

    cpu = None
    S = min(args.cpu_sample, N)
    if S > 0:
        import oracle
        t = time.time()
        want = oracle.join_count(x[:S], y[:S], polys)
        dt = time.time() - t
        sub = ctx.join_count(dx[:S].contiguous(), dy[:S].contiguous(), dpolys).cpu().numpy().astype(np.uint64)
        parity = bool(np.array_equal(sub, want))
        cpu = {"value": round(S / dt, 1), "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "first %d of the %d points, all %d polygons, join-count" % (S, N, polys["n_polys"]),
               "seconds": round(dt, 2), "gpu_matches_oracle_on_sample": parity}
        log("cpu oracle: %d points in %.2fs on %d threads; GPU parity on sample: %s"
            % (S, dt, oracle.num_threads(), parity))
        if not parity:
            raise SystemExit("GPU counts differ from the oracle on the sample")

    serving = None
    if args.serve_seconds > 0:
        del dx, dy
        torch.cuda.empty_cache()
        serving = serving_leg(args.serve_seconds, args.serve_qps, args.serve_points, 200)

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
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
