"""Writes tests/golden/full_size.json: expected results of the full-size
workloads, computed by the CPU oracle alone.

Calls only ``oracle`` and ``workloads`` (never the HIP library).  Large
outputs are stored as SHA-256 digests of their canonical little-endian
arrays (ids and pair columns as uint32, counts as uint64) with their sizes;
small ones are stored in full.  Run from the repository root:

    python tests/golden/make_golden.py [--only NAME ...]

It takes about an hour on 8 cores (the 500M-point selection dominates).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import gen  # noqa: E402
from workloads import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def digest(*arrays):
    h = hashlib.sha256()
    for a, dt in arrays:
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def c2_pairs():
    x, y = configs.c2_points()
    polys = configs.c2_polys()
    pt, pg = oracle.join_pairs(x, y, polys)
    counts = oracle.join_count(x, y, polys)
    return {"n_points": int(x.size), "n_pairs": int(pt.size),
            "pairs_sha256": digest((pt, "<u4"), (pg, "<u4")),
            "counts": [int(c) for c in counts]}


def c3_select():
    x, y = configs.c3_points()
    star = configs.c3_star()
    ids = oracle.select(x, y, star)
    return {"n_points": int(x.size), "n_ids": int(ids.size), "ids_sha256": digest((ids, "<u4"))}


def c4_join_40k():
    x, y = configs.c4_points()
    cells = configs.c4_census()
    counts = oracle.join_count(x, y, cells)
    return {"n_points": int(x.size), "n_polys": int(cells["n_polys"]), "sum": int(counts.sum()),
            "counts_sha256": digest((counts, "<u8"))}


def c4_select_subsample():
    x, y = configs.c4_points()
    idx = configs.c4_subsample(x.size)
    xs, ys = x[idx], y[idx]
    del x, y
    stars, _ = configs.c4_stars()
    n = []
    h = hashlib.sha256()
    for q in range(int(stars["n_polys"])):
        ids = oracle.select(xs, ys, stars, q)
        n.append(int(ids.size))
        h.update(np.ascontiguousarray(idx[ids.astype(np.int64)], dtype="<u4").tobytes())
    return {"n_subsample": int(idx.size), "per_query": n, "ids_sha256": h.hexdigest()}


def c4_select_full16():
    x, y = configs.c4_points()
    stars, _ = configs.c4_stars()
    qs = configs.c4_full_queries()
    res = {}
    for q in qs:
        ids = oracle.select(x, y, stars, int(q))
        res[str(int(q))] = {"n_ids": int(ids.size), "ids_sha256": digest((ids, "<u4"))}
    return {"n_points": int(x.size), "queries": res}


JOBS = {"c2_pairs": c2_pairs, "c4_join_40k": c4_join_40k, "c4_select_subsample": c4_select_subsample,
        "c4_select_full16": c4_select_full16, "c3_select": c3_select}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name, fn in JOBS.items():
        if a.only and name not in a.only:
            continue
        t = time.time()
        data[name] = fn()
        data[name]["oracle_seconds"] = round(time.time() - t, 1)
        data[name]["oracle_threads"] = oracle.num_threads()
        print("%s done in %.1fs" % (name, time.time() - t), flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
