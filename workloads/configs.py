"""The five benchmark workloads as seeded generator calls.

One place fixes every seed, size and distribution of the configurations the
tests, the benchmark and the golden-value script share.  Nothing here
computes any part of a query: these are inputs only.

* C1: 100k uniform points in [0,1)^2 x 64 Voronoi-jitter cells (8-64
  vertices), seed 1.
* C2: 100M taxi-like clustered points (seed 2) x 260 Voronoi-jitter cells
  (50-500 vertices, seed 2) over the 60 km extent.
* C3: 500M clustered points (seed 3) x one 10k-vertex star, 30 % radius
  noise, about 15 % of the extent, centred in it (seed 3).
* C4: a resident table of 200M clustered points (seed 4); 1,024 query stars
  (8-20,000 vertices log-uniform, areas log-uniform in 1e-4..0.15 of the
  extent, centres from the points' mixture; seed 8); a 40,000-cell
  census-like tessellation (4-40 vertices, cell seeds from the points'
  mixture; seed 9).
* C5: the C4 table; Poisson arrivals at 200/s (seed 5); half selections from
  the C4 star law, half join-counts over one of 8 census-like tessellations
  with M log-spaced in [64, 40,000].
"""
from __future__ import annotations

import math

import numpy as np

from . import gen

L = gen.EXTENT_M

C2_N = 100_000_000
C3_N = 500_000_000
C4_N = 200_000_000
C4_Q = 1024
C4_AREA = (1e-4, 0.15)
C5_QPS = 200.0
C5_TESS_M = [int(round(v)) for v in np.exp(np.linspace(math.log(64), math.log(40_000), 8))]


def c1_points():
    return gen.uniform_points(100_000, seed=1)


def c1_polys():
    return gen.voronoi_jitter(64, 8, 64, seed=1, L=1.0)


def c2_points(n: int = C2_N):
    return gen.mixture_points(n, seed=2, L=L)


def c2_polys(return_info: bool = False):
    return gen.voronoi_jitter(260, 50, 500, seed=2, L=L, return_info=return_info)


def c3_points(n: int = C3_N):
    return gen.mixture_points(n, seed=3, L=L)


def c3_star():
    return gen.star_polygon(10_000, 0.15, (L / 2, L / 2), L=L, seed=3)


def c4_points(n: int = C4_N):
    return gen.mixture_points(n, seed=4, L=L)


def c4_stars(nq: int = C4_Q):
    """(polys, qbound): query q is polygon q."""
    return gen.query_stars(nq, 8, 20_000, seed=8, L=L, area=C4_AREA, data_seed=4)


def c4_census(M: int = 40_000):
    return gen.census_cells(M, 4, 40, seed=9, data_seed=4, L=L)


def c4_subsample(n: int, size: int = 2_000_000):
    """Ascending seeded sample of table point ids for whole-batch checks."""
    return np.sort(gen.rng_for(4, 11).choice(n, size=min(size, n), replace=False))


def c4_full_queries(k: int = 16):
    """Seeded queries whose selections are checked over the whole table."""
    return np.sort(gen.rng_for(4, 12).choice(C4_Q, size=k, replace=False))


def c5_arrivals(seconds: float, seed: int = 5):
    return gen.poisson_arrivals(C5_QPS, seconds, seed=seed)


def c5_tessellations():
    """The 8 census-like tessellations join-count requests draw from."""
    return [gen.census_cells(m, 4, 40, seed=20 + i, data_seed=4, L=L) for i, m in enumerate(C5_TESS_M)]
