"""Generator checks (no GPU): determinism, extent, shared edges, simplicity."""
import numpy as np

from workloads import gen


def test_mixture_deterministic_and_in_extent():
    x1, y1 = gen.mixture_points(100_000, seed=2)
    x2, y2 = gen.mixture_points(100_000, seed=2)
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
    assert x1.min() >= 0 and x1.max() < gen.EXTENT_M and y1.min() >= 0 and y1.max() < gen.EXTENT_M
    # chunking: a prefix is reproducible on its own
    x3, _ = gen.mixture_points(gen.CHUNK + 10, seed=2)
    x4, _ = gen.mixture_points(gen.CHUNK, seed=2)
    assert np.array_equal(x3[:gen.CHUNK], x4)


def test_voronoi_shared_edges_bit_identical():
    polys = gen.voronoi_jitter(30, 20, 80, seed=3, L=60000.0)
    rv = polys["ring_vtx_off"]
    edges = {}
    for k in range(polys["n_polys"]):
        px, py = polys["vx"][rv[k]:rv[k + 1]], polys["vy"][rv[k]:rv[k + 1]]
        n = px.size
        for j in range(n):
            a = (px[j], py[j])
            b = (px[(j + 1) % n], py[(j + 1) % n])
            edges.setdefault((min(a, b), max(a, b)), []).append(k)
    L = 60000.0
    for (a, b), owners in edges.items():
        on_side = (a[0] == b[0] and a[0] in (0.0, L)) or (a[1] == b[1] and a[1] in (0.0, L))
        assert len(owners) == (1 if on_side else 2), (a, b, owners)


def test_voronoi_vertex_count_range_and_area():
    polys, info = gen.voronoi_jitter(260, 50, 500, seed=2, L=60000.0, return_info=True)
    vc = info["vertex_counts"]
    assert vc.max() <= 500 and np.median(vc) >= 50
    assert abs(info["area_sum"] / 3.6e9 - 1.0) < 1e-9


def test_star_polygon_shape():
    p = gen.star_polygon(10000, 0.15, (30000.0, 30000.0), seed=3)
    assert p["vx"].size == 10000
    x, y = p["vx"], p["vy"]
    area = 0.5 * abs(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
    assert 0.12 < area / 3.6e9 < 0.18


def test_poisson_arrivals():
    t = gen.poisson_arrivals(200.0, 10.0, seed=5)
    assert np.all(np.diff(t) > 0) and t[-1] < 10.0
    assert 1700 < t.size < 2300
