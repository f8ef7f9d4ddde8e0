"""Seeded synthetic stand-ins for the paper's point and polygon datasets.

The paper evaluates on NYC taxi pickups, tweets, neighbourhood / census /
county / zip-code polygons (Sec. 6, Table 1).  None of those datasets is
used here; these generators reproduce their shape instead:

* ``uniform_points``   -- i.i.d. uniform points in [0, 1)^2.
* ``mixture_points``   -- "taxi-like" clustered points: a mixture of 32
  anisotropic Gaussians (weights Dirichlet(1), sigmas 200..3000 m, random
  rotation) over an L x L metre extent, rejected to the half-open extent.
  Chunked: every 2^22 points come from their own spawned PCG64 stream, so any
  prefix or chunk is reproducible on its own.
* ``voronoi_jitter``   -- "neighbourhood/census-like" tessellations: Voronoi
  cells of seeds (mirrored across the extent sides so the cells tile the
  extent exactly), every shared ridge subdivided ONCE with a tapered
  perpendicular jitter so both neighbours carry bit-identical vertices, and
  ridges on the extent sides kept exactly on the sides.  Every cell is
  checked to be simple and counter-clockwise, which makes the cells an exact
  tiling: each point of the extent lies in exactly one cell.
* ``star_polygon``     -- a star-shaped query polygon with i.i.d. 30 % radius
  noise (the selection constraint).
* ``lattice_points`` / ``rect_grid`` / ``right_triangle`` -- dyadic fixtures
  with closed-form answers.
* ``poisson_arrivals`` -- request arrival times for the server.

Polygon sets are returned as a dict in CSR layout:
``{"n_polys": M, "poly_ring_off": int64[M+1] or None, "ring_vtx_off":
int64[R+1], "vx": float64[V], "vy": float64[V]}``; rings are implicitly
closed (the first vertex is not repeated).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng_for", "uniform_points", "mixture_params", "mixture_points",
    "voronoi_jitter", "star_polygon", "lattice_points", "rect_grid",
    "right_triangle", "poisson_arrivals", "polys_from_rings", "concat_polys",
    "census_cells", "offset_frame", "WEB_MERCATOR_ORIGIN",
    "poly_vertex_counts", "EXTENT_M",
]

EXTENT_M = 60000.0          # side of the metre extent used by the clustered configs
CHUNK = 1 << 22             # points per independently seeded chunk


def rng_for(seed, *path):
    """PCG64 generator for ``seed`` and an optional spawn path."""
    ss = np.random.SeedSequence(seed)
    for p in path:
        ss = ss.spawn(p + 1)[p]
    return np.random.Generator(np.random.PCG64(ss))


# ---------------------------------------------------------------- points

def uniform_points(n: int, seed: int = 1):
    """n points uniform in [0,1)^2 (multiples of 2^-53)."""
    rng = rng_for(seed, 0)
    x = rng.random(n)
    y = rng.random(n)
    return x, y


def mixture_params(seed: int, L: float = EXTENT_M, K: int = 32):
    """Component weights, centres, sigmas and rotations of the taxi-like mixture."""
    rng = rng_for(seed, 1)
    w = rng.dirichlet(np.ones(K))
    c = rng.uniform(0.1 * L, 0.9 * L, size=(K, 2))
    # sigmas of 200..3000 m on the 60 km extent, scaled with the extent
    s = rng.uniform(200.0, 3000.0, size=(K, 2)) * (float(L) / EXTENT_M)
    th = rng.uniform(0.0, math.pi, size=K)
    return {"w": w, "c": c, "s": s, "th": th, "L": float(L)}


def _mixture_chunk(params, n, rng):
    w, c, s, th, L = params["w"], params["c"], params["s"], params["th"], params["L"]
    cos, sin = np.cos(th), np.sin(th)
    outx = np.empty(n)
    outy = np.empty(n)
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.1) + 64
        comp = rng.choice(w.size, size=m, p=w)
        z = rng.standard_normal((m, 2))
        u = z[:, 0] * s[comp, 0]
        v = z[:, 1] * s[comp, 1]
        x = c[comp, 0] + cos[comp] * u - sin[comp] * v
        y = c[comp, 1] + sin[comp] * u + cos[comp] * v
        ok = (x >= 0.0) & (x < L) & (y >= 0.0) & (y < L)
        x, y = x[ok], y[ok]
        take = min(x.size, n - filled)
        outx[filled:filled + take] = x[:take]
        outy[filled:filled + take] = y[:take]
        filled += take
    return outx, outy


def mixture_points(n: int, seed: int = 2, L: float = EXTENT_M, out=None, workers: int = 0):
    """n taxi-like clustered points in [0,L)^2, generated chunk by chunk.

    ``out`` may be a pair of preallocated float64 arrays (e.g. memory maps).
    Chunks are independent streams, so ``workers`` threads give the same
    result as one (0 = up to 16 threads).
    """
    import os
    from concurrent.futures import ThreadPoolExecutor

    params = mixture_params(seed, L)
    if out is None:
        x = np.empty(n)
        y = np.empty(n)
    else:
        x, y = out
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(ci):
        lo = ci * CHUNK
        m = min(CHUNK, n - lo)
        cx, cy = _mixture_chunk(params, m, rng_for(seed, 2, ci))
        x[lo:lo + m] = cx
        y[lo:lo + m] = cy

    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    if workers == 1 or nchunks <= 1:
        for ci in range(nchunks):
            work(ci)
    else:
        with ThreadPoolExecutor(min(workers, nchunks)) as ex:
            list(ex.map(work, range(nchunks)))
    return x, y


def lattice_points(nx: int, ny: int, h: float, x0: float = 0.0, y0: float = 0.0):
    """Points (x0 + i h, y0 + j h) for 0 <= i < nx, 0 <= j < ny (row-major in j)."""
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    X, Y = np.meshgrid(x0 + i * h, y0 + j * h)
    return X.ravel().copy(), Y.ravel().copy()


def poisson_arrivals(rate: float, duration: float, seed: int = 5):
    rng = rng_for(seed, 3)
    n = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration]


# --------------------------------------------------------------- polygons

def polys_from_rings(polys_rings):
    """List (per polygon) of list of rings (arrays [n,2]) -> CSR dict."""
    pro = [0]
    rvo = [0]
    xs, ys = [], []
    for rings in polys_rings:
        for ring in rings:
            ring = np.asarray(ring, dtype=np.float64).reshape(-1, 2)
            xs.append(ring[:, 0])
            ys.append(ring[:, 1])
            rvo.append(rvo[-1] + ring.shape[0])
        pro.append(len(rvo) - 1)
    vx = np.concatenate(xs) if xs else np.zeros(0)
    vy = np.concatenate(ys) if ys else np.zeros(0)
    return {"n_polys": len(polys_rings), "poly_ring_off": np.asarray(pro, dtype=np.int64),
            "ring_vtx_off": np.asarray(rvo, dtype=np.int64), "vx": vx, "vy": vy}


def concat_polys(a, b):
    """Polygon set a followed by polygon set b."""
    def rings_of(p):
        pro = p.get("poly_ring_off")
        M = p["n_polys"]
        return pro if pro is not None else np.arange(M + 1, dtype=np.int64)
    pa, pb = rings_of(a), rings_of(b)
    ra, rb = a["ring_vtx_off"], b["ring_vtx_off"]
    nva = ra[-1]
    return {"n_polys": a["n_polys"] + b["n_polys"],
            "poly_ring_off": np.concatenate([pa, pb[1:] + pa[-1]]).astype(np.int64),
            "ring_vtx_off": np.concatenate([ra, rb[1:] + nva]).astype(np.int64),
            "vx": np.concatenate([a["vx"], b["vx"]]), "vy": np.concatenate([a["vy"], b["vy"]])}


def poly_vertex_counts(polys):
    pro = polys.get("poly_ring_off")
    rvo = np.asarray(polys["ring_vtx_off"])
    per_ring = np.diff(rvo)
    if pro is None:
        return per_ring
    cs = np.concatenate([[0], np.cumsum(per_ring)])
    return cs[np.asarray(pro)[1:]] - cs[np.asarray(pro)[:-1]]


def rect_grid(nx: int, ny: int, x0: float, y0: float, w: float, h: float):
    """nx*ny axis-aligned rectangles tiling [x0, x0+nx w) x [y0, y0+ny h)."""
    rings = []
    for j in range(ny):
        for i in range(nx):
            a, b = x0 + i * w, x0 + (i + 1) * w
            c, d = y0 + j * h, y0 + (j + 1) * h
            rings.append([np.array([[a, c], [b, c], [b, d], [a, d]])])
    return polys_from_rings(rings)


def right_triangle(A: float, B: float, x0: float = 0.0, y0: float = 0.0):
    """Triangle (x0,y0), (x0+A,y0), (x0,y0+B)."""
    return polys_from_rings([[np.array([[x0, y0], [x0 + A, y0], [x0, y0 + B]])]])


def star_polygon(V: int, area_frac: float, centre, L: float = EXTENT_M, seed: int = 3,
                 noise: float = 0.3):
    """Star-shaped polygon: theta_j = 2 pi j / V, r_j = R (1 + noise u_j), u ~ U(-1,1).

    R = sqrt(area_frac L^2 / pi) so the expected area is area_frac L^2.
    """
    rng = rng_for(seed, 4, V)
    R = math.sqrt(area_frac * L * L / math.pi)
    th = 2.0 * math.pi * np.arange(V) / V
    r = R * (1.0 + noise * rng.uniform(-1.0, 1.0, size=V))
    ring = np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)
    return polys_from_rings([[ring]])


def road_lines(n_lines: int, n_vertices: int, step: float, seed: int = 7, L: float = EXTENT_M,
               turn: float = 0.35, data_seed: int = 2):
    """Road-like polylines for distance selections: each starts at a point of
    the taxi-like mixture of ``data_seed`` and walks ``n_vertices - 1`` steps
    of length ~ U(0.5, 1.5) ``step`` with a heading that turns by
    N(0, ``turn``) radians per step, clipped to the extent.  Returned as a
    CSR set with one ring (an open polyline) per line."""
    rng = rng_for(seed, 7)
    sx, sy = _mixture_chunk(mixture_params(data_seed, L), n_lines, rng)
    rings = []
    for k in range(n_lines):
        h = rng.uniform(0, 2 * math.pi)
        hs = h + np.cumsum(rng.normal(0.0, turn, size=n_vertices - 1))
        st = step * rng.uniform(0.5, 1.5, size=n_vertices - 1)
        xs = np.concatenate([[sx[k]], sx[k] + np.cumsum(st * np.cos(hs))])
        ys = np.concatenate([[sy[k]], sy[k] + np.cumsum(st * np.sin(hs))])
        rings.append([np.stack([np.clip(xs, 0.0, L), np.clip(ys, 0.0, L)], axis=1)])
    return polys_from_rings(rings)


def query_stars(nq: int, vmin: int, vmax: int, seed: int = 6, L: float = EXTENT_M,
                area=(1e-4, 1e-2), data_seed: int = 2, noise: float = 0.3):
    """A batch of nq star-shaped selection polygons (one per query).

    Vertex counts are log-uniform in [vmin, vmax]; areas are log-uniform in
    ``area`` (fractions of L^2); centres are drawn from the taxi-like mixture
    of ``data_seed`` (queries look where the data is).  Returns (polys,
    qbound) with query q = polygon q.
    """
    rng = rng_for(seed, 6)
    V = np.floor(np.exp(rng.uniform(math.log(vmin), math.log(vmax + 1), size=nq))).astype(np.int64)
    V = np.clip(V, vmin, vmax)
    af = np.exp(rng.uniform(math.log(area[0]), math.log(area[1]), size=nq))
    cx, cy = _mixture_chunk(mixture_params(data_seed, L), nq, rng_for(seed, 7))
    th_off = rng.uniform(0.0, 2.0 * math.pi, size=nq)
    rings = []
    for q in range(nq):
        R = math.sqrt(af[q] * L * L / math.pi)
        th = th_off[q] + 2.0 * math.pi * np.arange(V[q]) / V[q]
        r = R * (1.0 + noise * rng.uniform(-1.0, 1.0, size=V[q]))
        rings.append([np.stack([cx[q] + r * np.cos(th), cy[q] + r * np.sin(th)], axis=1)])
    return polys_from_rings(rings), np.arange(nq + 1, dtype=np.int64)


def census_cells(M: int, vmin: int, vmax: int, seed: int, data_seed: int, L: float = EXTENT_M,
                 return_info: bool = False):
    """Census-block-like tessellation: a Voronoi-jitter tessellation whose
    cell seeds are drawn from the taxi-like mixture of ``data_seed``, so the
    cells are small where the points are dense."""
    sx, sy = _mixture_chunk(mixture_params(data_seed, L), M, rng_for(seed, 9))
    return voronoi_jitter(M, vmin, vmax, seed, L, seed_points=np.stack([sx, sy], 1), return_info=return_info)


WEB_MERCATOR_ORIGIN = (-8.27e6, 4.94e6)   # metres; a New-York-like offset frame


def offset_frame(x, y, polys, L: float = EXTENT_M, origin=WEB_MERCATOR_ORIGIN):
    """Points and polygons of a [0, L)^2 workload moved to a large offset
    frame (coordinates of Web-Mercator size), each coordinate rounded once.

    Shared vertices stay bit-identical (the same addition of the same
    values), and the extent sides move to exactly representable values, so a
    tessellation of the extent stays an exact tiling.  Points whose rounded
    coordinates leave the half-open shifted extent are dropped, so every
    remaining point lies in exactly one cell of such a tessellation.
    """
    ox, oy = float(origin[0]), float(origin[1])
    xs = np.asarray(x, dtype=np.float64) + ox
    ys = np.asarray(y, dtype=np.float64) + oy
    keep = (xs >= ox) & (xs < ox + L) & (ys >= oy) & (ys < oy + L)
    out = dict(polys)
    out["vx"] = np.asarray(polys["vx"], dtype=np.float64) + ox
    out["vy"] = np.asarray(polys["vy"], dtype=np.float64) + oy
    return np.ascontiguousarray(xs[keep]), np.ascontiguousarray(ys[keep]), out


# ------------------------------------------------- Voronoi jitter tessellation

def _seg_intersections_ring(ring):
    """True if a closed ring (n,2) has two non-adjacent edges that touch."""
    n = ring.shape[0]
    if n < 4:
        return False
    a = ring
    b = np.roll(ring, -1, axis=0)

    def orient(p, q, r):
        return (q[..., 0] - p[..., 0]) * (r[..., 1] - p[..., 1]) - \
               (q[..., 1] - p[..., 1]) * (r[..., 0] - p[..., 0])

    A = a[:, None, :]
    B = b[:, None, :]
    C = a[None, :, :]
    D = b[None, :, :]
    o1 = orient(A, B, C)
    o2 = orient(A, B, D)
    o3 = orient(C, D, A)
    o4 = orient(C, D, B)
    hit = (o1 * o2 <= 0) & (o3 * o4 <= 0)
    idx = np.arange(n)
    di = np.abs(idx[:, None] - idx[None, :])
    adjacent = (di <= 1) | (di == n - 1)
    hit &= ~adjacent
    # bounding-box overlap guard for collinear (zero-orientation) false alarms
    bx0 = np.minimum(A[..., 0], B[..., 0]); bx1 = np.maximum(A[..., 0], B[..., 0])
    by0 = np.minimum(A[..., 1], B[..., 1]); by1 = np.maximum(A[..., 1], B[..., 1])
    cx0 = np.minimum(C[..., 0], D[..., 0]); cx1 = np.maximum(C[..., 0], D[..., 0])
    cy0 = np.minimum(C[..., 1], D[..., 1]); cy1 = np.maximum(C[..., 1], D[..., 1])
    hit &= (bx0 <= cx1) & (cx0 <= bx1) & (by0 <= cy1) & (cy0 <= by1)
    return bool(hit.any())


def _ring_area(ring):
    x, y = ring[:, 0], ring[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def voronoi_jitter(M: int, vmin: int, vmax: int, seed: int, L: float = 1.0,
                   seed_points=None, jitter: float = 0.15, return_info: bool = False):
    """Voronoi tessellation of [0,L]^2 with jittered, subdivided shared ridges.

    ``seed_points``: optional (M,2) array of cell seeds (otherwise uniform).
    Per-cell vertex totals are steered into [vmin, vmax]; the achieved counts
    are returned in ``info`` when ``return_info``.
    """
    from scipy.spatial import Voronoi

    rng = rng_for(seed, 5)
    if seed_points is None:
        pts = rng.uniform(0.0, L, size=(M, 2))
    else:
        pts = np.asarray(seed_points, dtype=np.float64).reshape(M, 2)
    # keep seeds strictly inside so mirrors never coincide with originals
    tiny = 1e-7 * L
    pts = np.clip(pts, tiny, L - tiny)
    mirrors = [pts,
               np.stack([-pts[:, 0], pts[:, 1]], 1),
               np.stack([2 * L - pts[:, 0], pts[:, 1]], 1),
               np.stack([pts[:, 0], -pts[:, 1]], 1),
               np.stack([pts[:, 0], 2 * L - pts[:, 1]], 1)]
    vor = Voronoi(np.concatenate(mirrors, 0))
    V = vor.vertices.copy()
    tol = 1e-9 * L
    for col in (0, 1):
        V[np.abs(V[:, col]) < tol, col] = 0.0
        V[np.abs(V[:, col] - L) < tol, col] = L

    # regions of the original seeds, as ordered vertex-index cycles (CCW)
    cells = []
    for i in range(M):
        reg = vor.regions[vor.point_region[i]]
        if -1 in reg or len(reg) < 3:
            raise RuntimeError("unbounded Voronoi cell for an original seed")
        reg = list(reg)
        ring = V[reg]
        if _ring_area(ring) < 0:
            reg = reg[::-1]
        # merge vertices that snapping made identical
        dedup = [reg[0]]
        for v in reg[1:]:
            if not np.array_equal(V[v], V[dedup[-1]]):
                dedup.append(v)
        if np.array_equal(V[dedup[0]], V[dedup[-1]]) and len(dedup) > 1:
            dedup.pop()
        cells.append(dedup)

    def on_side(p, q):
        return ((V[p, 0] == V[q, 0]) and (V[p, 0] in (0.0, L))) or \
               ((V[p, 1] == V[q, 1]) and (V[p, 1] in (0.0, L)))

    # ridges keyed by sorted vertex pair
    ridge_cells = {}
    for k, reg in enumerate(cells):
        n = len(reg)
        for j in range(n):
            p, q = reg[j], reg[(j + 1) % n]
            key = (min(p, q), max(p, q))
            ridge_cells.setdefault(key, []).append(k)
    keys = sorted(ridge_cells)
    deg = np.array([len(c) for c in cells])
    target = rng.integers(vmin, vmax + 1, size=M)
    want = np.maximum(0.0, (target - deg) / np.maximum(deg, 1))
    nsub = {}
    for key in keys:
        cs = ridge_cells[key]
        q = min(want[c] for c in cs)
        nsub[key] = int(math.floor(q))

    def totals():
        t = deg.copy()
        for key in keys:
            for c in ridge_cells[key]:
                t[c] += nsub[key]
        return t

    # steer totals into range: raise cells below target where neighbours have slack
    for _ in range(6):
        tot = totals()
        changed = False
        for k in rng.permutation(M):
            if tot[k] >= max(vmin, min(target[k], vmax)):
                continue
            reg = cells[k]
            n = len(reg)
            for j in range(n):
                if tot[k] >= target[k]:
                    break
                p, q = reg[j], reg[(j + 1) % n]
                key = (min(p, q), max(p, q))
                others = [c for c in ridge_cells[key] if c != k]
                slack = min([vmax - tot[c] for c in others], default=vmax)
                add = int(min(target[k] - tot[k], max(slack, 0), max(1, (target[k] - tot[k]) // max(1, n - j))))
                if add > 0:
                    nsub[key] += add
                    tot[k] += add
                    for c in others:
                        tot[c] += add
                    changed = True
        if not changed:
            break

    # subdivide every ridge once (from the lower vertex index to the higher)
    ridge_u = {key: rng.uniform(-1.0, 1.0, size=nsub[key]) for key in keys}
    scale = {key: 1.0 for key in keys}

    def ridge_pts(key):
        p, q = key
        m = nsub[key]
        if m == 0:
            return np.zeros((0, 2))
        A, B = V[p], V[q]
        t = np.arange(1, m + 1) / (m + 1)
        base = A[None, :] + t[:, None] * (B - A)[None, :]
        if on_side(p, q):
            # stay exactly on the extent side: copy the constant coordinate
            if A[0] == B[0]:
                base[:, 0] = A[0]
            else:
                base[:, 1] = A[1]
            return base
        d = B - A
        ln = math.hypot(d[0], d[1])
        nrm = np.array([-d[1], d[0]]) / ln
        amp = jitter * ln * scale[key] * np.sin(math.pi * t) * ridge_u[key]
        return base + amp[:, None] * nrm[None, :]

    def build_ring(k):
        reg = cells[k]
        n = len(reg)
        out = []
        for j in range(n):
            p, q = reg[j], reg[(j + 1) % n]
            out.append(V[p][None, :])
            key = (min(p, q), max(p, q))
            pts_r = ridge_cells_pts[key]
            out.append(pts_r if p < q else pts_r[::-1])
        return np.concatenate(out, 0)

    bad = list(range(M))
    for attempt in range(12):
        ridge_cells_pts = {key: ridge_pts(key) for key in keys}
        rings = [None] * M
        newbad = []
        for k in range(M):
            ring = build_ring(k)
            rings[k] = ring
            if k in bad or attempt == 0:
                if _ring_area(ring) <= 0 or _seg_intersections_ring(ring):
                    newbad.append(k)
        if not newbad:
            break
        for k in newbad:
            reg = cells[k]
            n = len(reg)
            for j in range(n):
                p, q = reg[j], reg[(j + 1) % n]
                scale[(min(p, q), max(p, q))] *= 0.5
        touched = set(newbad)
        for k in newbad:
            reg = cells[k]
            n = len(reg)
            for j in range(n):
                p, q = reg[j], reg[(j + 1) % n]
                touched.update(ridge_cells[(min(p, q), max(p, q))])
        bad = sorted(touched)
    else:
        raise RuntimeError("could not make every cell simple")

    polys = polys_from_rings([[r] for r in rings])
    if return_info:
        counts = poly_vertex_counts(polys)
        info = {"vertex_counts": counts, "area_sum": float(sum(_ring_area(r) for r in rings)),
                "L": L}
        return polys, info
    return polys
