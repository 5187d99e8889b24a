"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and lays them out; it contains none of
the inclusion method's arithmetic, so both the oracle-side tests and the GPU
side can use it.  The paper tests random points around one polygon
(Section 6.1) and batches of 1e6 points against polygons with 3..15 edges
(Section 6.2); its applications are lidar collision checking against a car
footprint, point queries against polygon databases and rasterisation
(Section 1).  There is no dataset: every array below is drawn from
``numpy.random.Generator(PCG64(BASE_SEED + config_index))``.

Polygons are convex by construction (vertices at sorted angles on a circle),
counter-clockwise, float64.  Points are float32 unless stated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 2007153850


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence([BASE_SEED + config, salt])
    return np.random.Generator(np.random.PCG64(ss))


def circle_polygon(n: int, radius: float, center, rng: np.random.Generator) -> np.ndarray:
    """n vertices at sorted uniform angles on a circle, float64 [n][2], CCW.

    Angles closer than 1e-9 rad are redrawn so that no edge is degenerate.
    """
    for _ in range(100):
        th = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=n))
        gaps = np.diff(np.concatenate([th, [th[0] + 2.0 * math.pi]]))
        if gaps.min() > 1e-9 and gaps.max() < math.pi:  # keeps the centre inside
            break
    V = np.empty((n, 2), dtype=np.float64)
    V[:, 0] = center[0] + radius * np.cos(th)
    V[:, 1] = center[1] + radius * np.sin(th)
    return V


def uniform_points(rng, m: int, lo: float, hi: float, dtype=np.float32) -> np.ndarray:
    """m points uniform in [lo, hi]^2, interleaved x,y ([m][2])."""
    if dtype == np.float32:
        q = rng.random((m, 2), dtype=np.float32)
        q *= np.float32(hi - lo)
        q += np.float32(lo)
        return q
    return rng.uniform(lo, hi, size=(m, 2)).astype(dtype)


def near_edge_points(rng, V: np.ndarray, k: int, max_offset: float) -> np.ndarray:
    """k float64 points within max_offset of the polygon's boundary.

    An edge is drawn with probability proportional to its length, a position
    t ~ U(0, 1) along it and a perpendicular offset s ~ U(-max_offset,
    max_offset).  Pure placement geometry (input generation only).
    """
    W = np.roll(V, 1, axis=0)            # W[i] = v_{i-1}: edge i = W[i] -> V[i]
    e = V - W
    L = np.hypot(e[:, 0], e[:, 1])
    edge = rng.choice(len(V), size=k, p=L / L.sum())
    t = rng.random(k)
    s = rng.uniform(-max_offset, max_offset, size=k)
    nx = e[edge, 1] / L[edge]
    ny = -e[edge, 0] / L[edge]
    px = W[edge, 0] + t * e[edge, 0] + s * nx
    py = W[edge, 1] + t * e[edge, 1] + s * ny
    return np.stack([px, py], axis=1)


# ---------------------------------------------------------------------------
# single polygon, float64 (correctness configuration)
# ---------------------------------------------------------------------------
def single_polygon_fp64(m: int = 1_000_000, n: int = 8, seed_salt: int = 0):
    """8-gon on the unit circle at the origin; m float64 points in [-1.5,1.5]^2."""
    rng = rng_for(1, seed_salt)
    V = circle_polygon(n, 1.0, (0.0, 0.0), rng)
    Q = rng.uniform(-1.5, 1.5, size=(m, 2))
    return V, Q


# ---------------------------------------------------------------------------
# streaming sweep: one polygon, very many float32 points
# ---------------------------------------------------------------------------
STREAM_NS = (3, 4, 8, 16, 32, 64)
STREAM_M = 1 << 28


def streaming_polygon(n: int, seed_salt: int = 0) -> np.ndarray:
    rng = rng_for(2, 1000 * n + seed_salt)
    c = rng.uniform(-0.1, 0.1, size=2)
    return circle_polygon(n, 1.0, c, rng)


def streaming_points(V: np.ndarray, m: int, near_frac: float = 0.01, near_offset: float = 1e-6,
                     seed_salt: int = 0) -> np.ndarray:
    """m float32 points in [-1.5,1.5]^2; floor(near_frac*m) random slots are
    replaced by points within near_offset of an edge (placed in float64, then
    rounded to float32)."""
    rng = rng_for(2, 7919 * len(V) + seed_salt + 1)
    Q = uniform_points(rng, m, -1.5, 1.5)
    k = int(math.floor(near_frac * m))
    if k > 0:
        slots = rng.choice(m, size=k, replace=False)
        Q[slots] = near_edge_points(rng, V, k, near_offset).astype(np.float32)
    return Q


def star_polygon(n: int = 64, r_lo: float = 0.4, r_hi: float = 1.0, seed_salt: int = 0) -> np.ndarray:
    """Simple non-convex polygon (float64 [n][2], counter-clockwise), star-
    shaped about the origin: one angle per sector of 2 pi / n, away from the
    sector ends, radii uniform in [r_lo, r_hi]."""
    rng = rng_for(7, 1000 * n + seed_salt)
    th = (np.arange(n) + rng.uniform(0.1, 0.9, n)) * (2 * np.pi / n)
    r = rng.uniform(r_lo, r_hi, n)
    return np.stack([r * np.cos(th), r * np.sin(th)], 1)


# ---------------------------------------------------------------------------
# uneven batch: thousands of polygons, each with its own point set
# ---------------------------------------------------------------------------
@dataclass
class Batch:
    vtx_off: np.ndarray   # int64 [P+1]
    V: np.ndarray         # float64 [sum n][2]
    pt_off: np.ndarray    # int64 [P+1]
    Q: np.ndarray         # float32 [sum s][2]
    lbl_word_off: np.ndarray  # int64 [P+1], each set starts on a fresh 32-bit word

    @property
    def num_polygons(self) -> int:
        return len(self.vtx_off) - 1

    @property
    def num_tests(self) -> int:
        return int(self.pt_off[-1])


def label_word_offsets(pt_off: np.ndarray) -> np.ndarray:
    sizes = np.diff(pt_off)
    words = (sizes + 31) // 32
    return np.concatenate([[0], np.cumsum(words)]).astype(np.int64)


def uneven_batch(P: int = 4096, size_lo: float = 1e3, size_hi: float = 1e6, n_lo: int = 3,
                 n_hi: int = 32, seed_salt: int = 0) -> Batch:
    """P polygons: n ~ U{n_lo..n_hi}, radius log-uniform [0.5, 50], centre
    uniform in [-1000, 1000]^2; set sizes log-uniform [size_lo, size_hi];
    points gaussian around the centre with sigma = 1.2 * radius (float32)."""
    rng = rng_for(3, seed_salt)
    ns = rng.integers(n_lo, n_hi + 1, size=P)
    radii = np.exp(rng.uniform(math.log(0.5), math.log(50.0), size=P))
    centres = rng.uniform(-1000.0, 1000.0, size=(P, 2))
    sizes = np.rint(np.exp(rng.uniform(math.log(size_lo), math.log(size_hi), size=P))).astype(
        np.int64)
    polys = [circle_polygon(int(ns[k]), float(radii[k]), centres[k], rng) for k in range(P)]
    vtx_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    Q = np.empty((int(pt_off[-1]), 2), dtype=np.float32)
    for k in range(P):
        a, b = pt_off[k], pt_off[k + 1]
        z = rng.standard_normal((b - a, 2), dtype=np.float32)
        z *= np.float32(1.2 * radii[k])
        z += centres[k].astype(np.float32)
        Q[a:b] = z
    return Batch(vtx_off, np.concatenate(polys, axis=0), pt_off, Q, label_word_offsets(pt_off))


# ---------------------------------------------------------------------------
# car footprint, lidar cloud, poses and trajectories
# ---------------------------------------------------------------------------
def car_footprint() -> np.ndarray:
    """4.8 x 1.9 m rectangle with 0.3 m chamfers, centred, CCW (float64)."""
    return np.array([[2.1, -0.95], [2.4, -0.65], [2.4, 0.65], [2.1, 0.95],
                     [-2.1, 0.95], [-2.4, 0.65], [-2.4, -0.65], [-2.1, -0.95]],
                    dtype=np.float64)


def lidar_cloud(points_per_ring: int = 2048, rings: int = 64, r_lo: float = 0.5,
                r_hi: float = 80.0, noise: float = 0.02, config: int = 4,
                seed_salt: int = 0) -> np.ndarray:
    """rings x points_per_ring float32 points: ring ranges log-uniform in
    [r_lo, r_hi], azimuth uniform, +-noise relative range jitter."""
    rng = rng_for(config, 11 + seed_salt)
    base = np.exp(rng.uniform(math.log(r_lo), math.log(r_hi), size=rings))
    az = rng.uniform(0.0, 2.0 * math.pi, size=(rings, points_per_ring))
    rho = base[:, None] * (1.0 + rng.uniform(-noise, noise, size=(rings, points_per_ring)))
    xy = np.stack([rho * np.cos(az), rho * np.sin(az)], axis=-1).reshape(-1, 2)
    return xy.astype(np.float32)


def random_poses(K: int = 2048, extent: float = 40.0, seed_salt: int = 0):
    """K poses: (x, y) uniform in [-extent, extent]^2 and theta uniform in
    [-pi, pi) as float32 [K][3]; (cos, sin) of the float32 theta in float64
    [K][2], drawn once here so nobody recomputes them."""
    rng = rng_for(4, 23 + seed_salt)
    xy = rng.uniform(-extent, extent, size=(K, 2))
    th = rng.uniform(-math.pi, math.pi, size=K)
    poses = np.concatenate([xy, th[:, None]], axis=1).astype(np.float32)
    t64 = poses[:, 2].astype(np.float64)
    cs = np.stack([np.cos(t64), np.sin(t64)], axis=1)
    return poses, cs


def trajectories(T: int = 1024, steps: int = 64, dt: float = 0.1, extent: float = 40.0,
                 seed_salt: int = 0) -> np.ndarray:
    """T unicycle rollouts of `steps` poses, float32 [T][steps][3]."""
    rng = rng_for(5, 31 + seed_salt)
    x = rng.uniform(-extent, extent, size=T)
    y = rng.uniform(-extent, extent, size=T)
    th = rng.uniform(-math.pi, math.pi, size=T)
    v = rng.uniform(2.0, 15.0, size=T)
    w = rng.uniform(-0.3, 0.3, size=T)
    out = np.empty((T, steps, 3), dtype=np.float64)
    for t in range(steps):
        out[:, t, 0], out[:, t, 1], out[:, t, 2] = x, y, th
        x = x + v * np.cos(th) * dt
        y = y + v * np.sin(th) * dt
        th = th + w * dt
    return out.astype(np.float32)


def dyadic_grid(lo: float = -0.5, hi: float = 1.5, k: int = 17) -> np.ndarray:
    """k x k grid of exactly representable points (float64 [k*k][2])."""
    g = np.linspace(lo, hi, k)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


# ---------------------------------------------------------------------------
# polygon database for point location (GIS use, Section 1)
# ---------------------------------------------------------------------------
@dataclass
class Partition:
    vtx_off: np.ndarray   # [P+1] int64
    V: np.ndarray         # [total, 2] float64
    cell_of: np.ndarray   # [P] int64: grid cell (row-major) each polygon came from
    lo: tuple             # domain corner
    hi: tuple             # opposite corner


def jittered_partition(gx: int, gy: int, cell: float = 1.0, jitter: float = 0.2,
                       split: float = 0.5, origin=(0.0, 0.0), config: int = 6,
                       seed_salt: int = 0) -> Partition:
    """A planar partition of [origin, origin + (gx, gy) * cell] into convex
    cells: grid vertices moved by up to `jitter` * cell in each coordinate
    (multiples of 2^-10 cell, so shared vertices are exactly equal), each
    quad kept (counter-clockwise) or, with probability `split`, cut along its
    diagonal into two triangles.  Cells are listed row by row.  A jitter of
    at most 0.25 keeps every quad convex."""
    rng = rng_for(config, seed_salt)
    q = 1024.0
    jx = np.rint(rng.uniform(-jitter, jitter, size=(gy + 1, gx + 1)) * q) / q
    jy = np.rint(rng.uniform(-jitter, jitter, size=(gy + 1, gx + 1)) * q) / q
    I, J = np.meshgrid(np.arange(gx + 1), np.arange(gy + 1))
    X = origin[0] + (I + jx) * cell
    Y = origin[1] + (J + jy) * cell
    cut = rng.random((gy, gx)) < split
    polys, cells = [], []
    for j in range(gy):
        for i in range(gx):
            a = (X[j, i], Y[j, i])
            b = (X[j, i + 1], Y[j, i + 1])
            c = (X[j + 1, i + 1], Y[j + 1, i + 1])
            d = (X[j + 1, i], Y[j + 1, i])
            if cut[j, i]:
                polys += [np.array([a, b, c]), np.array([a, c, d])]
                cells += [j * gx + i, j * gx + i]
            else:
                polys.append(np.array([a, b, c, d]))
                cells.append(j * gx + i)
    ns = np.array([len(p) for p in polys])
    vtx_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    lo = (origin[0] - jitter * cell, origin[1] - jitter * cell)
    hi = (origin[0] + (gx + jitter) * cell, origin[1] + (gy + jitter) * cell)
    return Partition(vtx_off, np.concatenate(polys).astype(np.float64), np.array(cells), lo, hi)


def locate_points(part: Partition, m: int, margin: float = 0.02, config: int = 6,
                  seed_salt: int = 1) -> np.ndarray:
    """m float32 query points uniform over the partition's domain widened by
    `margin` of its size on each side (a few fall outside every cell)."""
    rng = rng_for(config, seed_salt)
    w = (part.hi[0] - part.lo[0], part.hi[1] - part.lo[1])
    x = rng.uniform(part.lo[0] - margin * w[0], part.hi[0] + margin * w[0], m)
    y = rng.uniform(part.lo[1] - margin * w[1], part.hi[1] + margin * w[1], m)
    return np.stack([x, y], 1).astype(np.float32)
