"""Pins of the FP64 oracle against facts fixed outside the oracle.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises
``AssertionError`` when the oracle disagrees with a closed form, an exact
rational evaluation, a hand-worked fixture (``tests/golden``) or an invariant
that the paper's mathematics fixes.  ``test_oracle_pins.py`` runs them on the
real oracle; ``test_oracle_mutants.py`` runs them on copies of the oracle with
a planted mistake and requires that some pin fails.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import exact
import polydecomp
from oracle import pack_bits, unpack_bits
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _rng(salt):
    return np.random.default_rng(1234 + salt)


def small_int_convex(rng, n, scale=20):
    """Convex polygon with small-integer vertices (CCW): a random convex hull."""
    for _ in range(1000):
        pts = rng.integers(-scale, scale + 1, size=(4 * n, 2))
        hull = _hull(pts)
        if len(hull) >= 3:
            return np.array(hull[:], dtype=np.float64)
    raise RuntimeError("no hull")


def _hull(pts):
    pts = sorted(set(map(tuple, pts.tolist())))
    if len(pts) < 3:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


# ---------------------------------------------------------------------------
# Section 3: centroid and generators
# ---------------------------------------------------------------------------
def pin_square_and_triangle(o):
    sq = golden("unit_square.json")
    V = np.array(sq["vertices_ccw"], dtype=float)
    g0, area, rc = o.centroid(V)
    assert rc == 0 and area == sq["area_ccw"] and list(g0) == sq["centroid"]
    P, rc = o.generators(V)
    assert rc == 0 and P.tolist() == sq["generators_ccw"], P
    g0, area, _ = o.centroid(V[::-1])
    assert area == -1.0 and list(g0) == sq["centroid"]          # CW: signed area
    tri = golden("triangle.json")
    V = np.array(tri["vertices"], dtype=float)
    g0, area, _ = o.centroid(V)
    assert area == tri["area"] and list(g0) == tri["centroid"]
    P, _ = o.generators(V)
    assert P.tolist() == tri["generators"], P


def pin_regular_ngon(o):
    """Regular n-gon of radius R: area (n/2) R^2 sin(2 pi/n), centroid at the
    centre, generator of edge j at distance 2 R cos(pi/n) from the centre at
    the mid-angle of the edge."""
    for n in (3, 5, 8, 13, 64):
        R = 2.5
        th = 2 * math.pi * np.arange(n) / n
        V = np.stack([R * np.cos(th), R * np.sin(th)], 1)
        g0, area, _ = o.centroid(V)
        assert abs(area - 0.5 * n * R * R * math.sin(2 * math.pi / n)) < 1e-12 * R * R
        assert np.all(np.abs(g0) < 1e-14 * R)
        P, _ = o.generators(V)
        for j in range(n):
            mid = th[j] - math.pi / n          # edge j runs v_{j-1} -> v_j
            want = 2 * R * math.cos(math.pi / n) * np.array([math.cos(mid), math.sin(mid)])
            assert np.allclose(P[1 + j], want, rtol=0, atol=1e-13 * R), (n, j)


def pin_generators_exact_rational(o):
    """Random small-integer convex polygons: float64 centroid and generators
    agree with exact rationals to a few units in the last place."""
    rng = _rng(1)
    for t in range(30):
        V = small_int_convex(rng, 6 + t % 5)
        if t % 3 == 2:
            V = V[::-1].copy()
        Pe = exact.generators(V.tolist())
        P, rc = o.generators(V)
        assert rc == 0
        scale = np.abs(V).max() + 1
        for (ex, ey), (fx, fy) in zip(Pe, P):
            assert abs(float(ex) - fx) <= 1e-13 * scale and abs(float(ey) - fy) <= 1e-13 * scale


def pin_generator_invariants(o):
    """Eq. 2: every point of edge i is equidistant from p_0 and p_i; Eq. 6:
    the midpoint of p_0 p_i lies on edge line i and p_i - p_0 is
    perpendicular to it; |p_i - p_0| = 2 dist(p_0, line i)."""
    rng = _rng(2)
    for t in range(20):
        n = int(rng.integers(3, 20))
        c = rng.uniform(-5, 5, 2)
        V = W.circle_polygon(n, float(rng.uniform(0.1, 10)), c, rng)
        P, _ = o.generators(V)
        g0 = P[0]
        for i in range(n):
            a, b = V[i - 1], V[i]
            e = b - a
            gi = P[1 + i]
            h = gi - g0
            L = np.hypot(*e)
            scale = np.abs(V).max() ** 2 + 1
            for s in (0.0, 0.25, 0.5, 1.0):
                x = a + s * e
                d0 = np.sum((x - g0) ** 2)
                di = np.sum((x - gi) ** 2)
                assert abs(d0 - di) <= 1e-12 * scale
            mid = 0.5 * (g0 + gi)
            assert abs(e[0] * (mid[1] - a[1]) - e[1] * (mid[0] - a[0])) <= 1e-12 * scale
            assert abs(np.dot(h, e)) <= 1e-12 * scale
            dist = abs(e[0] * (g0[1] - a[1]) - e[1] * (g0[0] - a[0])) / L
            assert abs(np.hypot(*h) - 2 * dist) <= 1e-12 * math.sqrt(scale)


def pin_degenerate_status(o):
    _, rc = o.generators(np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]]))
    assert rc == -1                       # zero area
    _, rc = o.generators(np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
    assert rc == -2                       # zero-length edge


# ---------------------------------------------------------------------------
# Algorithms 1, 2, 5 on exact inputs
# ---------------------------------------------------------------------------
def pin_unit_square_grid(o):
    sq = golden("unit_square.json")
    G = W.dyadic_grid(sq["grid"]["lo"], sq["grid"]["hi"], sq["grid"]["k"])
    V = np.array(sq["vertices_ccw"], dtype=float)
    want = sq["grid_inside_counts"]
    for orient, VV in (("ccw", V), ("cw", V[::-1].copy())):
        assert int(o.voronoi(VV, G).sum()) == want["voronoi"][orient]
        assert int(o.sign_of_offset(VV, G).sum()) == want["sign_of_offset"][orient]
        assert int(o.ray_crossing(VV, G).sum()) == want["ray_crossing"][orient]
    # the 81 Voronoi points are exactly the closed square, the 64 ray
    # crossing points exactly [0,1)^2
    vin = o.voronoi(V, G)
    closed = (G[:, 0] >= 0) & (G[:, 0] <= 1) & (G[:, 1] >= 0) & (G[:, 1] <= 1)
    assert np.array_equal(vin, closed)
    half = (G[:, 0] >= 0) & (G[:, 0] < 1) & (G[:, 1] >= 0) & (G[:, 1] < 1)
    assert np.array_equal(o.ray_crossing(V, G), half)


def pin_exact_rational_labels(o):
    """Small-integer polygons, dyadic points: all three float64 tests equal
    the exact-rational evaluation of the same algorithm, and the exact
    Voronoi predicate equals the closed half-plane definition of the convex
    polygon (brute force), whenever the point is not within float64 reach of
    the boundary.  Points exactly on a vertex or edge are included: the exact
    Voronoi answer there is 'inside'."""
    rng = _rng(3)
    checked = 0
    for t in range(12):
        V = small_int_convex(rng, 5 + t % 4, scale=8)
        if t % 2:
            V = V[::-1].copy()
        Pe = exact.generators(V.tolist())
        pts = rng.integers(-40, 41, size=(150, 2)) / 4.0
        pts = np.concatenate([pts, V, 0.5 * (V + np.roll(V, 1, 0))])
        vor = o.voronoi(V, pts)
        soo = o.sign_of_offset(V, pts)
        ray = o.ray_crossing(V, pts)
        P, _ = o.generators(V)
        Pf = [(float(x), float(y)) for x, y in Pe]
        for k, p in enumerate(pts.tolist()):
            ve = exact.voronoi(V.tolist(), p, Pe)
            assert ve == exact.convex_contains(V.tolist(), p)
            margins = exact.voronoi_margins(Pe, p)
            mmax = max(margins)
            # float64 error of the oracle's squared distances, generously
            r2 = max((p[0] - gx) ** 2 + (p[1] - gy) ** 2 for gx, gy in Pf)
            gen_err = 1e-12 * (np.abs(V).max() + abs(p[0]) + abs(p[1]) + 1) ** 2
            if abs(float(mmax)) > 1e-13 * r2 + gen_err:
                assert bool(vor[k]) == ve, (t, p)
            assert bool(soo[k]) == exact.sign_of_offset(V.tolist(), p), (t, p)
            assert bool(ray[k]) == exact.ray_crossing(V.tolist(), p), (t, p)
            checked += 1
        # generators in float64 match the exact ones closely
        assert np.allclose(P, np.array(Pf), rtol=0, atol=1e-12 * (np.abs(V).max() + 1))
    assert checked > 1000


def pin_three_tests_agree_away_from_edges(o):
    """The paper's own correctness experiment (Section 6.1): on random points
    around a polygon the Voronoi labels equal sign-of-offset labels; ray
    crossing agrees too.  Points within 1e-9 of an edge line are skipped
    (boundary conventions differ there by design)."""
    rng = _rng(4)
    for t in range(6):
        n = int(rng.integers(3, 16))
        V = W.circle_polygon(n, 1.0, rng.uniform(-0.1, 0.1, 2), rng)
        if t % 2:
            V = V[::-1].copy()
        Q = rng.uniform(-1.5, 1.5, size=(20000, 2))
        Wv = np.roll(V, 1, 0)
        e = V - Wv
        L = np.hypot(e[:, 0], e[:, 1])
        d = np.abs((e[None, :, 0] * (Q[:, None, 1] - Wv[None, :, 1]) -
                    e[None, :, 1] * (Q[:, None, 0] - Wv[None, :, 0])) / L[None, :])
        far = d.min(axis=1) > 1e-9
        a, b, c = o.voronoi(V, Q), o.sign_of_offset(V, Q), o.ray_crossing(V, Q)
        assert np.array_equal(a[far], b[far]) and np.array_equal(a[far], c[far])
        assert 0.1 < a.mean() < 0.6


def pin_label_invariants(o):
    """Labels are invariant under translation and 90-degree rotation for
    points off the edge lines, convex combinations of vertices with
    weights >= 1e-3 are inside, and reflecting an interior point across an
    edge line (landing >= 1e-9 from it) gives an outside point."""
    rng = _rng(5)
    for t in range(8):
        V = small_int_convex(rng, 7, scale=16)
        Q = rng.integers(-80, 81, size=(2000, 2)) / 4.0
        base = o.voronoi(V, Q)
        # the centroid divides by 6A, so generators are rounded: points on an
        # edge line may flip under a motion; compare the rest
        far = _min_edge_dist(V, Q) > 1e-9
        sh = np.array([64.0, -32.0])
        assert np.array_equal(base[far], o.voronoi(V + sh, Q + sh)[far])
        rot = lambda A: np.stack([-A[:, 1], A[:, 0]], 1)
        assert np.array_equal(base[far], o.voronoi(rot(V), rot(Q))[far])
        wts = rng.uniform(1e-3, 1.0, size=(500, len(V)))
        wts /= wts.sum(1, keepdims=True)
        inner = wts @ V
        for test in (o.voronoi, o.sign_of_offset, o.ray_crossing):
            assert test(V, inner).all()
        i = int(rng.integers(len(V)))
        a, b = V[i - 1], V[i]
        e = (b - a) / np.hypot(*(b - a))
        nrm = np.array([e[1], -e[0]])
        dist = (inner - a) @ nrm
        refl = inner - 2 * dist[:, None] * nrm[None, :]
        keep = np.abs(dist) > 1e-9
        assert not o.voronoi(V, refl[keep]).any()
        assert not o.sign_of_offset(V, refl[keep]).any()
        assert not o.ray_crossing(V, refl[keep]).any()


def pin_nonfinite_points(o):
    V = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=float)
    Q = np.array([[np.nan, 0.5], [0.5, np.inf], [-np.inf, 0.5], [0.5, 0.5]])
    assert o.voronoi(V, Q).tolist() == [False, False, False, True]


def pin_max_margin(o):
    """The largest margin is <= 0 exactly for the inside points and equals
    the exact rational max margin on dyadic data."""
    rng = _rng(6)
    V = small_int_convex(rng, 6, scale=8)
    Q = rng.integers(-40, 41, size=(300, 2)) / 4.0
    mm = o.voronoi_max_margin(V, Q)
    assert np.array_equal(mm <= 0, o.voronoi(V, Q))
    Pe = exact.generators(V.tolist())
    for k, p in enumerate(Q.tolist()):
        want = float(max(exact.voronoi_margins(Pe, p)))
        assert abs(want - mm[k]) <= 1e-11 * (1 + abs(p[0]) + abs(p[1])) ** 2 * 64


# ---------------------------------------------------------------------------
# poses, all pairs
# ---------------------------------------------------------------------------
def pin_pose_polygon(o):
    F = W.car_footprint()
    Wp = o.pose_polygon(F, 3.0, -2.0, 0.0, 1.0)            # theta = pi/2
    assert np.array_equal(Wp, np.stack([-F[:, 1] + 3.0, F[:, 0] - 2.0], 1))
    Wp = o.pose_polygon(F, 0.5, 0.25, 1.0, 0.0)
    assert np.array_equal(Wp, F + np.array([0.5, 0.25]))


def pin_allpairs(o):
    F = W.car_footprint()
    rng = _rng(7)
    K = 6
    xy = rng.uniform(-3, 3, size=(K, 2))
    th = rng.uniform(-math.pi, math.pi, K)
    cs = np.stack([np.cos(th), np.sin(th)], 1)
    Q = rng.uniform(-6, 6, size=(1000, 2))
    bits, counts = o.allpairs(F, xy, cs, Q)
    for k in range(K):
        # inside the rotated, shifted footprint == inside the footprint after
        # undoing the motion (brute force half-plane test, away from edges)
        d = Q - xy[k]
        body = np.stack([cs[k, 0] * d[:, 0] + cs[k, 1] * d[:, 1],
                         -cs[k, 1] * d[:, 0] + cs[k, 0] * d[:, 1]], 1)
        lab = unpack_bits(bits[k], len(Q))
        inside = np.array([exact.convex_contains(F.tolist(), p) for p in body.tolist()])
        ok = _min_edge_dist(F, body) > 1e-9
        assert np.array_equal(lab[ok], inside[ok])
        assert counts[k] == lab.sum()
        assert np.array_equal(bits[k], pack_bits(lab))


def pin_raster_exact(o):
    """Dyadic raster of the rectangle [0,1] x [0,1/2]: exactly the pixels of
    the closed rectangle (fixture worked by hand), in either orientation."""
    g = golden("raster_unit_square.json")
    V = np.array(g["vertices_ccw"], dtype=float)
    r = g["raster"]
    (c0, c1), (r0, r1) = g["inside_columns"], g["inside_rows"]
    want = np.zeros((r["height"], r["width"]), dtype=bool)
    want[r0:r1 + 1, c0:c1 + 1] = True
    assert int(want.sum()) == g["inside_count"]
    for VV in (V, V[::-1].copy()):
        got = o.voronoi_raster(VV, r["x0"], r["y0"], r["dx"], r["dy"], r["width"], r["height"])
        assert np.array_equal(got, want)


def pin_raster_area(o):
    """Coverage of a regular heptagon and a triangle on non-square rasters:
    pixel count times pixel area is the polygon's area (closed form) within
    the cells the boundary crosses, perimeter (dx + dy) + 4 dx dy; and the
    raster equals the labels of its pixel points formed here row by row."""
    cases = ((7, 1.0, (0.3, -0.2), 301, 257), (3, 2.5, (-4.0, 7.0), 190, 333))
    for n, R, c, width, height in cases:
        th = 2 * math.pi * np.arange(n) / n + 0.1
        V = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th)], 1)
        x0, y0 = c[0] - 1.3 * R, c[1] - 1.2 * R
        dx, dy = 2.6 * R / (width - 1), 2.4 * R / (height - 1)
        got = o.voronoi_raster(V, x0, y0, dx, dy, width, height)
        assert got.shape == (height, width)
        area = 0.5 * n * R * R * math.sin(2 * math.pi / n)
        per = n * 2 * R * math.sin(math.pi / n)
        assert abs(got.sum() * dx * dy - area) <= per * (dx + dy) + 4 * dx * dy
        px = x0 + np.arange(width) * dx
        py = y0 + np.arange(height) * dy
        X, Y = np.meshgrid(px, py)              # [height, width], row j holds y_j
        Q = np.stack([X.reshape(-1), Y.reshape(-1)], 1)
        assert np.array_equal(got.reshape(-1), o.voronoi(V, Q))


def pin_locate_hand_worked(o):
    """Four unit squares (fixture worked by hand): shared corners and edges go
    to the smallest containing index, points outside to -1."""
    g = golden("locate_2x2.json")
    polys = [np.array(p, dtype=float) for p in g["polygons"]]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])])
    ids = o.locate(off, np.concatenate(polys), np.array(g["points"], dtype=float))
    assert ids.tolist() == g["ids"]
    bad = o.locate(off, np.concatenate(polys), np.array([[np.nan, 1.0], [1.0, np.inf]]))
    assert bad.tolist() == [-1, -1]


def pin_locate_partition(o):
    """A jittered partition into convex quads and triangles: points strictly
    inside cell k (convex combinations of its vertices with weights >= 1e-3,
    so at least ~1e-4 from every edge) locate to k, since cells have disjoint
    interiors; points outside the domain locate to -1."""
    rng = _rng(31)
    part = W.jittered_partition(9, 7, cell=0.5, origin=(-3.0, 1.0), seed_salt=3)
    off, V = part.vtx_off, part.V
    pts, want = [], []
    for k in range(len(off) - 1):
        Pk = V[off[k]:off[k + 1]]
        w = rng.uniform(1e-3, 1.0, size=(6, len(Pk)))
        w /= w.sum(1, keepdims=True)
        pts.append(w @ Pk)
        want += [k] * 6
    out = np.array([[part.lo[0] - 0.01, 2.0], [part.hi[0] + 0.3, 2.0], [0.0, part.hi[1] + 1.0],
                    [0.0, part.lo[1] - 1e-3]])
    ids = o.locate(off, V, np.concatenate(pts + [out]))
    assert ids[:len(want)].tolist() == want
    assert (ids[len(want):] == -1).all()


def pin_locate_overlapping(o):
    """Nested and overlapping polygons: the id is the smallest index whose
    polygon contains the point (exact rational membership, points away from
    edges), in either listing order."""
    rng = _rng(32)
    polys = [small_int_convex(rng, int(rng.integers(3, 9)), scale=12) for _ in range(14)]
    Q = rng.uniform(-13, 13, size=(3000, 2))
    ok = np.min([_min_edge_dist(p, Q) for p in polys], axis=0) > 1e-6
    for order in (polys, polys[::-1]):
        off = np.concatenate([[0], np.cumsum([len(p) for p in order])])
        ids = o.locate(off, np.concatenate(order).astype(float), Q)
        for j in np.nonzero(ok)[0][:600]:
            inside = [k for k, p in enumerate(order) if exact.convex_contains(p.tolist(), Q[j].tolist())]
            assert ids[j] == (inside[0] if inside else -1), j


def _min_edge_dist(V, Q):
    Wv = np.roll(V, 1, 0)
    e = V - Wv
    L = np.hypot(e[:, 0], e[:, 1])
    d = np.abs((e[None, :, 0] * (Q[:, None, 1] - Wv[None, :, 1]) -
                e[None, :, 1] * (Q[:, None, 0] - Wv[None, :, 0])) / L[None, :])
    return d.min(axis=1)


# ---------------------------------------------------------------------------
# collision cost and its gradient
# ---------------------------------------------------------------------------
def _footprint(spec):
    return W.car_footprint() if spec == "car" else np.array(spec, dtype=float)


def pin_cost_fixtures(o):
    for case in golden("collision_cost.json")["cases"]:
        F = _footprint(case["footprint"])
        c = o.cost(F, np.array([case["pose"]]), np.array(case["points"], dtype=float))
        assert abs(c[0] - case["cost"]) < 1e-12, (case, c)


def pin_cost_rigid_invariance(o):
    """Moving the points and the pose by the same rigid motion leaves the
    cost unchanged."""
    rng = _rng(8)
    F = W.car_footprint()
    Q = rng.uniform(-4, 4, size=(3000, 2))
    pose = np.array([[0.3, -0.2, 0.4]])
    c0 = o.cost(F, pose, Q)[0]
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    t = np.array([5.0, -3.0])
    Q2 = Q @ R.T + t
    p2 = np.array([[*(R @ pose[0, :2] + t), pose[0, 2] + a]])
    c1 = o.cost(F, p2, Q2)[0]
    assert c0 > 0 and abs(c0 - c1) < 1e-10 * max(1.0, c0)


def _fd_cost(o, F, poses, Q, h=1e-6):
    """Central differences of the oracle cost; entries whose (active,
    argmin) state changes between +h and -h are marked invalid."""
    K = len(poses)
    gp = np.zeros((K, 3))
    okp = np.ones((K, 3), dtype=bool)
    for k in range(K):
        for d in range(3):
            pp = poses[k].copy()
            pm = poses[k].copy()
            pp[d] += h
            pm[d] -= h
            cp = o.cost(F, pp[None], Q)[0]
            cm = o.cost(F, pm[None], Q)[0]
            gp[k, d] = (cp - cm) / (2 * h)
            okp[k, d] = np.array_equal(o.cost_state(F, pp, Q), o.cost_state(F, pm, Q))
    gF = np.zeros_like(F)
    okF = np.ones(F.shape, dtype=bool)
    for i in range(len(F)):
        for d in range(2):
            Fp = F.copy()
            Fm = F.copy()
            Fp[i, d] += h
            Fm[i, d] -= h
            gF[i, d] = (o.cost(Fp, poses, Q).sum() - o.cost(Fm, poses, Q).sum()) / (2 * h)
            okF[i, d] = all(np.array_equal(o.cost_state(Fp, poses[k], Q),
                                           o.cost_state(Fm, poses[k], Q)) for k in range(K))
    return gp, okp, gF, okF


def pin_cost_gradient_fd(o):
    """The closed-form reference gradient matches float64 central finite
    differences (h = 1e-6) of the cost to pose and to footprint vertices."""
    rng = _rng(9)
    F = W.car_footprint()
    Q = rng.uniform(-3, 3, size=(400, 2))
    poses = np.stack([rng.uniform(-0.5, 0.5, 4), rng.uniform(-0.5, 0.5, 4),
                      rng.uniform(-math.pi, math.pi, 4)], 1)
    gp, gF = o.cost_grad(F, poses, Q)
    fp, okp, fF, okF = _fd_cost(o, F, poses, Q)
    assert okp.sum() >= 10 and okF.sum() >= 12
    assert np.all(np.abs(gp - fp)[okp] <= 1e-5 * (1 + np.abs(fp)[okp]))
    assert np.all(np.abs(gF - fF)[okF] <= 1e-5 * (1 + np.abs(fF)[okF]))
    # weighted form: w scales pose rows and the footprint sum
    w = rng.uniform(0.5, 2.0, len(poses))
    gpw, gFw = o.cost_grad(F, poses, Q, w)
    assert np.allclose(gpw, gp * w[:, None], rtol=1e-12, atol=1e-12)
    gF_sum = sum(o.cost_grad(F, poses[k:k + 1], Q, w[k:k + 1])[1] for k in range(len(poses)))
    assert np.allclose(gFw, gF_sum, rtol=1e-10, atol=1e-10)


def pin_cost_gradient_cw(o):
    """A clockwise footprint describes the same set: same cost, same pose
    gradient, and the vertex gradient permuted with the vertex order."""
    rng = _rng(10)
    F = W.car_footprint()
    Fcw = F[::-1].copy()
    Q = rng.uniform(-3, 3, size=(500, 2))
    poses = np.array([[0.1, 0.2, 0.3], [-0.2, 0.1, -1.0]])
    assert np.allclose(o.cost(F, poses, Q), o.cost(Fcw, poses, Q), rtol=1e-12, atol=1e-12)
    gp, gF = o.cost_grad(F, poses, Q)
    gp2, gF2 = o.cost_grad(Fcw, poses, Q)
    assert np.allclose(gp, gp2, rtol=1e-9, atol=1e-9)
    assert np.allclose(gF, gF2[::-1], rtol=1e-9, atol=1e-9)


def pin_cost_hash(o):
    """oracle_cost_with_hash returns the same costs as oracle_cost, a hash
    that changes when one point crosses the footprint boundary, and the
    same hash when a far point moves a little."""
    rng = _rng(11)
    F = W.car_footprint()
    Q = rng.uniform(-3, 3, size=(800, 2))
    poses = np.array([[0.1, 0.0, 0.2], [0.5, -0.3, 1.1]])
    c, h = o.cost_with_hash(F, poses, Q)
    assert np.allclose(c, o.cost(F, poses, Q), rtol=0, atol=0)
    Q2 = Q.copy()
    Q2[0] = [0.0, 0.0]          # now inside both placements
    Q2[1] = [50.0, 50.0]
    _, h2 = o.cost_with_hash(F, poses, Q2)
    Q3 = Q2.copy()
    Q3[1] = [50.0, 50.5]        # far point moves: state unchanged
    _, h3 = o.cost_with_hash(F, poses, Q3)
    assert np.all(h2 == h3) and np.any(h != h2)
    gp, gF, ap, aF = o.cost_grad(F, poses, Q, with_scale=True)
    assert np.all(np.abs(gp) <= ap + 1e-12) and np.all(np.abs(gF) <= aF + 1e-12)


def pin_cost_argmin(o):
    """Hand-worked states of the unit square (``tests/golden/cost_argmin_square.json``):
    the minimising edge of each inside point, the lowest index on exact
    ties, -1 on the boundary and outside; the cost and the pose gradient,
    which follows the tie rule (every value is exact in binary64)."""
    g = golden("cost_argmin_square.json")
    F = np.array(g["footprint"], dtype=float)
    pose = np.array(g["pose"], dtype=float)
    Q = np.array(g["points"], dtype=float)
    st = o.cost_state(F, pose, Q)
    assert st.tolist() == g["state"], st
    assert o.cost(F, pose[None], Q)[0] == g["cost"]
    gp, _ = o.cost_grad(F, pose[None], Q)
    assert gp[0].tolist() == g["grad_pose"], gp
    # the hash follows the state: a tie point nudged towards its second edge
    # changes the hash, and nudging it towards its own edge does not
    _, h0 = o.cost_with_hash(F, pose[None], Q)
    Q1 = Q.copy()
    Q1[4] = [0.25 + 2.0 ** -20, 0.25]   # now edge 1 is nearer
    _, h1 = o.cost_with_hash(F, pose[None], Q1)
    Q2 = Q.copy()
    Q2[4] = [0.25 - 2.0 ** -20, 0.25]   # edge 0 stays the minimum
    _, h2 = o.cost_with_hash(F, pose[None], Q2)
    assert h1[0] != h0[0] and h2[0] == h0[0]


def pin_locate_far_rounding(o):
    """Far beyond a polygon, Algorithm 5's binary64 squared distances all
    round to one value: for p = (2^100, 2^100) and generators of magnitude
    below 2^40, every p - g rounds to 2^100 and every squared distance to
    2^201, so M_0 <= M_i holds for every edge and the smallest index wins
    (the y terms of (2^100, 2^20), about 2^40, are absorbed below the
    spacing 2^148 of 2^200, so that point is inside too).  At (2^20, 2^20)
    the margins (about 2^21) dwarf the rounding (about 2^-12): outside."""
    polys = [np.array([[2.0, 0], [3, 0], [3, 1], [2, 1]]), np.array([[0.0, 0], [1, 0], [0, 1]])]
    off = np.array([0, 4, 7])
    V = np.concatenate(polys)
    Q = np.array([[2.0 ** 100, 2.0 ** 100], [-(2.0 ** 100), 2.0 ** 100]])
    assert o.locate(off, V, Q).tolist() == [0, 0]
    assert o.voronoi(polys[1], Q).tolist() == [True, True]
    assert o.voronoi(polys[1], np.array([[2.0 ** 100, 2.0 ** 20]])).tolist() == [True]
    assert o.locate(off, V, np.array([[2.0 ** 20, 2.0 ** 20]])).tolist() == [-1]



def _pieces_exact_union(V, off, idx, p):
    """Exact union-of-pieces label: some piece's exact Voronoi predicate
    (Eq. 1 in rationals) holds."""
    for k in range(len(off) - 1):
        piece = [tuple(V[i]) for i in idx[off[k]:off[k + 1]]]
        if exact.voronoi(piece, p):
            return True
    return False


def pin_pieces_L_shape_exact(o):
    """L-shaped polygon (a collinear vertex at (0, 2) closes the cut) split
    into a 4 x 2 rectangle and a 2 x 2 square: every centroid, generator and
    squared distance is dyadic, so on a dyadic grid the float64 union of the
    two closed Voronoi tests is exactly the closed L: the points with
    0 <= x <= 4, 0 <= y <= 2 or 0 <= x <= 2, 0 <= y <= 4 (boundary and cut
    included)."""
    V = np.array([[0, 0], [4, 0], [4, 2], [2, 2], [2, 4], [0, 4], [0, 2]], dtype=np.float64)
    off = np.array([0, 5, 9], np.int64)
    idx = np.array([0, 1, 2, 3, 6, 6, 3, 4, 5], np.int64)
    g = np.arange(-4, 21) / 4.0
    X, Y = np.meshgrid(g, g)
    Q = np.stack([X.ravel(), Y.ravel()], 1)
    got = o.voronoi_pieces(V, off, idx, Q)
    x, y = Q[:, 0], Q[:, 1]
    want = ((x >= 0) & (x <= 4) & (y >= 0) & (y <= 2)) | ((x >= 0) & (x <= 2) & (y >= 0) & (y <= 4))
    assert np.array_equal(got, want), int((got != want).sum())
    assert int(want.sum()) == 17 * 9 + 9 * 8
    # piece order does not matter; a reversed index list (other orientation) neither
    off2 = np.array([0, 4, 9], np.int64)
    idx2 = np.array([5, 4, 3, 6, 6, 3, 2, 1, 0], np.int64)
    assert np.array_equal(o.voronoi_pieces(V, off2, idx2, Q), want)


def pin_pieces_exact_rational(o):
    """Small-integer simple non-convex polygons, decomposed exactly (ear
    clipping, merged and unmerged): the exact union of the pieces' closed
    Voronoi predicates is the closed polygon (exact brute force), and the
    float64 label equals it wherever no piece's exact largest margin lies
    within float64 reach of zero."""
    rng = _rng(21)
    checked = 0
    for t in range(8):
        V = polydecomp.star_polygon(rng, 7 + t % 5, r_lo=0.35, r_hi=1.0, integer_scale=9)
        if t % 2:
            V = V[::-1].copy()
        off, idx = polydecomp.decompose(V, merged=t % 3 != 0)
        Vl = [tuple(v) for v in V.tolist()]
        pts = rng.integers(-44, 45, size=(120, 2)) / 4.0
        mids = [0.5 * (V[i] + V[i - 1]) for i in range(len(V))]
        diag = [0.5 * (V[idx[off[k] + a]] + V[idx[off[k] + (a + 1) % (off[k + 1] - off[k])]])
                for k in range(len(off) - 1) for a in range(off[k + 1] - off[k])]
        pts = np.concatenate([pts, V, np.array(mids), np.array(diag)])
        got = o.voronoi_pieces(V, off, idx, pts)
        gens = []
        for k in range(len(off) - 1):
            piece = [Vl[i] for i in idx[off[k]:off[k + 1]]]
            gens.append((piece, exact.generators(piece)))
        for q, p in enumerate(pts.tolist()):
            ex = any(exact.voronoi(pc, p, Pe) for pc, Pe in gens)
            assert ex == polydecomp.closed_contains(Vl, p), (t, p)
            near = False
            for pc, Pe in gens:
                mm = max(exact.voronoi_margins(Pe, p))
                r2 = max((p[0] - float(gx)) ** 2 + (p[1] - float(gy)) ** 2 for gx, gy in Pe)
                if abs(float(mm)) <= 1e-13 * r2 + 1e-12 * (np.abs(V).max() + abs(p[0]) + abs(p[1]) + 1) ** 2:
                    near = True
            if not near:
                assert bool(got[q]) == ex, (t, p)
                checked += 1
    assert checked > 800


def pin_pieces_single_and_fan(o):
    """A convex polygon given as one piece is Algorithm 5 itself (labels
    bit-identical to the convex test); split into a fan of triangles from
    vertex 0 it has the same labels away from the fan's diagonals."""
    rng = _rng(22)
    for t in range(4):
        n = 5 + 4 * t
        V = W.circle_polygon(n, 1.0, rng.uniform(-0.2, 0.2, 2), rng)
        Q = rng.uniform(-1.3, 1.3, (20000, 2))
        one = o.voronoi_pieces(V, np.array([0, n]), np.arange(n), Q)
        assert np.array_equal(one, o.voronoi(V, Q))
        off = 3 * np.arange(n - 1)
        idx = np.array([[0, i, i + 1] for i in range(1, n - 1)]).ravel()
        fan = o.voronoi_pieces(V, off, idx, Q)
        segs = [(V[0], V[i]) for i in range(2, n - 1)] + [(V[i - 1], V[i]) for i in range(n)]
        d = np.full(len(Q), np.inf)
        for a, b in segs:
            e = b - a
            dd = np.abs(e[0] * (Q[:, 1] - a[1]) - e[1] * (Q[:, 0] - a[0])) / np.hypot(*e)
            d = np.minimum(d, dd)
        far = d > 1e-9
        assert np.array_equal(fan[far], one[far])
        assert far.sum() > 19000


def pin_pieces_agree_with_ray_crossing(o):
    """Random star-shaped non-convex polygons (float vertices): away from
    every edge and every diagonal of the decomposition (1e-9), the union of
    the pieces' Voronoi tests equals ray crossing (Algorithm 1, which
    handles simple polygons directly)."""
    rng = _rng(23)
    for t in range(6):
        n = int(rng.integers(8, 40))
        V = polydecomp.star_polygon(rng, n, center=tuple(rng.uniform(-5, 5, 2)))
        if t % 2:
            V = V[::-1].copy()
        off, idx = polydecomp.decompose(V, merged=t % 3 != 2)
        c = V.mean(0)
        Q = c + rng.uniform(-1.2, 1.2, (20000, 2))
        got = o.voronoi_pieces(V, off, idx, Q)
        ray = o.ray_crossing(V, Q)
        d = np.full(len(Q), np.inf)
        for k in range(len(off) - 1):
            pc = idx[off[k]:off[k + 1]]
            for a_, b_ in zip(pc, np.roll(pc, -1)):
                a, b = V[a_], V[b_]
                e = b - a
                t_ = np.clip(((Q - a) @ e) / (e @ e), 0, 1)
                dd = np.hypot(*(Q - (a + t_[:, None] * e)).T)
                d = np.minimum(d, dd)
        far = d > 1e-9
        assert np.array_equal(got[far], ray[far]), int((got[far] != ray[far]).sum())
        assert 0.1 < got.mean() < 0.7


ALL_PINS = [
    pin_pieces_L_shape_exact,
    pin_pieces_exact_rational,
    pin_pieces_single_and_fan,
    pin_pieces_agree_with_ray_crossing,
    pin_square_and_triangle,
    pin_raster_exact,
    pin_raster_area,
    pin_locate_hand_worked,
    pin_locate_partition,
    pin_locate_overlapping,
    pin_locate_far_rounding,
    pin_regular_ngon,
    pin_generators_exact_rational,
    pin_generator_invariants,
    pin_degenerate_status,
    pin_unit_square_grid,
    pin_exact_rational_labels,
    pin_three_tests_agree_away_from_edges,
    pin_label_invariants,
    pin_nonfinite_points,
    pin_max_margin,
    pin_pose_polygon,
    pin_allpairs,
    pin_cost_fixtures,
    pin_cost_rigid_invariance,
    pin_cost_gradient_fd,
    pin_cost_gradient_cw,
    pin_cost_hash,
    pin_cost_argmin,
]
