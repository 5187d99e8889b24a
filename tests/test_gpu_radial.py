"""GPU tests of the radial pre-screen of pip_voronoi.

The thresholds (pip_voronoi_radial_bounds) are checked against the FP64
oracle directly: float32 points placed just inside T_in and just beyond
T_out in every octant (dense in angle, octant boundaries included) must get
the oracle's inside and outside labels respectively, and for regular
polygons the thresholds must be tight (T_in near the apothem squared in
every octant, T_out near the circumradius squared).  The labels of the radial
kernel are compared with the oracle bit for bit on adversarial point sets:
rings at the thresholds, octant boundaries, near-edge points, huge and
non-finite coordinates, queues that fill on every chunk, ragged sizes.
"""
from __future__ import annotations

import math
import sys
import zlib

import numpy as np
import pytest

import workloads as W
from oracle import pack_bits, unpack_bits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_15385_amd as P
    P.load_library()
    old = P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES)
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3)  # every polygon takes the radial kernel
    yield P
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old)


def regular(n, R=1.0, c=(0.0, 0.0), phase=0.0, cw=False):
    th = phase + 2 * math.pi * np.arange(n) / n
    V = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th)], 1)
    return V[::-1].copy() if cw else V


def polygons():
    """(name, V, convex): the shapes the bounds are checked on."""
    rng = np.random.default_rng(20071538)
    out = []
    for n in (3, 4, 5, 8, 12, 16, 33, 64):
        out.append((f"regular{n}", regular(n, phase=0.3 * n), True))
    out.append(("regular8_axis", regular(8), True))            # normals on octant boundaries
    out.append(("regular4_diag", regular(4, phase=math.pi / 4), True))
    out.append(("regular16_cw", regular(16, phase=0.1, cw=True), True))
    for n in (12, 16, 32, 64):
        out.append((f"stream{n}", W.streaming_polygon(n), True))
    for n in (6, 20, 48):
        V = W.circle_polygon(n, 1.0, (0.0, 0.0), rng)
        V[:, 0] *= 1000.0                                         # 1000:1 aspect
        out.append((f"long{n}", V, True))
    V = W.circle_polygon(24, 3.0, (1.0e4, -2.0e4), rng)
    out.append(("far1e4", V, True))
    V = W.circle_polygon(10, 0.5, (3.0e6, 1.0e6), rng)
    out.append(("far3e6", V, True))
    # nearly collinear vertices: gaps of 1e-7 rad between some angles
    th = np.sort(np.concatenate([rng.uniform(0, 2 * math.pi, 9), [1.0, 1.0 + 1e-7, 1.0 + 2e-7]]))
    out.append(("collinear", np.stack([np.cos(th), np.sin(th)], 1), True))
    out.append(("nonconvex", np.array([[0.0, 0], [2, 0], [1, 0.3], [1, 2], [0.2, 1.5]]), False))
    return out


POLYS = polygons()
# Polygons whose screen may be switched off: float32 normals of nearly
# collinear edges can turn back by ~1e-7 rad; at 3e6 from the origin the
# binary64 centroid of Algorithm 3 loses most digits (p_0 falls outside the
# polygon, so the normals seen from it do not wind once around p_0).
MAY_BE_OFF = {"collinear", "far3e6"}


def bounds(P, V):
    t = P.pip_voronoi_radial_bounds(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    torch.cuda.synchronize()
    b = t.cpu().numpy()
    return b[:8], b[8:16], float(b[16])


def octant(X, Y):
    sx = (X.view(np.uint32) >> 31).astype(np.int64)
    sy = (Y.view(np.uint32) >> 31).astype(np.int64)
    return 4 * sx + 2 * sy + (np.abs(Y) > np.abs(X)).astype(np.int64)


OCT_START = {0: 0.0, 1: 45.0, 2: -45.0, 3: -90.0, 4: 135.0, 5: 90.0, 6: 180.0, 7: 225.0}


def ring_points(ox, oy, r, o, k=4001):
    """float32 points at radius r (float64 construction) from the local origin
    over octant o's closed arc, plus the arc's end directions exactly."""
    th = np.deg2rad(OCT_START[o] + np.linspace(0.0, 45.0, k))
    px = (np.float64(ox) + r * np.cos(th)).astype(np.float32)
    py = (np.float64(oy) + r * np.sin(th)).astype(np.float32)
    return np.stack([px, py], 1)


def local(Q, ox, oy):
    X = (Q[:, 0] - np.float32(ox)).astype(np.float32)
    Y = (Q[:, 1] - np.float32(oy)).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("name,V,convex", POLYS, ids=[p[0] for p in POLYS])
def test_bounds_sound_against_oracle(P, oracle, name, V, convex):
    tin, tout, tfar = bounds(P, V)
    p0 = oracle.centroid(V)[0]
    ox, oy = np.float32(p0[0]), np.float32(p0[1])
    say(f"[case] radial bounds {name}: T_in {tin.min():.6g}..{tin.max():.6g}, "
        f"T_out {tout.min():.6g}..{tout.max():.6g}, T_far {tfar:.3g}")
    if not convex:
        assert (tin == 0).all() and np.isinf(tout).all()
        return
    if name in MAY_BE_OFF and (tin == 0).all() and np.isinf(tout).all():
        return  # screen off for this polygon: every point takes the per-edge screen
    assert (tin > 0).all() and np.isfinite(tout).all() and (tout < tfar).all()
    pts_in, pts_out = [], []
    for o in range(8):
        for f in (1.0, 1 - 1e-7, 1 - 1e-6, 1 - 1e-4):
            Q = ring_points(ox, oy, math.sqrt(tin[o]) * f, o)
            X, Y = local(Q, ox, oy)
            r2 = X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2
            keep = (octant(X, Y) == o) & (r2 * (1 + 2.0 ** -22) < tin[o])
            pts_in.append(Q[keep])
        for f in (1.0, 1 + 1e-7, 1 + 1e-6, 1 + 1e-4, 1.5, 1e3):
            Q = ring_points(ox, oy, math.sqrt(tout[o]) * f, o)
            X, Y = local(Q, ox, oy)
            r2 = X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2
            keep = (octant(X, Y) == o) & (r2 > tout[o] * (1 + 2.0 ** -22)) & \
                   (r2 * (1 + 2.0 ** -22) < tfar)
            pts_out.append(Q[keep])
    Qi = np.concatenate(pts_in)
    Qo = np.concatenate(pts_out)
    say(f"[stat] {len(Qi)} points under T_in, {len(Qo)} beyond T_out")
    assert len(Qi) > 0 and len(Qo) > 0
    li = oracle.voronoi(V, Qi.astype(np.float64))
    lo = oracle.voronoi(V, Qo.astype(np.float64))
    assert li.all(), f"{name}: {int((~li).sum())} points under T_in are outside"
    assert not lo.any(), f"{name}: {int(lo.sum())} points beyond T_out are inside"


@pytest.mark.parametrize("n", [3, 4, 8, 12, 16, 33, 64])
def test_bounds_tight_for_regular_polygons(P, oracle, n):
    """Centred at the origin: T_in >= apothem^2 (1 - 1e-5) in every octant
    (the inner radius is the nearest edge line, further where no normal
    points into the octant) and T_out within 1e-5 of the circumradius^2
    in octants that hold a vertex direction's arc."""
    V = regular(n, phase=0.3 * n)
    tin, tout, tfar = bounds(P, V)
    apothem = math.cos(math.pi / n)
    assert (tin >= apothem ** 2 * (1 - 1e-5)).all(), (tin, apothem ** 2)
    assert (tout <= 1.0 * (1 + 1e-5)).all() and (tout >= apothem ** 2).all(), tout
    assert tfar > 1e20


def labels_gpu(P, V, Q):
    Vt = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda()
    Qt = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    w = P.pip_voronoi(Vt, Qt, status=st)
    torch.cuda.synchronize()
    return w.cpu().numpy().view(np.uint32), int(st.item())


def adversarial_points(oracle, V, rng, m_uniform=20000):
    p0 = oracle.centroid(V)[0]
    ox, oy = np.float32(p0[0]), np.float32(p0[1])
    span = float(np.abs(V - p0).max())
    parts = [(p0 + rng.uniform(-1.6 * span, 1.6 * span, (m_uniform, 2))).astype(np.float32)]
    parts.append(W.near_edge_points(rng, V, 4000, 1e-6 * span).astype(np.float32))
    parts.append(V.astype(np.float32))
    # axis and diagonal directions from the local origin (octant boundaries)
    r = np.linspace(0.0, 1.6 * span, 700)
    for dx, dy in ((1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)):
        parts.append(np.stack([(ox + dx * r).astype(np.float32), (oy + dy * r).astype(np.float32)], 1))
    parts.append(np.array([[ox, oy], [-0.0, oy], [ox, -0.0], [-0.0, -0.0], [0.0, 0.0]], np.float32))
    # huge and non-finite coordinates
    big = np.array([1e10, -1e16, 1e19, 2e19, 1e30, 3.4e38], np.float32)
    parts.append(np.stack([big, np.full_like(big, oy)], 1))
    parts.append(np.stack([np.full_like(big, ox), -big], 1))
    parts.append(np.array([[np.nan, oy], [ox, np.inf], [-np.inf, -np.inf], [np.nan, np.nan]], np.float32))
    return np.concatenate(parts), (ox, oy)


@pytest.mark.parametrize("name,V,convex", POLYS, ids=[p[0] for p in POLYS])
def test_labels_adversarial(P, oracle, name, V, convex):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    Q, (ox, oy) = adversarial_points(oracle, V, rng)
    tin, tout, tfar = bounds(P, V)
    # rings at every octant's thresholds
    rings = []
    for o in range(8):
        for t in (tin[o], tout[o]):
            if 0 < t < np.inf:
                for f in (1 - 1e-6, 1 - 1e-7, 1.0, 1 + 1e-7, 1 + 1e-6):
                    rings.append(ring_points(ox, oy, math.sqrt(t) * f, o, k=301))
    if rings:
        Q = np.concatenate([Q] + rings)
    Q = Q[rng.permutation(len(Q))]
    say(f"[case] radial labels {name}: m={len(Q)}")
    got, st = labels_gpu(P, V, Q)
    want = pack_bits(oracle.voronoi(V, Q.astype(np.float64)))
    if not np.array_equal(got, want):
        bad = np.nonzero(unpack_bits(got, len(Q)) != unpack_bits(want, len(Q)))[0]
        raise AssertionError(f"{name}: {len(bad)} mismatches, first {Q[bad[:5]]}")
    assert (st == 0) == convex


@pytest.mark.parametrize("m", [1, 63, 511, 512, 513, 4097, 100003])
def test_labels_ragged_sizes(P, oracle, m):
    V = W.streaming_polygon(32)
    Q = W.streaming_points(V, m, seed_salt=m)
    got, _ = labels_gpu(P, V, Q)
    assert np.array_equal(got, pack_bits(oracle.voronoi(V, Q.astype(np.float64))))


def test_queue_full_every_chunk(P, oracle):
    """Every point in the annulus (on the boundary +- 1e-3), then stretches
    with none, then single annulus points: the queue fills on every chunk,
    flushes mid-stream and at the end."""
    rng = np.random.default_rng(11)
    V = W.streaming_polygon(64)
    ring = W.near_edge_points(rng, V, 300_000, 1e-3).astype(np.float32)
    p0 = oracle.centroid(V)[0]
    inner = (p0 + rng.uniform(-0.05, 0.05, (200_000, 2))).astype(np.float32)
    sparse = inner[:100_000].copy()
    sparse[::997] = ring[:len(sparse[::997])]
    Q = np.concatenate([ring, inner, sparse, ring[:1000]])
    got, _ = labels_gpu(P, V, Q)
    want = pack_bits(oracle.voronoi(V, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_same_labels_as_other_screens(P):
    """Word for word against the vector and matrix-core screens on the
    streaming workload shape (2^22 points, every polygon size)."""
    for n in W.STREAM_NS:
        V = W.streaming_polygon(n)
        Q = W.streaming_points(V, 1 << 22)
        Vt = torch.from_numpy(V).cuda()
        Qt = torch.from_numpy(Q).cuda()
        a = P.pip_voronoi(Vt, Qt).clone()
        old = P.get_option(P.PIP_OPT_MFMA_MIN_EDGES)
        try:
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 0)
            for mf in (0, 3):
                P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, mf)
                b = P.pip_voronoi(Vt, Qt)
                torch.cuda.synchronize()
                assert torch.equal(a, b), (n, mf)
        finally:
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3)
            P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, old)


def test_option_range(P):
    with pytest.raises(P.PipError):
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, -1)
    with pytest.raises(P.PipError):
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 66)
    assert P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES) == 3


def random_polygons(count, seed):
    """Convex polygons with random vertex counts, aspect ratios up to 300:1,
    rotations and centres up to 1e4 from the origin."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(3, 65))
        V = W.circle_polygon(n, 1.0, (0.0, 0.0), rng)
        V[:, 0] *= float(np.exp(rng.uniform(0.0, np.log(300.0))))
        a = rng.uniform(0.0, 2.0 * math.pi)
        R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
        V = V @ R.T * float(np.exp(rng.uniform(np.log(1e-2), np.log(1e2))))
        V += rng.uniform(-1e4, 1e4, 2) * (rng.random() < 0.5)
        out.append(V)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bounds_sound_random_polygons(P, oracle, seed):
    """60 random convex polygons: every point just under an octant's T_in is
    inside and every point just beyond its T_out (short of T_far) outside."""
    checked = 0
    for V in random_polygons(20, seed):
        tin, tout, tfar = bounds(P, V)
        if (tin == 0).all():
            continue  # screen off for this polygon (allowed; labels still exact)
        p0 = oracle.centroid(V)[0]
        ox, oy = np.float32(p0[0]), np.float32(p0[1])
        pin, pout = [], []
        for o in range(8):
            for f in (1.0, 1 - 1e-6, 1 - 1e-3):
                Q = ring_points(ox, oy, math.sqrt(tin[o]) * f, o, k=1001)
                X, Y = local(Q, ox, oy)
                r2 = X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2
                pin.append(Q[(octant(X, Y) == o) & (r2 * (1 + 2.0 ** -22) < tin[o])])
            if np.isfinite(tout[o]):
                for f in (1.0, 1 + 1e-6, 1 + 1e-3, 2.0):
                    Q = ring_points(ox, oy, math.sqrt(tout[o]) * f, o, k=1001)
                    X, Y = local(Q, ox, oy)
                    r2 = X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2
                    pout.append(Q[(octant(X, Y) == o) & (r2 > tout[o] * (1 + 2.0 ** -22)) &
                                  (r2 * (1 + 2.0 ** -22) < tfar)])
        Qi, Qo = np.concatenate(pin), np.concatenate(pout)
        assert oracle.voronoi(V, Qi.astype(np.float64)).all(), "a point under T_in is outside"
        assert not oracle.voronoi(V, Qo.astype(np.float64)).any(), "a point beyond T_out is inside"
        checked += 1
    say(f"[stat] seed {seed}: {checked} of 20 polygons with the screen on")
    assert checked >= 8
