"""GPU parity of the float32 pre-screen of ray crossing (Section 2.1,
Algorithm 1) at the cases its exactness argument rests on: vertex heights
that are not float32 values (the in-range flag compares Q_y with the height
rounded up to float32), points whose Q_y is that rounded height or one of its
float32 neighbours, points on the edges' lines (the line test's band sends
them to binary64), horizontal edges, non-convex polygons and non-finite
points.  Labels must equal the FP64 oracle's bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

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
    return P


def f32_neighbours(y):
    """float32 values around binary64 y: rounded down, rounded up, and one
    float32 step beyond each."""
    f = np.float32(y)
    lo = f if float(f) <= y else np.nextafter(f, np.float32(-np.inf))
    hi = f if float(f) >= y else np.nextafter(f, np.float32(np.inf))
    return [np.nextafter(lo, np.float32(-np.inf)), lo, hi, np.nextafter(hi, np.float32(np.inf))]


def run(P, oracle, V, Q, tag):
    Vt = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda()
    Qt = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    w = P.pip_ray_crossing(Vt, Qt, status=st)
    torch.cuda.synchronize()
    got = w.cpu().numpy().view(np.uint32)
    want = pack_bits(oracle.ray_crossing(V, Q.astype(np.float64)))
    if not np.array_equal(got, want):
        bad = np.nonzero(unpack_bits(got, len(Q)) != unpack_bits(want, len(Q)))[0]
        raise AssertionError(f"{tag}: {len(bad)} label mismatches, first at {bad[:10]}")
    return int(st.item())


def height_probe_points(rng, V, per_height=64):
    """For every vertex: rows of points at Q_y in the float32 neighbourhood of
    its height, with Q_x spread over the polygon's x range and placed on the
    vertex's x and on the polygon's edges' lines at that height."""
    xs_lo, xs_hi = V[:, 0].min() - 0.1, V[:, 0].max() + 0.1
    pts = []
    for vx, vy in V:
        for fy in f32_neighbours(vy):
            qx = rng.uniform(xs_lo, xs_hi, per_height)
            qx[:4] = [vx, np.float32(vx), np.nextafter(np.float32(vx), np.float32(np.inf)),
                      np.nextafter(np.float32(vx), np.float32(-np.inf))]
            pts.append(np.stack([qx, np.full(per_height, float(fy))], 1))
    # points on the edges' lines, inside and beyond the edges
    Wv = np.roll(V, 1, 0)
    t = rng.uniform(-0.5, 1.5, size=(len(V), 40))
    line = Wv[:, None, :] + t[..., None] * (V - Wv)[:, None, :]
    pts.append(line.reshape(-1, 2))
    return np.concatenate(pts).astype(np.float32)


@pytest.mark.parametrize("seed", range(6))
def test_vertex_heights_between_float32_values(P, oracle, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(3, 40))
    ang = np.sort(rng.uniform(0, 2 * np.pi, n))
    r = 10.0 ** rng.uniform(-3, 3)
    c = rng.uniform(-1e3, 1e3, 2)
    V = np.stack([c[0] + r * np.cos(ang), c[1] + r * np.sin(ang)], 1)
    # heights a third of a float32 step off a float32 value (not representable)
    fy = V[:, 1].astype(np.float32)
    ulp = np.abs(np.nextafter(fy, np.float32(np.inf)) - fy).astype(np.float64)
    V[:, 1] = fy.astype(np.float64) + rng.choice([-1 / 3, 1 / 3, 0.0], n) * ulp
    Q = np.concatenate([height_probe_points(rng, V),
                        rng.uniform(c - 1.5 * r, c + 1.5 * r, size=(20000, 2)).astype(np.float32)])
    say(f"[case] ray filter heights seed={seed} n={n} r={r:.3g} m={len(Q)}")
    assert run(P, oracle, V, Q, f"seed {seed}") == 0


def test_horizontal_edges_and_nonconvex(P, oracle):
    """A non-convex polygon with horizontal edges (never in range) and
    vertices at one height, plus non-finite points."""
    rng = np.random.default_rng(9)
    V = np.array([[0, 0], [4, 0], [4, 1], [3, 1], [3, 3], [2, 3], [2, 1], [1, 1], [1, 3],
                  [0, 3]], float) * 0.1 + 0.05
    Q = np.concatenate([height_probe_points(rng, V, 256),
                        rng.uniform(-0.1, 0.6, size=(50000, 2)).astype(np.float32),
                        np.array([[np.nan, 0.1], [0.1, np.inf], [-np.inf, -np.inf]], np.float32)])
    say(f"[case] ray filter non-convex m={len(Q)}")
    run(P, oracle, V, Q, "non-convex")
