"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Labels must be bit-identical; generators bit-identical; the float32 margin
within its proven band.  Every input is seeded and synthetic.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import pack_bits, unpack_bits
from shapes import placed_convex

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


@pytest.fixture(autouse=True, params=["radial", "mfma", "valu"])
def screen(request, P):
    """Every test runs with each float32 screen forced for all polygon sizes:
    the radial pre-screen (Voronoi only; the other tests take the vector
    screen), the matrix-core screen and the vector screen."""
    old = (P.get_option(P.PIP_OPT_MFMA_MIN_EDGES), P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES))
    P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, 3 if request.param == "mfma" else 0)
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3 if request.param == "radial" else 0)
    yield request.param
    P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, old[0])
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old[1])


TESTS = {
    "voronoi": ("pip_voronoi", "voronoi"),
    "sign_of_offset": ("pip_sign_of_offset", "sign_of_offset"),
    "ray_crossing": ("pip_ray_crossing", "ray_crossing"),
}


def run_gpu(P, fn, V, Q, status=None):
    Vt = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda()
    Qt = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    w = getattr(P, fn)(Vt, Qt, status=st)
    torch.cuda.synchronize()
    out = w.cpu().numpy().view(np.uint32)
    if status is not None:
        status.append(int(st.item()))
    return out


def expect(oracle, test, V, Q):
    return pack_bits(getattr(oracle, test)(V, np.asarray(Q, dtype=np.float64)))


def assert_same(got, want, m, tag):
    if not np.array_equal(got, want):
        g = unpack_bits(got, m)
        w = unpack_bits(want, m)
        bad = np.nonzero(g != w)[0]
        raise AssertionError(f"{tag}: {len(bad)} label mismatches, first at {bad[:10]}")


def near_edge(rng, V, k, offsets):
    """Points at given signed offsets from random edge positions, plus the
    vertices and edge midpoints (float64)."""
    Wv = np.roll(V, 1, 0)
    e = V - Wv
    L = np.hypot(e[:, 0], e[:, 1])
    nrm = np.stack([e[:, 1] / L, -e[:, 0] / L], 1)
    out = [V, 0.5 * (V + Wv)]
    for s in offsets:
        i = rng.integers(len(V), size=k)
        t = rng.random(k)
        out.append(Wv[i] + t[:, None] * e[i] + s * nrm[i])
    return np.concatenate(out)


# ---------------------------------------------------------------------------
def test_generators_bit_exact(P, oracle):
    rng = np.random.default_rng(11)
    polys = [np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float),
             np.array([[0, 0], [3, 0], [0, 3]], float)]
    for n in (3, 4, 5, 8, 13, 16, 31, 32, 33, 63, 64):
        for c in (0.0, 1000.0, -987.25):
            r = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e3))))
            V = W.circle_polygon(n, r, (c, -c / 2), rng)
            polys += [V, V[::-1].copy()]
    for V in polys:
        want, _ = oracle.generators(V)
        Vt = torch.from_numpy(V).cuda()
        got = P.polygon_to_generators(Vt).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (len(V), V[0])


@pytest.mark.parametrize("test", list(TESTS))
@pytest.mark.parametrize("qdt", ["f32", "f64"])
def test_labels_ragged_sizes(P, oracle, test, qdt):
    rng = np.random.default_rng(12)
    fn, otest = TESTS[test]
    for n in (3, 5, 8, 17, 64):
        V = W.circle_polygon(n, 1.0, rng.uniform(-0.1, 0.1, 2), rng)
        for m in (1, 31, 32, 33, 255, 256, 257, 1000, 65537):
            Q = rng.uniform(-1.5, 1.5, size=(m, 2))
            k = m // 10
            if k:
                Q[:k] = near_edge(rng, V, k, [1e-7])[:k]
            Q = Q.astype(np.float32 if qdt == "f32" else np.float64)
            say(f"[case] {test} {qdt} n={n} m={m}")
            got = run_gpu(P, fn, V, Q)
            assert_same(got, expect(oracle, otest, V, Q), m, f"{test} n={n} m={m}")


@pytest.mark.parametrize("test", list(TESTS))
@pytest.mark.parametrize("centre", [0.0, 1000.0, -1e5])
@pytest.mark.parametrize("qdt", ["f32", "f64"])
def test_adversarial_near_edges(P, oracle, test, centre, qdt):
    """Points on edges, on vertices, and at 1 ulp .. 1e-6 from edges, for
    polygons near the origin and far from it."""
    rng = np.random.default_rng(13)
    fn, otest = TESTS[test]
    for n in (3, 4, 8, 32, 64):
        for orient in (1, -1):
            r = 1.0 if centre == 0.0 else 7.5
            V = W.circle_polygon(n, r, (centre, 0.5 * centre), rng)[::orient].copy()
            scale = abs(centre) + r
            offs = [0.0, 1e-12 * scale, -1e-12 * scale, 1e-9, -1e-9, 1e-7, -1e-7, 1e-6, -1e-6,
                    3e-5, -3e-5]
            Q = near_edge(rng, V, 600, offs)
            Q = Q.astype(np.float32 if qdt == "f32" else np.float64)
            say(f"[case] {test} {qdt} centre={centre} n={n} orient={orient}")
            got = run_gpu(P, fn, V, Q)
            assert_same(got, expect(oracle, otest, V, Q), len(Q), f"{test} n={n}")


@pytest.mark.parametrize("test", ["voronoi", "sign_of_offset"])
def test_all_points_undecided(P, oracle, test):
    """Every point within 1e-9 of an edge: the float32 screen decides none of
    them, so the per-wave queue fills and is flushed repeatedly."""
    rng = np.random.default_rng(14)
    fn, otest = TESTS[test]
    V = W.circle_polygon(8, 1.0, (0.01, -0.02), rng)
    Q = near_edge(rng, V, 300_000, [0.0])[:300_000] + rng.uniform(-1e-9, 1e-9, (300_000, 2))
    Q = Q.astype(np.float64)
    say(f"[case] {test} all undecided m={len(Q)}")
    got = run_gpu(P, fn, V, Q)
    assert_same(got, expect(oracle, otest, V, Q), len(Q), test)


@pytest.mark.parametrize("test", ["voronoi", "sign_of_offset"])
def test_all_points_undecided_float32_many_chunks(P, oracle, test):
    """8M float32 points on the edges of an 8-gon (every one inside the
    band): each wave of the float32 screens walks several 512-point chunks
    and flushes its recheck queue on every one, so queue codes of later
    chunks are exercised."""
    rng = np.random.default_rng(18)
    fn, otest = TESTS[test]
    V = W.circle_polygon(8, 1.0, (0.01, -0.02), rng)
    m = 8 << 20
    Q = near_edge(rng, V, m, [0.0])[:m].astype(np.float32)
    say(f"[case] {test} float32 all undecided m={m}")
    got = run_gpu(P, fn, V, Q)
    assert_same(got, expect(oracle, otest, V, Q), m, test)


@pytest.mark.parametrize("test", list(TESTS))
def test_nonfinite_points(P, oracle, test):
    fn, otest = TESTS[test]
    V = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    Q = np.array([[np.nan, 0.5], [0.5, np.inf], [-np.inf, 0.5], [0.5, 0.5], [np.nan, np.nan],
                  [0.25, 0.75], [1e30, 0.5], [3e38, -3e38]] * 40, dtype=np.float32)
    got = run_gpu(P, fn, V, Q)
    assert_same(got, expect(oracle, otest, V, Q), len(Q), test)


def test_status_codes(P, oracle):
    Q = np.zeros((5, 2), np.float32)
    cases = [
        (np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float), 0),
        (np.array([[0, 0], [1, 0], [2, 0]], float), 2),                 # zero area
        (np.array([[0, 0], [1, 0], [1, 0], [0, 1]], float), 2),         # zero-length edge
        (np.array([[0, 0], [2, 0], [1, 0.2], [1, 2]], float), 3),       # non-convex
        (np.array([[0, 0], [np.nan, 0], [1, 1]], float), 1),            # non-finite vertex
    ]
    for V, want in cases:
        st = []
        run_gpu(P, "pip_voronoi", V, Q, status=st)
        assert st == [want], (V, st)
        st = []
        run_gpu(P, "pip_ray_crossing", V, Q, status=st)
        assert st == [0 if want == 3 else want]
    # labels still follow the binary64 algorithm for the degenerate inputs
    for V, _ in cases:
        Qr = np.random.default_rng(3).uniform(-1, 2, (500, 2)).astype(np.float32)
        for test, (fn, otest) in TESTS.items():
            assert_same(run_gpu(P, fn, V, Qr), expect(oracle, otest, V, Qr), 500, test)


def test_empty_input(P):
    V = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    st = []
    got = run_gpu(P, "pip_voronoi", V, np.zeros((0, 2), np.float32), status=st)
    assert st == [0] and got.size <= 1


def test_max_margin_within_band(P, oracle):
    """float32 largest margin vs the binary64 one: the error stays within
    4.05 u (alpha|X| + beta|Y| + gamma) plus the binary64 terms, the bound
    the band is built on (u = 2^-24)."""
    rng = np.random.default_rng(15)
    worst = 0.0
    for n in (3, 8, 64):
        for c in (0.0, 1000.0):
            V = W.circle_polygon(n, 2.0, (c, c), rng)
            Q = (rng.uniform(-3, 3, size=(50_000, 2)) + np.array([c, c])).astype(np.float32)
            Vt = torch.from_numpy(V).cuda()
            mm = P.pip_voronoi_max_margin(Vt, torch.from_numpy(Q).cuda()).cpu().numpy()
            want = oracle.voronoi_max_margin(V, Q.astype(np.float64))
            Pg, _ = oracle.generators(V)
            g0 = Pg[0]
            o = g0.astype(np.float32).astype(np.float64)
            h = Pg[1:] - g0
            A = np.abs(2 * h[:, 0]).max()
            B = np.abs(2 * h[:, 1]).max()
            C = np.abs(((Pg[1:] - o) ** 2).sum(1) - ((g0 - o) ** 2).sum()).max()
            X = np.abs(Q[:, 0].astype(np.float64) - o[0])
            Y = np.abs(Q[:, 1].astype(np.float64) - o[1])
            u = 2.0 ** -24
            bound = 4.05 * u * (A * X + B * Y + C) + 1e-12 * (1 + X * X + Y * Y)
            err = np.abs(mm.astype(np.float64) - want)
            assert np.all(err <= bound), (n, c, float((err / bound).max()))
            worst = max(worst, float((err / (A * X + B * Y + C)).max() / u))
    say(f"[stat] worst float32 margin error = {worst:.3f} u of (alpha|X|+beta|Y|+gamma)")


def test_fp32_plain_mismatches_only_near_edges(P, oracle):
    rng = np.random.default_rng(16)
    V = W.streaming_polygon(16)
    Q = W.streaming_points(V, 1 << 20)
    got = unpack_bits(run_gpu(P, "pip_voronoi_fp32_plain", V, Q), len(Q))
    want = oracle.voronoi(V, Q.astype(np.float64))
    bad = np.nonzero(got != want)[0]
    Wv = np.roll(V, 1, 0)
    e = V - Wv
    L = np.hypot(e[:, 0], e[:, 1])
    Qb = Q[bad].astype(np.float64)
    d = np.abs((e[None, :, 0] * (Qb[:, None, 1] - Wv[None, :, 1]) -
                e[None, :, 1] * (Qb[:, None, 0] - Wv[None, :, 0])) / L[None, :]).min(1)
    say(f"[stat] fp32-plain mismatches: {len(bad)} of {len(Q)}")
    assert np.all(d < 1e-5)


def test_deterministic(P):
    V = W.streaming_polygon(8)
    Q = W.streaming_points(V, 1 << 20)
    a = run_gpu(P, "pip_voronoi", V, Q)
    b = run_gpu(P, "pip_voronoi", V, Q)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# the configurations of the paper-shaped workloads at full size
# ---------------------------------------------------------------------------
def test_single_polygon_fp64_all_three_tests(P, oracle):
    V, Q = W.single_polygon_fp64()
    res = {}
    for test, (fn, otest) in TESTS.items():
        say(f"[case] single polygon fp64 {test}")
        got = run_gpu(P, fn, V, Q)
        assert_same(got, expect(oracle, otest, V, Q), len(Q), test)
        res[test] = unpack_bits(got, len(Q))
    # the paper's correctness experiment: the three tests agree here
    assert np.array_equal(res["voronoi"], res["sign_of_offset"])
    assert np.array_equal(res["voronoi"], res["ray_crossing"])


@pytest.mark.parametrize("n", W.STREAM_NS)
def test_streaming_full_size_sampled(P, oracle, n):
    """2^28 float32 points with 1% within 1e-6 of an edge, the launch that
    the benchmark times; the oracle checks a 3M-point sample plus every
    point whose float32 margin is small."""
    V = W.streaming_polygon(n)
    say(f"[case] streaming n={n}: generating 2^28 points")
    Q = W.streaming_points(V, W.STREAM_M)
    Vt = torch.from_numpy(V).cuda()
    Qt = torch.from_numpy(Q).cuda()
    say(f"[case] streaming n={n}: GPU")
    lab = P.pip_voronoi(Vt, Qt)
    mm = P.pip_voronoi_max_margin(Vt, Qt)
    torch.cuda.synchronize()
    labels = lab.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(100 + n)
    idx = np.unique(np.concatenate([
        rng.integers(0, W.STREAM_M, 3_000_000),
        np.arange(0, 100_000), np.arange(W.STREAM_M - 100_000, W.STREAM_M),
        torch.nonzero(mm.abs() < 1e-5).flatten()[:2_000_000].cpu().numpy()]))
    want = oracle.voronoi(V, Q[idx].astype(np.float64))
    got = ((labels[idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(bool)
    bad = np.nonzero(got != want)[0]
    say(f"[stat] n={n} checked {len(idx)} sampled points, {len(bad)} mismatches, "
        f"inside fraction {got.mean():.4f}")
    assert len(bad) == 0
    assert labels.size == W.STREAM_M // 32


@pytest.mark.parametrize("n", W.STREAM_NS)
def test_reference_tests_full_size_sampled(P, oracle, screen, n):
    """Sign of offset (Algorithm 2) and ray crossing (Algorithm 1) on the
    benchmark's 2^28-point launches: a 3M-point sample, the first and last
    100k points and every point whose Voronoi margin is small (the near-edge
    points) against the oracle.  Sign of offset takes the vector and the
    matrix-core screens (the radial pre-screen is Voronoi's only); ray
    crossing has no float32 screen and runs once."""
    tests = {"valu": ["sign_of_offset", "ray_crossing"], "mfma": ["sign_of_offset"]}.get(screen)
    if not tests:
        pytest.skip("the same launches as the vector-screen run")
    V = W.streaming_polygon(n)
    say(f"[case] reference tests n={n} ({screen}): generating 2^28 points")
    Q = W.streaming_points(V, W.STREAM_M)
    Vt = torch.from_numpy(V).cuda()
    Qt = torch.from_numpy(Q).cuda()
    mm = P.pip_voronoi_max_margin(Vt, Qt)
    rng = np.random.default_rng(200 + n)
    idx = np.unique(np.concatenate([
        rng.integers(0, W.STREAM_M, 3_000_000),
        np.arange(0, 100_000), np.arange(W.STREAM_M - 100_000, W.STREAM_M),
        torch.nonzero(mm.abs() < 1e-5).flatten()[:2_000_000].cpu().numpy()]))
    del mm
    Qs = Q[idx].astype(np.float64)
    for test in tests:
        fn, otest = TESTS[test]
        say(f"[case] {test} n={n} 2^28 points, GPU")
        lab = getattr(P, fn)(Vt, Qt)
        torch.cuda.synchronize()
        labels = lab.cpu().numpy().view(np.uint32)
        assert labels.size == W.STREAM_M // 32
        want = getattr(oracle, otest)(V, Qs)
        got = ((labels[idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(bool)
        bad = np.nonzero(got != want)[0]
        say(f"[stat] {test} n={n}: checked {len(idx)} sampled points, {len(bad)} mismatches")
        assert len(bad) == 0


@pytest.mark.parametrize("qdt", [np.float32, np.float64])
def test_ray_crossing_nonconvex(P, oracle, qdt):
    """Ray crossing (Algorithm 1) handles simple non-convex polygons: a
    10-point star and a U shape, 200k points plus every vertex and edge
    midpoint, bit-identical to the binary64 oracle."""
    rng = np.random.default_rng(44)
    t = np.arange(10) * (2 * np.pi / 10)
    r = np.where(np.arange(10) % 2 == 0, 1.0, 0.38)
    star = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    ushape = np.array([[0, 0], [3, 0], [3, 3], [2, 3], [2, 1], [1, 1], [1, 3], [0, 3]], float)
    for V in (star, ushape):
        lo, hi = V.min(0) - 0.3, V.max(0) + 0.3
        Q = rng.uniform(lo, hi, size=(200_000, 2))
        mids = 0.5 * (V + np.roll(V, 1, axis=0))
        Q = np.concatenate([Q, V, mids]).astype(qdt)
        st = []
        got = run_gpu(P, "pip_ray_crossing", V, Q, status=st)
        assert st == [0]
        want = oracle.ray_crossing(V, Q.astype(np.float64))
        assert_same(got, pack_bits(want), len(Q), "ray_crossing")
        # the inside fraction of the uniform part matches the polygon's area
        x, y = V[:, 0], V[:, 1]
        area = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
        frac = want[:200_000].mean()
        assert abs(frac - area / np.prod(hi - lo)) < 0.01, (frac, area / np.prod(hi - lo))


@pytest.mark.parametrize("test", list(TESTS))
@pytest.mark.parametrize("qdt", ["f32", "f64"])
def test_irregular_polygons(P, oracle, test, qdt):
    """Irregular convex polygons (random edge lengths and turning angles, 3 to
    64 vertices), stretched up to 10^4:1, rotated, at sizes 10^-4..10^4 and
    centres up to 10^5 from the origin, in both orientations: uniform points
    over the bounding box, points at 0..10^-5 of the size from the edges,
    the vertices and their float32 neighbours.  Labels bit-identical to the
    oracle's; valid polygons report status 0."""
    rng = np.random.default_rng(61)
    fn, otest = TESTS[test]
    for n in (3, 4, 5, 7, 12, 20, 33, 48, 64):
        for stretch, size, centre in ((1.0, 1.0, 0.0), (1e2, 1e-3, 1e3), (1e4, 1e4, -1e5),
                                      (30.0, 1e-4, 0.5)):
            V = placed_convex(rng, n, stretch, size, centre)
            lo, hi = V.min(0), V.max(0)
            span = hi - lo
            Q = rng.uniform(lo - 0.25 * span, hi + 0.25 * span, size=(6000, 2))
            scale = float(np.abs(V).max())
            offs = [0.0, 1e-12 * scale, -1e-12 * scale, 1e-9 * size, -1e-9 * size, 1e-7 * size,
                    -1e-7 * size, 1e-5 * size, -1e-5 * size]
            Qe = near_edge(rng, V, 400, offs)
            fv = V.astype(np.float32)
            nb = np.concatenate([np.stack([np.nextafter(fv[:, 0], np.float32(s)), fv[:, 1]], 1)
                                 for s in (-np.inf, np.inf)]).astype(np.float64)
            Q = np.concatenate([Q, Qe, nb]).astype(np.float32 if qdt == "f32" else np.float64)
            say(f"[case] {test} {qdt} irregular n={n} stretch={stretch:g} size={size:g} "
                f"centre={centre:g}")
            st = []
            got = run_gpu(P, fn, V, Q, status=st)
            assert st == [0], (n, stretch, size, centre, st)
            assert_same(got, expect(oracle, otest, V, Q), len(Q),
                        f"{test} n={n} stretch={stretch:g} size={size:g}")


@pytest.mark.parametrize("test", list(TESTS))
def test_ragged_tail_after_many_chunks(P, oracle, test):
    """3 x 5120 x 512 + 333 float32 points (every wave of the persistent
    screens walks three or four full chunks before one wave takes the
    333-point tail), 1% of them within 1e-7 of an edge so that the recheck
    queues hold codes of later chunks; every label checked."""
    rng = np.random.default_rng(77)
    fn, otest = TESTS[test]
    m = 3 * 5120 * 512 + 333
    for n in (8, 33):
        V = W.circle_polygon(n, 1.0, (0.02, -0.01), rng)
        Q = rng.uniform(-1.5, 1.5, size=(m, 2))
        k = m // 100
        sel = rng.choice(m, size=k, replace=False)
        Q[sel] = near_edge(rng, V, k, [1e-7, -1e-7])[2 * len(V):][rng.permutation(2 * k)[:k]]
        Q = Q.astype(np.float32)
        say(f"[case] {test} ragged tail n={n} m={m}")
        got = run_gpu(P, fn, V, Q)
        assert got.size == (m + 31) // 32
        assert_same(got, expect(oracle, otest, V, Q), m, f"{test} n={n} m={m}")
