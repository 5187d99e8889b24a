"""GPU parity of the point-location index against the brute-force FP64
oracle: every id equal (smallest containing polygon index, or -1), for
partitions, overlapping and degenerate polygon sets, several grid shapes and
the full-size partition; the plain and the binned query give the same ids."""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_15385_amd as P
    P.load_library()
    return P


def locate_gpu(P, off, V, Q, cells=0, status=None):
    idx = P.LocateIndex(torch.from_numpy(np.asarray(off, np.int64)).cuda(),
                        torch.from_numpy(np.ascontiguousarray(V, np.float64)).cuda(), cells=cells,
                        status=status)
    Qt = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).cuda()
    ids = idx.locate(Qt, binned=False)
    ids_b = idx.locate(Qt, binned=True)  # points binned by super-cell first
    torch.cuda.synchronize()
    out = ids.cpu().numpy()
    assert np.array_equal(out, ids_b.cpu().numpy()), "binned query differs"
    info = idx.info()
    idx.close()
    return out, info


def check(P, oracle, off, V, Q, cells=0, tag=""):
    Q = np.ascontiguousarray(Q, np.float32)
    say(f"[case] locate {tag} P={len(off) - 1} m={len(Q)} cells={cells}")
    got, info = locate_gpu(P, off, V, Q, cells)
    want = oracle.locate(off, V, Q.astype(np.float64))
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{tag}: {len(bad)} ids differ, first {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"
    return want, info


def partition_points(rng, part, m):
    """Uniform points, every grid vertex, edge midpoints and points within
    1e-12 .. 1e-6 of cell edges."""
    off, V = part.vtx_off, part.V
    pts = [W.locate_points(part, m, seed_salt=int(rng.integers(1 << 30))).astype(np.float64), V]
    for k in range(0, len(off) - 1, 3):
        Pk = V[off[k]:off[k + 1]]
        e = np.roll(Pk, -1, 0) - Pk
        L = np.hypot(e[:, 0], e[:, 1])[:, None]
        nrm = np.stack([e[:, 1], -e[:, 0]], 1) / L
        t = rng.random((len(Pk), 1))
        for s in (0.0, 1e-12, -1e-9, 1e-7, -1e-6):
            pts.append(Pk + t * e + s * nrm)
        pts.append(Pk + 0.5 * e)
    return np.concatenate(pts)


def test_locate_hand_worked(P, oracle):
    with open(os.path.join(GOLDEN, "locate_2x2.json")) as f:
        g = json.load(f)
    polys = [np.array(p, dtype=float) for p in g["polygons"]]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])])
    Q = np.array(g["points"] + [[np.nan, 1.0], [1.0, np.inf], [-np.inf, 0.5]])
    got, _ = locate_gpu(P, off, np.concatenate(polys), Q)
    assert got.tolist() == g["ids"] + [-1, -1, -1]


@pytest.mark.parametrize("gx,gy,split", [(12, 9, 0.0), (40, 30, 0.5), (7, 61, 1.0)])
def test_locate_partition(P, oracle, gx, gy, split):
    rng = np.random.default_rng(gx * gy)
    part = W.jittered_partition(gx, gy, cell=0.5, split=split, origin=(-3.0, 2.0),
                                seed_salt=gx)
    Q = partition_points(rng, part, 60_000)
    want, info = check(P, oracle, part.vtx_off, part.V, Q, tag=f"partition {gx}x{gy}")
    say(f"[stat] cells {info[0]}, entries {info[1]}, located {int((want >= 0).sum())} of {len(Q)}")


@pytest.mark.parametrize("cells", [1, 7, 1000, 65536])
def test_locate_grid_shapes_agree(P, oracle, cells):
    """The grid only prunes candidates: any cell count gives the same ids."""
    rng = np.random.default_rng(5)
    part = W.jittered_partition(20, 16, cell=1.0, split=0.5, seed_salt=9)
    Q = partition_points(rng, part, 20_000)
    check(P, oracle, part.vtx_off, part.V, Q, cells=cells, tag="grid shapes")


def test_locate_overlapping_and_unusual(P, oracle):
    """Overlapping random polygons (smallest index wins), nested squares, a
    non-convex and a degenerate polygon and one with a non-finite vertex
    (kept in the global list), a 2-vertex polygon (contains nothing)."""
    rng = np.random.default_rng(17)
    polys = [W.circle_polygon(int(rng.integers(3, 20)), float(rng.uniform(0.5, 4.0)),
                              rng.uniform(-6, 6, 2), rng) for _ in range(60)]
    polys += [np.array([[-1.0, -1], [1, -1], [1, 1], [-1, 1]]) * s for s in (3.0, 2.0, 1.0)]
    polys.append(np.array([[0.0, 0], [4, 0], [2, 0.5], [2, 4]]))       # non-convex
    polys.append(np.array([[0.0, 0], [1, 1], [2, 2]]))                 # zero area
    polys.append(np.array([[0.0, 0], [np.inf, 0], [1, 1]]))            # non-finite
    polys.append(np.array([[5.0, 5], [6, 6]]))                         # 2 vertices
    polys.append(np.array([[0.0, 0], [1, 0], [1, 0], [0, 1]]))         # zero-length edge
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])])
    V = np.concatenate(polys)
    Q = np.concatenate([rng.uniform(-10, 10, (40_000, 2)),
                        np.concatenate([p for p in polys if np.isfinite(p).all()]),
                        [[np.nan, 0.0], [0.0, -np.inf]]])
    st = torch.full((len(polys),), -7, dtype=torch.int32, device="cuda")
    got, _ = locate_gpu(P, off, V, Q.astype(np.float32), status=st)
    want = oracle.locate(off, V, Q.astype(np.float32).astype(np.float64))
    assert np.array_equal(got, want)
    s = st.cpu().numpy()
    assert s[:-5].tolist() == [0] * (len(polys) - 5)
    assert s[-5:].tolist() == [3, 2, 1, 1, 2]  # non-convex, zero area, non-finite, 2 vertices, zero edge


def test_locate_long_cell_lists(P, oracle):
    """Concentric squares: 40 about one centre (cell lists of up to 40
    entries, kept in ascending index, several 8-entry batches per cell) and
    100 about another (lists longer than the 64 entries that are sorted, so
    they keep the fill order); listed smallest first (the answer is the
    smallest square containing the point) and then shuffled."""
    rng = np.random.default_rng(23)
    sq = np.array([[-1.0, -1], [1, -1], [1, 1], [-1, 1]])
    polys = []
    for cx, cnt in ((-5.0, 40), (5.0, 100)):
        polys += [sq * s + [cx, 0.25] for s in np.linspace(0.1, 4.0, cnt)]
    for name, perm in (("smallest first", np.arange(len(polys))),
                       ("shuffled", rng.permutation(len(polys)))):
        ps = [polys[i] for i in perm]
        off = np.concatenate([[0], np.cumsum([len(p) for p in ps])])
        V = np.concatenate(ps)
        Q = np.concatenate([rng.uniform(-10, 10, (30_000, 2)), V])
        check(P, oracle, off, V, Q, tag=f"long lists, {name}")


@pytest.mark.parametrize("origin", [(1000.0, -500.0), (1.0e5, 1.0e5)])
def test_locate_far_from_origin(P, oracle, origin):
    rng = np.random.default_rng(3)
    part = W.jittered_partition(25, 20, cell=2.0, split=0.5, origin=origin, seed_salt=4)
    Q = partition_points(rng, part, 30_000)
    check(P, oracle, part.vtx_off, part.V, Q, tag=f"far {origin}")


def _float32_rows_through_vertices(V, rng, xs=5, ys=1):
    """Points on the float32 rows through each vertex: y the float32 values
    nearest to the vertex's y (and ys neighbours each way), x the float32
    values nearest to its x (and xs neighbours each way)."""
    out = []
    for vx, vy in V:
        x32 = np.float32(vx)
        y32 = np.float32(vy)
        xv = [x32]
        for _ in range(xs):
            xv.append(np.nextafter(xv[-1], np.float32(np.inf)))
        x = x32
        for _ in range(xs):
            x = np.nextafter(x, np.float32(-np.inf))
            xv.append(x)
        yv = [y32]
        for _ in range(ys):
            yv.append(np.nextafter(yv[-1], np.float32(np.inf)))
        y = y32
        for _ in range(ys):
            y = np.nextafter(y, np.float32(-np.inf))
            yv.append(y)
        for a in xv:
            for b in yv:
                out.append((a, b))
    return np.array(out, dtype=np.float32)


def test_locate_partition_across_axis_far_in_y(P, oracle):
    """A jittered partition at (-25, 1e5) that crosses x = 0: small x
    coordinates and large y coordinates, where the rounding of the stored
    generators (scaled by the largest coordinate) exceeds the evaluation
    error scaled by x; points on the float32 rows through every vertex."""
    rng = np.random.default_rng(31)
    part = W.jittered_partition(25, 20, cell=2.0, split=0.5, origin=(-25.0, 1.0e5), seed_salt=6)
    Q = np.concatenate([partition_points(rng, part, 20_000).astype(np.float32),
                        _float32_rows_through_vertices(part.V, rng)])
    check(P, oracle, part.vtx_off, part.V, Q, tag="across x=0 at y=1e5")


def test_locate_thin_polygons_at_large_y(P, oracle):
    """Small polygons with x in 1e-9..1e-3 and y in 1e5..1e7 (x-extent far
    below the float32 spacing of y): points on the float32 rows through
    their vertices, each polygon indexed on its own and all together."""
    rng = np.random.default_rng(37)
    polys = []
    for _ in range(300):
        cx = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-9, -3)
        cy = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(5, 7)
        r = 10 ** rng.uniform(-9, -3)
        polys.append(W.circle_polygon(int(rng.integers(3, 12)), r, (cx, cy), rng))
    Q = np.concatenate([_float32_rows_through_vertices(p, rng, xs=8, ys=1) for p in polys])
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])])
    check(P, oracle, off, np.concatenate(polys), Q, tag="thin at large y, together")
    for k in range(0, 300, 30):
        q = _float32_rows_through_vertices(polys[k], rng, xs=12, ys=2)
        check(P, oracle, [0, len(polys[k])], polys[k], q, tag=f"thin at large y, polygon {k}")


def test_locate_points_beyond_the_near_region(P, oracle):
    """Points so far from every polygon that Algorithm 5's binary64 squared
    distances round to equal values (the oracle then calls them inside):
    they take the every-polygon path and get the oracle's ids; far points
    where rounding still decides outside get -1."""
    rng = np.random.default_rng(41)
    part = W.jittered_partition(12, 10, cell=1.0, split=0.5, origin=(-6.0, -5.0), seed_salt=2)
    far = np.array([[1e30, 1e30], [-1e25, 3e38], [2.0 ** 80, -2.0 ** 80], [1e15, 0.0],
                    [-3e38, -3e38], [1e7, 1e7], [0.0, 1e20], [5e18, -7e17]], dtype=np.float32)
    Q = np.concatenate([partition_points(rng, part, 5_000).astype(np.float32), far,
                        (rng.standard_normal((4000, 2)) * 10 ** rng.uniform(0, 38, (4000, 1)))
                        .astype(np.float32)])
    Q = Q[np.isfinite(Q).all(axis=1)]
    want, _ = check(P, oracle, part.vtx_off, part.V, Q, tag="beyond the near region")
    say(f"[stat] far points located by rounding: {int((want[-4000:] >= 0).sum())}")


def test_locate_empty_and_errors(P):
    V = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    got, _ = locate_gpu(P, [0, 4], V, np.zeros((0, 2)))
    assert got.size == 0
    got, _ = locate_gpu(P, [0], np.zeros((0, 2)), np.array([[0.5, 0.5]]))
    assert got.tolist() == [-1]
    big = W.circle_polygon(65, 1.0, (0, 0), np.random.default_rng(0))
    with pytest.raises(P.PipError):
        locate_gpu(P, [0, 65], big, np.zeros((1, 2)))
    with pytest.raises(P.PipError):  # vtx_off[P] != number of vertices
        P.LocateIndex(torch.tensor([0, 3], dtype=torch.int64).cuda(), torch.from_numpy(V).cuda())
    # the binned query indexes its copy of the points with 32-bit offsets: a
    # count of 2^31 is refused before anything is read or launched
    from paper_2007_15385_amd.api import _lib as _raw
    idx = P.LocateIndex(torch.tensor([0, 4], dtype=torch.int64).cuda(), torch.from_numpy(V).cuda())
    q = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    ids = torch.empty(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    s = _raw().pip_index_locate_binned(idx.handle, q.data_ptr(), 1 << 31, ids.data_ptr(),
                                       ws.data_ptr(), ws.numel(), None)
    assert s == 6  # PIP_EUNSUPPORTED
    idx.close()


def test_locate_full_size(P, oracle):
    """The 256 x 256 jittered partition (about 98k convex cells) against
    2^24 uniform points: every id checked on 20,000 sampled points against
    the brute-force oracle; at every point, points inside the cells' common
    interior are located and points outside every box get -1."""
    part = W.jittered_partition(256, 256, cell=1.0, split=0.5)
    Q = W.locate_points(part, 1 << 24)
    say(f"[case] locate full size: P={len(part.vtx_off) - 1}, GPU")
    got, info = locate_gpu(P, part.vtx_off, part.V, Q)
    rng = np.random.default_rng(8)
    sel = np.sort(rng.choice(len(Q), 20_000, replace=False))
    say("[case] locate full size: oracle sample")
    want = oracle.locate(part.vtx_off, part.V, Q[sel].astype(np.float64))
    assert np.array_equal(got[sel], want)
    inner = (Q[:, 0] > 0.25) & (Q[:, 0] < 255.75) & (Q[:, 1] > 0.25) & (Q[:, 1] < 255.75)
    assert (got[inner] >= 0).all()
    outer = (Q[:, 0] < -0.25) | (Q[:, 0] > 256.25) | (Q[:, 1] < -0.25) | (Q[:, 1] > 256.25)
    assert (got[outer] == -1).all()
    say(f"[stat] locate: cells {info[0]}, entries {info[1]}, located {int((got >= 0).sum())}")
