"""GPU parity of the non-convex (union of convex pieces) test against the
FP64 oracle: bit-identical labels for every point, float32 and binary64
points, decompositions from the library and from an exact test-side
routine, invalid pieces, ragged and empty inputs, errors, and a 2^26-point
launch checked on a sample and on every near-boundary point."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import polydecomp
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
    return P


def run(P, V, off, idx, Q):
    d = "cuda"
    lab, st = P.pip_voronoi_pieces(torch.from_numpy(np.ascontiguousarray(V)).to(d),
                                   torch.from_numpy(np.asarray(off, np.int32)).to(d),
                                   torch.from_numpy(np.asarray(idx, np.int32)).to(d),
                                   torch.from_numpy(np.ascontiguousarray(Q)).to(d))
    torch.cuda.synchronize()
    return lab.cpu().numpy().view(np.uint32)[: (len(Q) + 31) // 32], st.cpu().numpy()


def boundary_points(rng, V, off, idx, k, scale):
    """Points on, and within +-1e-7 scale of, the polygon's edges and the
    pieces' diagonals, plus the vertices."""
    segs = []
    for p in range(len(off) - 1):
        pc = idx[off[p]:off[p + 1]]
        segs += [(V[a], V[b]) for a, b in zip(pc, np.roll(pc, -1))]
    segs = np.array(segs)
    i = rng.integers(len(segs), size=k)
    t = rng.random(k)
    a, b = segs[i, 0], segs[i, 1]
    e = b - a
    L = np.hypot(e[:, 0], e[:, 1])[:, None]
    nrm = np.stack([-e[:, 1], e[:, 0]], 1) / L
    off_ = rng.choice([0.0, 1e-9, -1e-9, 1e-7, -1e-7], size=(k, 1)) * scale
    q = a + t[:, None] * e + off_ * nrm
    return np.concatenate([q, V])


def star_case(seed, n, center=(0.0, 0.0), scale=1.0):
    rng = np.random.default_rng(seed)
    V = polydecomp.star_polygon(rng, n, center=center) if scale == 1.0 else \
        (polydecomp.star_polygon(rng, n) * scale + np.asarray(center))
    return rng, V


@pytest.mark.parametrize("n", [5, 12, 40, 64, 200])
@pytest.mark.parametrize("qdt", ["f32", "f64"])
def test_pieces_star_polygons(P, oracle, n, qdt):
    rng, V = star_case(1000 + n, n, center=(0.3, -0.2))
    off, idx = P.convex_decompose(V, 64)
    say(f"[case] pieces: n={n} K={len(off) - 1} {qdt}")
    Q = np.concatenate([rng.uniform(-1.3, 1.3, (150_000, 2)) + (0.3, -0.2),
                        boundary_points(rng, V, off, idx, 20_000, 1.0)])
    Q = Q.astype(np.float32 if qdt == "f32" else np.float64)
    got, st = run(P, V, off, idx, Q)
    want = pack_bits(oracle.voronoi_pieces(V, off, idx, Q.astype(np.float64)))
    assert np.array_equal(got, want), int((unpack_bits(got, len(Q)) != unpack_bits(want, len(Q))).sum())
    assert (st == 0).all()


@pytest.mark.parametrize("merged", [False, True])
def test_pieces_exact_decomposition_far(P, oracle, merged):
    """Decomposition by the exact test-side routine (triangles, or merged);
    polygon far from the origin (centre 1e4) and large (scale 50)."""
    rng, V = star_case(77 + merged, 30, center=(1.0e4, -2.0e4), scale=50.0)
    off, idx = polydecomp.decompose(V, merged=merged)
    Q = np.concatenate([rng.uniform(-60, 60, (100_000, 2)) + (1.0e4, -2.0e4),
                        boundary_points(rng, V, off, idx, 20_000, 50.0)]).astype(np.float32)
    got, st = run(P, V, off, idx, Q)
    want = pack_bits(oracle.voronoi_pieces(V, off, idx, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_pieces_l_shape_exact(P, oracle):
    V = np.array([[0, 0], [4, 0], [4, 2], [2, 2], [2, 4], [0, 4], [0, 2]], dtype=np.float64)
    off = np.array([0, 5, 9])
    idx = np.array([0, 1, 2, 3, 6, 6, 3, 4, 5])
    g = np.arange(-4, 21) / 4.0
    X, Y = np.meshgrid(g, g)
    Q = np.stack([X.ravel(), Y.ravel()], 1).astype(np.float32)
    got, _ = run(P, V, off, idx, Q)
    x, y = Q[:, 0], Q[:, 1]
    want = ((x >= 0) & (x <= 4) & (y >= 0) & (y <= 2)) | ((x >= 0) & (x <= 2) & (y >= 0) & (y <= 4))
    assert np.array_equal(got, pack_bits(want))


@pytest.mark.parametrize("m", [0, 1, 31, 511, 512, 513, 4097, 65537])
def test_pieces_ragged(P, oracle, m):
    rng, V = star_case(5, 20)
    off, idx = P.convex_decompose(V, 64)
    Q = rng.uniform(-1.2, 1.2, (m, 2)).astype(np.float32)
    got, _ = run(P, V, off, idx, Q)
    want = pack_bits(oracle.voronoi_pieces(V, off, idx, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_pieces_all_undecided_queue(P, oracle):
    """Every point within the band of some piece (on edges and diagonals):
    the recheck queue fills on every chunk."""
    rng, V = star_case(9, 24)
    off, idx = P.convex_decompose(V, 8)
    Q = boundary_points(rng, V, off, idx, 300_000, 1.0).astype(np.float32)
    got, _ = run(P, V, off, idx, Q)
    want = pack_bits(oracle.voronoi_pieces(V, off, idx, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_pieces_invalid_pieces(P, oracle):
    """A two-vertex piece and a piece with an index out of range get
    PIP_EINVAL and contain no point; the other pieces are unaffected."""
    rng, V = star_case(11, 16)
    off, idx = P.convex_decompose(V, 64)
    pieces = [list(idx[off[k]:off[k + 1]]) for k in range(len(off) - 1)]
    bad = pieces[:1] + [[0, 1]] + pieces[1:] + [[0, 1, 999]]
    off2, idx2 = polydecomp.to_csr(bad)
    Q = rng.uniform(-1.2, 1.2, (50_000, 2)).astype(np.float32)
    got, st = run(P, V, off2, idx2, Q)
    assert st[1] == 1 and st[-1] == 1 and (np.delete(st, [1, len(st) - 1]) == 0).all()
    keep = pieces  # the oracle without the unusable pieces
    o3, i3 = polydecomp.to_csr(keep)
    want = pack_bits(oracle.voronoi_pieces(V, o3, i3, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_pieces_nonfinite_points(P, oracle):
    rng, V = star_case(12, 10)
    off, idx = P.convex_decompose(V, 64)
    Q = rng.uniform(-1, 1, (1000, 2)).astype(np.float32)
    Q[::7, 0] = np.nan
    Q[3::11, 1] = np.inf
    Q[5::13] = -np.inf
    got, _ = run(P, V, off, idx, Q)
    want = pack_bits(oracle.voronoi_pieces(V, off, idx, Q.astype(np.float64)))
    assert np.array_equal(got, want)


def test_pieces_errors(P):
    rng, V = star_case(13, 10)
    off, idx = P.convex_decompose(V, 64)
    d = "cuda"
    Vt = torch.from_numpy(V).to(d)
    Q = torch.zeros((10, 2), dtype=torch.float32, device=d)
    with pytest.raises(P.PipError) as ei:  # workspace too small
        P.pip_voronoi_pieces(Vt, torch.from_numpy(off).to(d), torch.from_numpy(idx).to(d), Q,
                             workspace=torch.empty(256, dtype=torch.uint8, device=d))
    assert ei.value.status == 1
    K = 3000  # tables beyond the LDS limit
    off_big = torch.arange(0, 3 * K + 1, 3, dtype=torch.int32, device=d)
    idx_big = torch.zeros(3 * K, dtype=torch.int32, device=d)
    with pytest.raises(P.PipError) as ei:
        P.pip_voronoi_pieces(Vt, off_big, idx_big, Q)
    assert ei.value.status == 6


def test_pieces_full_size_sampled(P, oracle):
    """A 64-vertex star polygon against 2^26 float32 points; the oracle
    checks 2M sampled points and every point within 1e-6 of a boundary."""
    rng, V = star_case(14, 64)
    off, idx = P.convex_decompose(V, 64)
    m = 1 << 26
    Q = rng.uniform(-1.1, 1.1, (m, 2)).astype(np.float32)
    nb = m // 100
    Q[:nb] = boundary_points(rng, V, off, idx, nb - len(V), 1.0).astype(np.float32)
    say(f"[case] pieces full size: K={len(off) - 1}, m={m}")
    got, st = run(P, V, off, idx, Q)
    sel = np.concatenate([np.arange(nb), rng.choice(np.arange(nb, m), 2_000_000, replace=False)])
    want = oracle.voronoi_pieces(V, off, idx, Q[sel].astype(np.float64))
    bits = unpack_bits(got, m)[sel]
    assert np.array_equal(bits, want), int((bits != want).sum())
