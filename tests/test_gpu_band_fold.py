"""GPU parity of the two band forms of the vector screens (single polygon and
batched): chunks whose points all satisfy |X| + |Y| <= RQ take the folded
linear band, chunks holding one point beyond RQ take the full band with its
quadratic term.  Labels must equal the FP64 oracle's (Algorithm 5) bit for
bit in both, including points within 1e-12..1e-6 of an edge, far points and
non-finite coordinates."""
from __future__ import annotations

import sys

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
    old = (P.get_option(P.PIP_OPT_MFMA_MIN_EDGES), P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES))
    P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, 0)  # vector screen for every size
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 0)
    yield P
    P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, old[0])
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old[1])


def screen_table(P, V):
    t = P.pip_screen_table(torch.from_numpy(V).cuda(), 0, 0).cpu().numpy()
    return {"ox": t[0], "oy": t[1], "KQ": float(t[2]), "KA": float(t[3]), "KB": float(t[4]),
            "KC": float(t[5]), "RQ": float(t[8])}


def edge_points(rng, V, k, offsets):
    Wv = np.roll(V, 1, 0)
    e = V - Wv
    L = np.hypot(e[:, 0], e[:, 1])
    i = rng.integers(len(V), size=k)
    t = rng.random(k)
    s = rng.choice(offsets, size=k)
    return np.stack([Wv[i, 0] + t * e[i, 0] + s * e[i, 1] / L[i],
                     Wv[i, 1] + t * e[i, 1] - s * e[i, 0] / L[i]], 1)


def fold_case_points(rng, V, T, chunks=24):
    """512-point chunks around V: even chunks near the polygon only, odd
    chunks the same with one point beyond RQ (in local coordinates) at a
    random lane, the last chunk ragged with far and non-finite points."""
    r = float(np.abs(V - V.mean(0)).max())
    ox, oy = float(T["ox"]), float(T["oy"])
    out = []
    for c in range(chunks):
        q = np.concatenate([edge_points(rng, V, 256, [0.0, 1e-12, -1e-12, 1e-9, -1e-9,
                                                      1e-6 * r, -1e-6 * r]),
                            V.mean(0) + rng.normal(0.0, 1.2 * r, size=(256, 2))])
        if c % 2:
            d = T["RQ"] * rng.uniform(1.01, 1e3)
            a = rng.uniform(0, 2 * np.pi)
            q[rng.integers(512)] = (ox + d * np.cos(a), oy + d * np.sin(a))
        out.append(q)
    tail = np.concatenate([edge_points(rng, V, 100, [0.0, 1e-9, -1e-9]),
                           rng.uniform(-1e20, 1e20, size=(20, 2)),
                           [[np.nan, oy], [ox, np.inf], [-np.inf, -np.inf]]])
    out.append(tail)
    return np.concatenate(out).astype(np.float32)


def test_screen_table_fold_radius(P):
    """RQ is 0 or a power of two, and the folded constants cover the
    quadratic term up to RQ: KQ RQ <= 2^-8 min(KA, KB)."""
    rng = np.random.default_rng(41)
    for n in (3, 8, 16, 24):
        for r in (1e-6, 1e-3, 1.0, 1e3, 1e6):
            V = W.circle_polygon(n, r, rng.uniform(-10 * r, 10 * r, 2), rng)
            T = screen_table(P, V)
            RQ = T["RQ"]
            assert RQ > 0.0
            m, e = np.frexp(RQ)
            assert m == 0.5, (n, r, RQ)
            assert T["KQ"] * RQ <= 2.0 ** -8 * min(T["KA"], T["KB"]) * (1 + 2.0 ** -20), (n, r)


@pytest.mark.parametrize("n", [3, 5, 8, 13, 16, 24])
@pytest.mark.parametrize("r", [1e-3, 1.0, 1e3])
def test_single_polygon_both_band_forms(P, oracle, n, r):
    rng = np.random.default_rng(1000 + n)
    V = W.circle_polygon(n, r, rng.uniform(-100 * r, 100 * r, 2), rng)
    T = screen_table(P, V)
    Q = fold_case_points(rng, V, T)
    say(f"[case] band fold single n={n} r={r} RQ={T['RQ']:.3g} m={len(Q)}")
    w = P.pip_voronoi(torch.from_numpy(V).cuda(), torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    got = w.cpu().numpy().view(np.uint32)
    want = pack_bits(oracle.voronoi(V, Q.astype(np.float64)))
    if not np.array_equal(got, want):
        bad = np.nonzero(unpack_bits(got, len(Q)) != unpack_bits(want, len(Q)))[0]
        raise AssertionError(f"{len(bad)} label mismatches, first at {bad[:10]}")


def test_batched_both_band_forms(P, oracle):
    rng = np.random.default_rng(77)
    polys, Qs = [], []
    for k in range(40):
        n = int(rng.integers(3, 33))
        r = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e3))))
        V = W.circle_polygon(n, r, rng.uniform(-1000, 1000, 2), rng)
        T = screen_table(P, V)
        q = fold_case_points(rng, V, T, chunks=int(rng.integers(1, 6)))
        polys.append(V)
        Qs.append(q[: int(rng.integers(1, len(q) + 1))])
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum([len(q) for q in Qs])]).astype(np.int64)
    B = W.Batch(vtx_off, np.concatenate(polys), pt_off, np.concatenate(Qs),
                W.label_word_offsets(pt_off))
    d = "cuda"
    say(f"[case] band fold batched P=40 points={int(pt_off[-1])}")
    labels, _, status = P.pip_voronoi_batched(
        torch.from_numpy(B.vtx_off).to(d), torch.from_numpy(B.V).to(d),
        torch.from_numpy(B.pt_off).to(d), torch.from_numpy(B.Q).to(d),
        torch.from_numpy(B.lbl_word_off).to(d))
    torch.cuda.synchronize()
    lab = labels.cpu().numpy().view(np.uint32)
    bad = []
    for k in range(B.num_polygons):
        p0, p1 = B.pt_off[k], B.pt_off[k + 1]
        w0, w1 = B.lbl_word_off[k], B.lbl_word_off[k + 1]
        want = pack_bits(oracle.voronoi(polys[k], Qs[k].astype(np.float64)))
        if not np.array_equal(lab[w0:w1], want):
            bad.append((k, int((unpack_bits(lab[w0:w1], p1 - p0) !=
                                unpack_bits(want, p1 - p0)).sum())))
    assert not bad, f"polygons with label mismatches (k, count): {bad[:10]}"
    assert (status.cpu().numpy() == 0).all()
