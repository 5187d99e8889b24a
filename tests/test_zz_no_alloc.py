"""The batched entry point that allocates nothing (pip_voronoi_batched_noalloc,
on the library's static scratch array) against pip_voronoi_batched with a
caller workspace: bit-identical labels and status on two calls in a row, the
second with a smaller batch, so the array still holds the first call's tables;
and the size limit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W
from oracle import pack_bits

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


def batch(seed: int, num: int, size_hi: float, n_hi: int) -> W.Batch:
    """num polygons (3..n_hi edges, radius 0.5..50, centres in
    [-1000, 1000]^2), each against log-uniform [0, size_hi] normal points,
    a fifth of them within 1e-7 of an edge."""
    rng = np.random.default_rng(seed)
    polys, Qs = [], []
    for k in range(num):
        n = int(rng.integers(3, n_hi + 1))
        r = float(np.exp(rng.uniform(np.log(0.5), np.log(50))))
        c = rng.uniform(-1000, 1000, 2)
        V = W.circle_polygon(n, r, c, rng)
        s = int(np.exp(rng.uniform(0, np.log(size_hi)))) if k % 7 else 0
        q = rng.normal(c, 1.2 * r, size=(s, 2))
        if s >= 5:
            Wv = np.roll(V, 1, 0)
            e = V - Wv
            i = rng.integers(n, size=s // 5)
            t = rng.random(s // 5)
            L = np.hypot(e[i, 0], e[i, 1])
            off = rng.uniform(-1e-7, 1e-7, s // 5) * r
            q[: s // 5, 0] = Wv[i, 0] + t * e[i, 0] + off * e[i, 1] / L
            q[: s // 5, 1] = Wv[i, 1] + t * e[i, 1] - off * e[i, 0] / L
        polys.append(V)
        Qs.append(q.astype(np.float32))
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum([len(q) for q in Qs])]).astype(np.int64)
    return W.Batch(vtx_off, np.concatenate(polys), pt_off, np.concatenate(Qs),
                   W.label_word_offsets(pt_off))


def to_dev(B):
    d = "cuda"
    return (torch.from_numpy(B.vtx_off).to(d), torch.from_numpy(B.V).to(d),
            torch.from_numpy(B.pt_off).to(d), torch.from_numpy(B.Q).to(d),
            torch.from_numpy(B.lbl_word_off).to(d))


@pytest.mark.parametrize("radial", [0, 3])
def test_noalloc_matches_workspace_call(P, oracle, radial):
    old = P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES)
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, radial)
    try:
        # first call: ~6e7 tests over 1500 polygons; second: a smaller batch
        for seed, num, size_hi, n_hi in ((11, 1500, 2e5, 64), (12, 300, 3e4, 16)):
            B = batch(seed, num, size_hi, n_hi)
            need = P.batched_workspace_bytes(B.num_polygons, len(B.V), len(B.Q))
            assert need <= P.PIP_BATCHED_SCRATCH_BYTES
            say(f"[case] no-alloc batched: radial {radial}, {B.num_polygons} polygons, "
                f"{B.num_tests} tests, workspace {need} B")
            vo, V, po, Q, lo = to_dev(B)
            nwords = int(B.lbl_word_off[-1])
            # outputs pre-filled with different garbage: every word must be written
            lab_ws = torch.full((nwords,), -1, dtype=torch.int32, device="cuda")
            lab_na = torch.full((nwords,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            st_ws = torch.full((B.num_polygons,), -7, dtype=torch.int32, device="cuda")
            st_na = torch.full((B.num_polygons,), 99, dtype=torch.int32, device="cuda")
            P.pip_voronoi_batched(vo, V, po, Q, lo, labels=lab_ws, status=st_ws)
            P.pip_voronoi_batched_noalloc(vo, V, po, Q, lo, labels=lab_na, status=st_na)
            torch.cuda.synchronize()
            assert torch.equal(lab_na, lab_ws), "labels differ from pip_voronoi_batched"
            assert torch.equal(st_na, st_ws)
            assert (st_na.cpu().numpy() == 0).all()
            # and a few polygons in full against the binary64 oracle
            lab = lab_na.cpu().numpy().view(np.uint32)
            rng = np.random.default_rng(seed)
            for k in rng.choice(B.num_polygons, 12, replace=False):
                v0, v1 = B.vtx_off[k], B.vtx_off[k + 1]
                p0, p1 = B.pt_off[k], B.pt_off[k + 1]
                w0, w1 = B.lbl_word_off[k], B.lbl_word_off[k + 1]
                want = pack_bits(oracle.voronoi(B.V[v0:v1], B.Q[p0:p1].astype(np.float64)))
                assert np.array_equal(lab[w0:w1], want), f"polygon {k}"
    finally:
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old)


def test_noalloc_size_limit(P):
    """A batch whose tables exceed the scratch array is refused on the host
    (300,000 triangles, no points: no kernel runs)."""
    num = 300_000
    rng = np.random.default_rng(13)
    tri = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    V = (tri[None, :, :] + rng.uniform(-100, 100, (num, 1, 2))).reshape(-1, 2)
    vtx_off = (3 * np.arange(num + 1)).astype(np.int64)
    pt_off = np.zeros(num + 1, np.int64)
    need = P.batched_workspace_bytes(num, len(V), 0)
    assert need > P.PIP_BATCHED_SCRATCH_BYTES
    d = "cuda"
    with pytest.raises(P.PipError) as ei:
        P.pip_voronoi_batched_noalloc(torch.from_numpy(vtx_off).to(d), torch.from_numpy(V).to(d),
                                      torch.from_numpy(pt_off).to(d),
                                      torch.zeros((0, 2), dtype=torch.float32, device=d))
    assert ei.value.status == 6  # PIP_EUNSUPPORTED
    assert "scratch" in str(ei.value)
