"""GPU parity of the batched persistent launch and its plans (autotuned tile
shape, hipGraph replay) against the FP64 oracle, polygon by polygon."""
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
    return P


@pytest.fixture(autouse=True, params=["radial", "per_edge"])
def screen(request, P):
    """Every test runs with the radial pre-screen forced for every polygon
    size and with it off (plans and workspaces take the setting at creation)."""
    old = P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES)
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3 if request.param == "radial" else 0)
    yield request.param
    P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old)


def to_dev(B):
    d = "cuda"
    return (torch.from_numpy(B.vtx_off).to(d), torch.from_numpy(B.V).to(d),
            torch.from_numpy(B.pt_off).to(d), torch.from_numpy(B.Q).to(d),
            torch.from_numpy(B.lbl_word_off).to(d))


def check_batch(oracle, B, labels, polys=None, status=None):
    lab = labels.cpu().numpy().view(np.uint32)
    bad = []
    ks = range(B.num_polygons) if polys is None else polys
    for k in ks:
        v0, v1 = B.vtx_off[k], B.vtx_off[k + 1]
        p0, p1 = B.pt_off[k], B.pt_off[k + 1]
        w0, w1 = B.lbl_word_off[k], B.lbl_word_off[k + 1]
        if p1 == p0:
            continue
        n = v1 - v0
        if 3 <= n <= 64:
            want = pack_bits(oracle.voronoi(B.V[v0:v1], B.Q[p0:p1].astype(np.float64)))
        else:
            want = np.zeros(w1 - w0, dtype=np.uint32)
        if not np.array_equal(lab[w0:w1], want):
            g = unpack_bits(lab[w0:w1], p1 - p0)
            wv = unpack_bits(want, p1 - p0)
            bad.append((k, int(n), int((g != wv).sum())))
    assert not bad, f"polygons with label mismatches (k, n, count): {bad[:10]}"


def small_batch(seed=0, P=60, far=True):
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 31, 32, 33, 255, 256, 257, 511, 1000, 4097] + \
        list(rng.integers(0, 3000, size=P - 11))
    ns = list(rng.integers(3, 65, size=P))
    polys, Qs = [], []
    for k in range(P):
        r = float(np.exp(rng.uniform(np.log(0.5), np.log(50))))
        c = rng.uniform(-1000, 1000, 2) if far else rng.uniform(-1, 1, 2)
        V = W.circle_polygon(int(ns[k]), r, c, rng)
        s = int(sizes[k])
        q = rng.normal(c, 1.2 * r, size=(s, 2))
        if s > 10:
            Wv = np.roll(V, 1, 0)
            e = V - Wv
            i = rng.integers(len(V), size=s // 5)
            t = rng.random(s // 5)
            L = np.hypot(e[i, 0], e[i, 1])
            off = rng.choice([0.0, 1e-9, -1e-9, 1e-7 * r, -1e-7 * r], size=s // 5)
            q[: s // 5, 0] = Wv[i, 0] + t * e[i, 0] + off * e[i, 1] / L
            q[: s // 5, 1] = Wv[i, 1] + t * e[i, 1] - off * e[i, 0] / L
        polys.append(V)
        Qs.append(q.astype(np.float32))
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum([len(q) for q in Qs])]).astype(np.int64)
    return W.Batch(vtx_off, np.concatenate(polys), pt_off,
                   np.concatenate(Qs) if pt_off[-1] else np.zeros((0, 2), np.float32),
                   W.label_word_offsets(pt_off))


@pytest.mark.parametrize("far", [False, True])
def test_batched_small(P, oracle, far):
    B = small_batch(1, far=far)
    vo, V, po, Q, lo = to_dev(B)
    labels, _, status = P.pip_voronoi_batched(vo, V, po, Q, lo)
    torch.cuda.synchronize()
    check_batch(oracle, B, labels)
    assert (status.cpu().numpy() == 0).all()


@pytest.mark.parametrize("cfg", [(1, 1), (1, 4), (3, 2), (16, 8), (1 << 30, 4), (64, 1)])
def test_batched_tile_shapes_agree(P, oracle, cfg):
    B = small_batch(2)
    vo, V, po, Q, lo = to_dev(B)
    say(f"[case] batched tile shape {cfg}")
    labels, _, _ = P.pip_voronoi_batched(vo, V, po, Q, lo, config=cfg)
    torch.cuda.synchronize()
    check_batch(oracle, B, labels)


def test_batched_invalid_polygons(P, oracle):
    """n = 2 -> PIP_EINVAL, n = 65 -> PIP_EUNSUPPORTED: their points are
    labelled 0; the other polygons are unaffected."""
    rng = np.random.default_rng(3)
    polys = [W.circle_polygon(5, 1.0, (0, 0), rng), np.array([[0.0, 0.0], [1.0, 1.0]]),
             W.circle_polygon(8, 2.0, (3, 3), rng), W.circle_polygon(65, 1.0, (0, 0), rng),
             np.array([[0, 0], [1, 0], [2, 0]], float)]
    Qs = [rng.uniform(-2, 5, (700, 2)).astype(np.float32) for _ in polys]
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum([len(q) for q in Qs])]).astype(np.int64)
    B = W.Batch(vtx_off, np.concatenate(polys), pt_off, np.concatenate(Qs),
                W.label_word_offsets(pt_off))
    vo, V, po, Q, lo = to_dev(B)
    labels, _, status = P.pip_voronoi_batched(vo, V, po, Q, lo)
    torch.cuda.synchronize()
    assert status.cpu().numpy().tolist() == [0, 1, 0, 6, 2]
    check_batch(oracle, B, labels)


def test_batched_empty_and_single(P, oracle):
    B = small_batch(4, P=12)
    vo, V, po, Q, lo = to_dev(B)
    labels, _, _ = P.pip_voronoi_batched(vo[:2], V, po[:2], Q, lo[:2])
    torch.cuda.synchronize()
    check_batch(oracle, B, labels, polys=[0])


def test_plan_autotune_and_graph_replay(P, oracle):
    B = small_batch(5, P=200)
    vo, V, po, Q, lo = to_dev(B)
    plan = P.BatchedPlan(vo, V, po, Q, lo)
    cfg, ms = plan.autotune(reps=2)
    say(f"[stat] autotuned tile shape {cfg}, {ms:.4f} ms")
    assert ms > 0
    want = None
    for r in range(4):
        plan.labels.zero_()
        plan.launch()
        torch.cuda.synchronize()
        check_batch(oracle, B, plan.labels)
        got = plan.labels.clone()
        want = got if want is None else want
        assert torch.equal(got, want)
        # eager work between replays
        torch.cuda.synchronize()
        _ = (Q * 2.0).sum().item()
    # the graph reads the bound buffers: new point values give new labels
    rng = np.random.default_rng(6)
    B.Q[:] = (B.Q + rng.normal(0, 0.05, B.Q.shape)).astype(np.float32)
    Q.copy_(torch.from_numpy(B.Q))
    plan.launch()
    torch.cuda.synchronize()
    check_batch(oracle, B, plan.labels)
    plan.set_config(4, 2)
    plan.launch()
    torch.cuda.synchronize()
    check_batch(oracle, B, plan.labels)
    plan.close()


def test_uneven_batch_full_size(P, oracle):
    """4096 polygons, n in [3, 32], set sizes log-uniform [1e3, 1e6] (about
    5.9e8 point-polygon tests) through an autotuned graph-captured plan; the
    oracle checks 96 polygons in full plus every polygon's first 2000 points."""
    say("[case] uneven batch: generating")
    B = W.uneven_batch()
    say(f"[case] uneven batch: {B.num_tests} tests, GPU")
    vo, V, po, Q, lo = to_dev(B)
    plan = P.BatchedPlan(vo, V, po, Q, lo)
    cfg, ms = plan.autotune(reps=2)
    plan.launch()
    torch.cuda.synchronize()
    say(f"[stat] uneven batch tile shape {cfg}: {ms:.3f} ms, "
        f"{B.num_tests / ms / 1e6:.1f} G tests/s")
    rng = np.random.default_rng(7)
    check_batch(oracle, B, plan.labels, polys=sorted(rng.choice(B.num_polygons, 96, replace=False)))
    lab = plan.labels.cpu().numpy().view(np.uint32)
    bad = 0
    for k in range(B.num_polygons):
        p0, p1 = B.pt_off[k], min(B.pt_off[k + 1], B.pt_off[k] + 2000)
        v0, v1 = B.vtx_off[k], B.vtx_off[k + 1]
        want = oracle.voronoi(B.V[v0:v1], B.Q[p0:p1].astype(np.float64))
        w0 = B.lbl_word_off[k]
        got = unpack_bits(lab[w0:w0 + (p1 - p0 + 31) // 32], p1 - p0)
        bad += int((got != want).sum())
    assert bad == 0
    assert (plan.status.cpu().numpy() == 0).all()
    plan.close()


def test_batched_irregular(P, oracle):
    """A batch of 72 irregular convex polygons (random edge lengths and
    turns, 3 to 64 vertices, stretched up to 10^4:1, sizes 10^-4..10^4,
    centres up to 10^5, either orientation), each with uniform points over
    its bounding box and points at 0..10^-5 of its size from its edges."""
    from shapes import placed_convex
    rng = np.random.default_rng(71)
    polys, Qs = [], []
    for k in range(72):
        n = int(rng.integers(3, 65))
        stretch, size, centre = [(1.0, 1.0, 0.0), (1e2, 1e-3, 1e3), (1e4, 1e4, -1e5),
                                 (30.0, 1e-4, 0.5)][k % 4]
        V = placed_convex(rng, n, stretch, size, centre)
        lo, hi = V.min(0), V.max(0)
        span = hi - lo
        s = int(rng.integers(1, 4000))
        q = rng.uniform(lo - 0.25 * span, hi + 0.25 * span, size=(s, 2))
        m = s // 4
        if m:
            Wv = np.roll(V, 1, 0)
            e = V - Wv
            i = rng.integers(n, size=m)
            t = rng.random(m)
            L = np.hypot(e[i, 0], e[i, 1])
            off = rng.choice([0.0, 1e-9 * size, -1e-9 * size, 1e-7 * size, -1e-5 * size], size=m)
            q[:m, 0] = Wv[i, 0] + t * e[i, 0] + off * e[i, 1] / L
            q[:m, 1] = Wv[i, 1] + t * e[i, 1] - off * e[i, 0] / L
        polys.append(V)
        Qs.append(q.astype(np.float32))
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    pt_off = np.concatenate([[0], np.cumsum([len(q) for q in Qs])]).astype(np.int64)
    B = W.Batch(vtx_off, np.concatenate(polys), pt_off, np.concatenate(Qs),
                W.label_word_offsets(pt_off))
    vo, V, po, Q, lo = to_dev(B)
    say(f"[case] batched irregular polygons, {int(pt_off[-1])} points")
    labels, _, status = P.pip_voronoi_batched(vo, V, po, Q, lo)
    torch.cuda.synchronize()
    check_batch(oracle, B, labels)
    assert (status.cpu().numpy() == 0).all()
