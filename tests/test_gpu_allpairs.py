"""GPU parity of the pose placement and the all-pairs test against the FP64
oracle: bit-identical world vertices, labels and inside-counts."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import workloads as W

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


def run_allpairs(P, F, poses, cs, Q):
    Ft = torch.from_numpy(F).cuda()
    pt = torch.from_numpy(poses).cuda()
    ct = torch.from_numpy(cs).cuda()
    Vw = P.pip_poses_to_polygons(Ft, pt, ct)
    lab, cnt, st = P.pip_voronoi_allpairs(Vw, torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    return Vw.cpu().numpy(), lab.cpu().numpy().view(np.uint32), cnt.cpu().numpy(), st.cpu().numpy()


def test_pose_polygons_bit_exact(P, oracle):
    F = W.car_footprint()
    poses, cs = W.random_poses(300)
    Ft = torch.from_numpy(F).cuda()
    Vw = P.pip_poses_to_polygons(Ft, torch.from_numpy(poses).cuda(),
                                 torch.from_numpy(cs).cuda()).cpu().numpy()
    for k in range(len(poses)):
        want = oracle.pose_polygon(F, float(poses[k, 0]), float(poses[k, 1]), cs[k, 0], cs[k, 1])
        assert np.array_equal(Vw[k].view(np.uint64), want.view(np.uint64)), k


@pytest.mark.parametrize("m", [1, 33, 1000, 1025, 5000])
def test_allpairs_small(P, oracle, m):
    rng = np.random.default_rng(m)
    F = W.car_footprint()
    poses, cs = W.random_poses(37, extent=3.0)
    Q = rng.uniform(-6, 6, size=(m, 2)).astype(np.float32)
    Vw, lab, cnt, st = run_allpairs(P, F, poses, cs, Q)
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    assert np.array_equal(lab, bits)
    assert np.array_equal(cnt, counts)
    assert (st == 0).all()


def test_allpairs_points_on_placed_edges(P, oracle):
    """Points on the world-frame edges of each placed footprint (and within
    1 ulp .. 1e-6 of them), for poses near and far from the origin."""
    rng = np.random.default_rng(21)
    F = W.car_footprint()
    poses, cs = W.random_poses(64, extent=40.0)
    pts = []
    for k in range(0, 64, 4):
        Wk = oracle.pose_polygon(F, float(poses[k, 0]), float(poses[k, 1]), cs[k, 0], cs[k, 1])
        Wr = np.roll(Wk, 1, 0)
        e = Wk - Wr
        L = np.hypot(e[:, 0], e[:, 1])
        for off in (0.0, 1e-12, -1e-9, 1e-7, -1e-6):
            i = rng.integers(8, size=40)
            t = rng.random(40)
            pts.append(np.stack([Wr[i, 0] + t * e[i, 0] + off * e[i, 1] / L[i],
                                 Wr[i, 1] + t * e[i, 1] - off * e[i, 0] / L[i]], 1))
        pts.append(Wk)
    Q = np.concatenate(pts).astype(np.float32)
    Vw, lab, cnt, st = run_allpairs(P, F, poses, cs, Q)
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    assert np.array_equal(lab, bits)
    assert np.array_equal(cnt, counts)


def test_allpairs_nonfinite_and_general_polygons(P, oracle):
    rng = np.random.default_rng(22)
    polys = np.stack([W.circle_polygon(13, 2.0, rng.uniform(-3, 3, 2), rng) for _ in range(20)])
    Q = rng.uniform(-5, 5, size=(3000, 2)).astype(np.float32)
    Q[::97] = np.nan
    Q[5::101, 0] = np.inf
    lab, cnt, st = P.pip_voronoi_allpairs(torch.from_numpy(polys).cuda(), torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    lab = lab.cpu().numpy().view(np.uint32)
    from oracle import pack_bits
    for k in range(len(polys)):
        want = oracle.voronoi(polys[k], Q.astype(np.float64))
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum())


def test_allpairs_full_size(P, oracle):
    """131,072 lidar points x 2048 poses of the car footprint (2^28 tests),
    every label and count against the oracle."""
    F = W.car_footprint()
    Q = W.lidar_cloud()
    poses, cs = W.random_poses()
    say("[case] all pairs full size: GPU")
    Vw, lab, cnt, st = run_allpairs(P, F, poses, cs, Q)
    say("[case] all pairs full size: oracle")
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    bad = np.nonzero((lab != bits).any(axis=1))[0]
    say(f"[stat] all pairs: {int(counts.sum())} inside pairs, {len(bad)} poses with mismatches")
    assert len(bad) == 0
    assert np.array_equal(cnt, counts)


def _allpairs_cull(P, F, poses, cs, Q, cull):
    P.set_option(P.PIP_OPT_ALLPAIRS_CULL, cull)
    try:
        return run_allpairs(P, F, poses, cs, Q)
    finally:
        P.set_option(P.PIP_OPT_ALLPAIRS_CULL, 0)


def test_allpairs_cull_full_size_identical(P):
    """The culled launch returns exactly the dense labels and counts on the
    2048-pose x 131,072-point lidar configuration."""
    F = W.car_footprint()
    Q = W.lidar_cloud()
    poses, cs = W.random_poses()
    _, lab0, cnt0, _ = _allpairs_cull(P, F, poses, cs, Q, 0)
    _, lab1, cnt1, _ = _allpairs_cull(P, F, poses, cs, Q, 1)
    assert np.array_equal(lab0, lab1)
    assert np.array_equal(cnt0, cnt1)
    say(f"[stat] cull: {int(cnt0.sum())} inside pairs, identical to dense")


def test_allpairs_cull_adversarial_identical(P, oracle):
    """Poses whose disk just touches a ring (ring radius = pose distance +- the
    footprint radius), a cloud far from the origin (|c| >> R, where float32
    rounding of the centre matters) and points on placed edges: culled ==
    dense == oracle."""
    rng = np.random.default_rng(77)
    F = W.car_footprint()
    R0 = float(np.sqrt((F ** 2).sum(1)).max())
    # rings at radii r, poses at distances r - R0 - s for tiny s (tangent from inside)
    rings = []
    for r in (3.0, 10.0, 25.0):
        az = rng.uniform(0, 2 * np.pi, 512)
        rings.append(np.stack([r * np.cos(az), r * np.sin(az)], 1))
    far = 1.0e5 + rng.uniform(-5, 5, size=(512, 2))  # a cluster far from the origin
    Q = np.concatenate(rings + [far]).astype(np.float32)
    K = 96
    th = rng.uniform(-np.pi, np.pi, K).astype(np.float32)
    d = np.concatenate([np.array([3.0, 10.0, 25.0])[rng.integers(0, 3, K - 16)]
                        - R0 * rng.choice([-1.0, 1.0], K - 16) * (1 + rng.uniform(-1e-3, 1e-3, K - 16)),
                        np.full(16, 1.0e5 * np.sqrt(2.0))])
    ang = rng.uniform(0, 2 * np.pi, K)
    ang[-16:] = np.pi / 4
    poses = np.stack([d * np.cos(ang), d * np.sin(ang), th], 1).astype(np.float32)
    cs = np.stack([np.cos(poses[:, 2].astype(np.float64)), np.sin(poses[:, 2].astype(np.float64))], 1)
    _, lab0, cnt0, _ = _allpairs_cull(P, F, poses, cs, Q, 0)
    _, lab1, cnt1, _ = _allpairs_cull(P, F, poses, cs, Q, 1)
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    assert np.array_equal(lab0, bits) and np.array_equal(cnt0, counts)
    assert np.array_equal(lab1, bits) and np.array_equal(cnt1, counts)
    say(f"[stat] adversarial cull: {int(counts.sum())} inside pairs of {K * len(Q)}")


def _allpairs_opts(P, F, poses, cs, Q, cull, pair):
    """Placed footprints through pip_voronoi_allpairs with the given options;
    also returns the pair count each polygon's table was built with (the
    int32 at byte 48 of its 64-byte workspace header)."""
    Ft = torch.from_numpy(F).cuda()
    Vw = P.pip_poses_to_polygons(Ft, torch.from_numpy(poses).cuda(), torch.from_numpy(cs).cuda())
    need = P.allpairs_workspace_bytes(Vw.shape[0], Vw.shape[1])
    ws = torch.zeros(max(need, 256), dtype=torch.uint8, device="cuda")
    P.set_option(P.PIP_OPT_ALLPAIRS_CULL, cull)
    P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, pair)
    try:
        lab, cnt, _ = P.pip_voronoi_allpairs(Vw, torch.from_numpy(Q).cuda(), workspace=ws)
        torch.cuda.synchronize()
    finally:
        P.set_option(P.PIP_OPT_ALLPAIRS_CULL, 0)
        P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, 0)
    npair = ws[: 64 * Vw.shape[0]].cpu().numpy().view(np.int32).reshape(-1, 16)[:, 12]
    return lab.cpu().numpy().view(np.uint32), cnt.cpu().numpy(), npair


def test_allpairs_pair_full_size(P, oracle):
    """Antipodal pairing (alone and with culling) on the 2048-pose x 131,072
    lidar configuration: every placed car footprint is paired (4 pairs) and
    every label and count equals the oracle's."""
    F = W.car_footprint()
    Q = W.lidar_cloud()
    poses, cs = W.random_poses()
    say("[case] all pairs paired full size: GPU")
    lab1, cnt1, np1 = _allpairs_opts(P, F, poses, cs, Q, 0, 1)
    lab2, cnt2, np2 = _allpairs_opts(P, F, poses, cs, Q, 1, 1)
    assert (np1 == 4).all() and (np2 == 4).all()
    say("[case] all pairs paired full size: oracle")
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    assert np.array_equal(lab1, bits) and np.array_equal(cnt1, counts)
    assert np.array_equal(lab2, bits) and np.array_equal(cnt2, counts)


@pytest.mark.parametrize("cull", [0, 1])
def test_allpairs_pair_adversarial(P, oracle, cull):
    """Pairing near the band: points on the placed edges, at vertices and
    within 1e-12 .. 1e-6 of edges, poses at up to 40 m (paired), at 1e3 m
    (the binary64 centroid's rounding leaves an asymmetry near the pairing
    limit) and at 1e5 m (far past it: per-edge table)."""
    rng = np.random.default_rng(31 + cull)
    F = W.car_footprint()
    poses, cs = W.random_poses(64, extent=40.0)
    poses[-16:-8, :2] = (1.0e3 + rng.uniform(-3, 3, size=(8, 2))).astype(np.float32)
    poses[-8:, :2] = (1.0e5 + rng.uniform(-3, 3, size=(8, 2))).astype(np.float32)
    pts = []
    for k in range(0, 64, 2):
        Wk = oracle.pose_polygon(F, float(poses[k, 0]), float(poses[k, 1]), cs[k, 0], cs[k, 1])
        Wr = np.roll(Wk, 1, 0)
        e = Wk - Wr
        L = np.hypot(e[:, 0], e[:, 1])
        for off in (0.0, 1e-12, -1e-9, 1e-7, -1e-6):
            i = rng.integers(8, size=24)
            t = rng.random(24)
            pts.append(np.stack([Wr[i, 0] + t * e[i, 0] + off * e[i, 1] / L[i],
                                 Wr[i, 1] + t * e[i, 1] - off * e[i, 0] / L[i]], 1))
        pts.append(Wk)
    Q = np.concatenate(pts).astype(np.float32)
    lab, cnt, npair = _allpairs_opts(P, F, poses, cs, Q, cull, 1)
    assert (npair[:48] == 4).all() and (npair[-8:] == 0).all()
    bits, counts = oracle.allpairs(F, poses[:, :2].astype(np.float64), cs, Q.astype(np.float64))
    assert np.array_equal(lab, bits)
    assert np.array_equal(cnt, counts)
    say(f"[stat] paired adversarial (cull {cull}): {int(counts.sum())} inside pairs, "
        f"pairs at 1e3 m: {npair[-16:-8].tolist()}")


@pytest.mark.parametrize("n,expect", [(4, 2), (6, 3), (16, 8), (64, 32), (7, 0)])
def test_allpairs_pair_regular_and_fallback(P, oracle, n, expect):
    """Regular polygons (centrally symmetric for even n: n/2 pairs, padded
    rows for n/2 not a multiple of 4), an odd n and a perturbed even polygon
    (both keep the per-edge table): labels equal the oracle's either way."""
    from oracle import pack_bits
    rng = np.random.default_rng(n)
    ang = 2 * np.pi * np.arange(n) / n + 0.3
    base = np.stack([1.7 * np.cos(ang), 1.7 * np.sin(ang)], 1)
    polys = [base + c for c in rng.uniform(-30, 30, size=(12, 2))]
    if n % 2 == 0:
        bent = base.copy()
        bent[0] *= 1.0 + 1e-4  # no longer symmetric
        polys.append(bent + 2.0)
    V = np.stack(polys).astype(np.float64)
    Q = np.concatenate([rng.uniform(-33, 33, size=(4000, 2))] +
                       [p[rng.integers(n, size=64)] + rng.normal(0, 1e-6, (64, 2)) for p in polys])
    Q = Q.astype(np.float32)
    need = P.allpairs_workspace_bytes(V.shape[0], n)
    ws = torch.zeros(max(need, 256), dtype=torch.uint8, device="cuda")
    P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, 1)
    try:
        lab, cnt, _ = P.pip_voronoi_allpairs(torch.from_numpy(V).cuda(), torch.from_numpy(Q).cuda(),
                                             workspace=ws)
        torch.cuda.synchronize()
    finally:
        P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, 0)
    npair = ws[: 64 * V.shape[0]].cpu().numpy().view(np.int32).reshape(-1, 16)[:, 12]
    assert (npair[:12] == expect).all()
    if n % 2 == 0:
        assert npair[12] == 0
    lab = lab.cpu().numpy().view(np.uint32)
    cnt = cnt.cpu().numpy()
    for k in range(len(V)):
        want = oracle.voronoi(V[k], Q.astype(np.float64))
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum())


def test_allpairs_plan_autotune_and_graph_replays(P):
    """The all-pairs plan: autotune times the four exact variants on the lidar
    configuration and keeps one; every replay of the captured graph (with eager
    work and synchronisations between replays) gives the eager dense labels and
    counts, and so does every forced variant."""
    F = W.car_footprint()
    Q = torch.from_numpy(W.lidar_cloud()).cuda()
    poses, cs = W.random_poses()
    Vw = P.pip_poses_to_polygons(torch.from_numpy(F).cuda(), torch.from_numpy(poses).cuda(),
                                 torch.from_numpy(cs).cuda())
    lab_e, cnt_e, _ = P.pip_voronoi_allpairs(Vw, Q)
    torch.cuda.synchronize()
    plan = P.AllpairsPlan(Vw, Q)
    try:
        cfg, ms = plan.autotune(reps=2)
        say(f"[stat] all-pairs plan: variant (cull, pair) = {cfg}, {ms:.4f} ms")
        assert cfg in ((0, 0), (1, 0), (0, 1), (1, 1)) and ms > 0
        for _ in range(3):
            plan.labels.zero_()
            plan.counts.fill_(-1)
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            assert torch.equal(plan.labels, lab_e) and torch.equal(plan.counts, cnt_e)
        for c in ((0, 0), (1, 0), (0, 1), (1, 1)):
            plan.set_config(*c)
            plan.labels.zero_()
            plan.launch()
            torch.cuda.synchronize()
            assert plan.config()[0] == c
            assert torch.equal(plan.labels, lab_e) and torch.equal(plan.counts, cnt_e)
        # the batched shape calls reject an all-pairs plan
        import ctypes
        from paper_2007_15385_amd._lib import BatchedConfig
        from paper_2007_15385_amd.api import _lib as lib
        assert lib().pip_plan_set_config(plan.handle, ctypes.byref(BatchedConfig(1, 1))) == 1
    finally:
        plan.close()


# ---------------------------------------------------------------------------
# CSR polygons of uneven vertex counts
# ---------------------------------------------------------------------------
def csr_polygons(rng, P, n_lo=3, n_hi=64, extent=40.0, r_lo=0.5, r_hi=6.0):
    polys = []
    for _ in range(P):
        n = int(rng.integers(n_lo, n_hi + 1))
        polys.append(W.circle_polygon(n, float(rng.uniform(r_lo, r_hi)),
                                      rng.uniform(-extent, extent, 2), rng))
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    return polys, vtx_off, np.concatenate(polys)


def run_csr(P, vtx_off, V, Q):
    lab, cnt, st = P.pip_voronoi_allpairs_csr(torch.from_numpy(vtx_off).cuda(),
                                              torch.from_numpy(V).cuda(),
                                              torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    return lab.cpu().numpy().view(np.uint32), cnt.cpu().numpy(), st.cpu().numpy()


@pytest.fixture(params=["dense", "cull_pair"])
def allpairs_variant(request, P):
    """Dense, then with culling and antipodal pairing switched on (labels and
    counts must not change)."""
    on = 1 if request.param == "cull_pair" else 0
    old = (P.get_option(P.PIP_OPT_ALLPAIRS_CULL), P.get_option(P.PIP_OPT_ALLPAIRS_PAIR))
    P.set_option(P.PIP_OPT_ALLPAIRS_CULL, on)
    P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, on)
    yield request.param
    P.set_option(P.PIP_OPT_ALLPAIRS_CULL, old[0])
    P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, old[1])


@pytest.mark.parametrize("m", [1, 513, 2048, 5001])
def test_allpairs_csr_small(P, oracle, allpairs_variant, m):
    from oracle import pack_bits
    rng = np.random.default_rng(300 + m)
    polys, vtx_off, V = csr_polygons(rng, 45, extent=4.0)
    # symmetric polygons (regular even n) exercise the paired rows
    th = np.arange(16) * np.pi / 8
    polys[3] = 2.0 * np.stack([np.cos(th), np.sin(th)], 1)
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    V = np.concatenate(polys)
    Q = rng.uniform(-8, 8, size=(m, 2)).astype(np.float32)
    lab, cnt, st = run_csr(P, vtx_off, V, Q)
    for k, Vk in enumerate(polys):
        want = oracle.voronoi(Vk, Q.astype(np.float64))
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum()), k
    assert (st == 0).all()


def test_allpairs_csr_edges_and_invalid(P, oracle, allpairs_variant):
    """Points on and within 1e-9..1e-6 of every polygon's edges; polygons
    with 2 and 65 vertices and an empty one get PIP_EINVAL /
    PIP_EUNSUPPORTED, zero labels and zero counts; the rest are exact."""
    from oracle import pack_bits
    rng = np.random.default_rng(31)
    polys, _, _ = csr_polygons(rng, 20, extent=30.0)
    polys.insert(5, np.array([[0.0, 0.0], [1.0, 1.0]]))
    polys.insert(9, W.circle_polygon(65, 3.0, (1.0, 2.0), rng))
    polys.insert(12, np.zeros((0, 2)))
    pts = []
    for Vk in polys:
        if not 3 <= len(Vk) <= 64:
            continue
        Wr = np.roll(Vk, 1, 0)
        e = Vk - Wr
        L = np.hypot(e[:, 0], e[:, 1])
        for off in (0.0, 1e-9, -1e-9, 1e-7, -1e-6):
            i = rng.integers(len(Vk), size=30)
            t = rng.random(30)
            pts.append(np.stack([Wr[i, 0] + t * e[i, 0] + off * e[i, 1] / L[i],
                                 Wr[i, 1] + t * e[i, 1] - off * e[i, 0] / L[i]], 1))
        pts.append(Vk)
    Q = np.concatenate(pts).astype(np.float32)
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    V = np.concatenate(polys)
    lab, cnt, st = run_csr(P, vtx_off, V, Q)
    for k, Vk in enumerate(polys):
        if len(Vk) < 3:
            assert st[k] == 1 and cnt[k] == 0 and not lab[k].any(), k
            continue
        if len(Vk) > 64:
            assert st[k] == 6 and cnt[k] == 0 and not lab[k].any(), k
            continue
        want = oracle.voronoi(Vk, Q.astype(np.float64))
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum()) and st[k] == 0, k


def test_allpairs_csr_matches_uniform(P):
    """Polygons of one vertex count through both entry points: identical
    labels and counts."""
    rng = np.random.default_rng(33)
    polys = np.stack([W.circle_polygon(8, 2.0, rng.uniform(-20, 20, 2), rng) for _ in range(300)])
    Q = rng.uniform(-25, 25, size=(20000, 2)).astype(np.float32)
    Qt = torch.from_numpy(Q).cuda()
    lab_u, cnt_u, _ = P.pip_voronoi_allpairs(torch.from_numpy(polys).cuda(), Qt)
    vtx_off = (8 * np.arange(301)).astype(np.int64)
    lab_c, cnt_c, _ = P.pip_voronoi_allpairs_csr(torch.from_numpy(vtx_off).cuda(),
                                                 torch.from_numpy(polys.reshape(-1, 2)).cuda(), Qt)
    torch.cuda.synchronize()
    assert torch.equal(lab_u, lab_c) and torch.equal(cnt_u, cnt_c)


def test_allpairs_csr_full_size(P, oracle):
    """2048 polygons of 3..64 vertices (centres in [-40, 40]^2, radii
    0.5..6) against the 131,072-point lidar cloud: 64 polygons checked in
    full and the first 4096 points of every polygon, plus every count of the
    checked polygons."""
    from oracle import pack_bits, unpack_bits
    rng = np.random.default_rng(34)
    polys, vtx_off, V = csr_polygons(rng, 2048)
    Q = W.lidar_cloud()
    say(f"[case] all pairs CSR: {len(polys)} polygons x {len(Q)} points")
    lab, cnt, st = run_csr(P, vtx_off, V, Q)
    assert (st == 0).all()
    Q64 = Q.astype(np.float64)
    for k in sorted(rng.choice(len(polys), 64, replace=False)):
        want = oracle.voronoi(polys[k], Q64)
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum()), k
    Qh = Q64[:4096]
    bad = 0
    for k in range(len(polys)):
        want = oracle.voronoi(polys[k], Qh)
        bad += int((unpack_bits(lab[k], len(Q))[:4096] != want).sum())
    assert bad == 0


def test_allpairs_csr_irregular(P, oracle, allpairs_variant):
    """40 irregular convex polygons (random edge lengths and turns, 3 to 64
    vertices, stretched up to 10^3:1, sizes 0.05..5, either orientation)
    spread over one cloud: uniform points plus points on and within
    10^-9..10^-5 of every polygon's edges, labels and counts exact."""
    from oracle import pack_bits
    from shapes import placed_convex
    rng = np.random.default_rng(401)
    polys = []
    for k in range(40):
        n = int(rng.integers(3, 65))
        V = placed_convex(rng, n, float(10.0 ** rng.uniform(0, 3)),
                          float(10.0 ** rng.uniform(np.log10(0.05), np.log10(5.0))), 0.0)
        polys.append(V + rng.uniform(-6, 6, 2))
    pts = [rng.uniform(-8, 8, size=(6000, 2))]
    for Vk in polys:
        Wr = np.roll(Vk, 1, 0)
        e = Vk - Wr
        L = np.hypot(e[:, 0], e[:, 1])
        for off in (0.0, 1e-9, -1e-9, 1e-7, -1e-5):
            i = rng.integers(len(Vk), size=20)
            t = rng.random(20)
            pts.append(np.stack([Wr[i, 0] + t * e[i, 0] + off * e[i, 1] / L[i],
                                 Wr[i, 1] + t * e[i, 1] - off * e[i, 0] / L[i]], 1))
        pts.append(Vk)
    Q = np.concatenate(pts).astype(np.float32)
    vtx_off = np.concatenate([[0], np.cumsum([len(v) for v in polys])]).astype(np.int64)
    V = np.concatenate(polys)
    lab, cnt, st = run_csr(P, vtx_off, V, Q)
    assert (st == 0).all(), st
    for k, Vk in enumerate(polys):
        want = oracle.voronoi(Vk, Q.astype(np.float64))
        assert np.array_equal(lab[k], pack_bits(want)), k
        assert int(cnt[k]) == int(want.sum()), k
