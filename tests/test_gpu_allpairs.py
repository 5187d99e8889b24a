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
