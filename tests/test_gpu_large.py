"""Point counts past 2^31 (64-bit indexing through the streaming screens,
their recheck queues, the label stores and the ragged tail): 2^31 + 2^20 +
333 float32 points, with points within 1e-7 of the polygon's edges placed at
the start, across index 2^31 and at the end, so that binary64 rechecks
happen on both sides of 2^31.  The oracle checks a 2M-point random sample
plus those three ranges; the padding bits of the last label word are 0."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

M = (1 << 31) + (1 << 20) + 333
SPAN = 100_000


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_15385_amd as P
    P.load_library()
    return P


def near_edge_points(rng, V, k):
    Wv = np.roll(V, 1, 0)
    e = V - Wv
    L = np.hypot(e[:, 0], e[:, 1])
    i = rng.integers(len(V), size=k)
    t = rng.random(k)
    s = rng.choice([0.0, 1e-7, -1e-7], size=k)
    return np.stack([Wv[i, 0] + t * e[i, 0] + s * e[i, 1] / L[i],
                     Wv[i, 1] + t * e[i, 1] - s * e[i, 0] / L[i]], 1).astype(np.float32)


@pytest.fixture(scope="module")
def cloud(P):
    """The 2^31 + 2^20 + 333 points on the device (17 GB), and the index ranges
    that hold near-edge points of the 8-gon and the 40-gon below."""
    g = torch.Generator(device="cuda")
    g.manual_seed(2031)
    say(f"[case] large: generating {M} float32 points on the device")
    Q = torch.rand((M, 2), generator=g, device="cuda", dtype=torch.float32)
    Q.mul_(3.0).sub_(1.5)
    rng = np.random.default_rng(2031)
    polys = {n: W.circle_polygon(n, 1.0, (0.03, -0.02), rng) for n in (8, 40)}
    starts = [0, (1 << 31) - SPAN // 2, M - SPAN]
    for s, n in zip(starts, (8, 40, 8)):
        Q[s:s + SPAN // 2] = torch.from_numpy(near_edge_points(rng, polys[n], SPAN // 2)).cuda()
        other = 40 if n == 8 else 8
        Q[s + SPAN // 2:s + SPAN] = torch.from_numpy(
            near_edge_points(rng, polys[other], SPAN // 2)).cuda()
    idx = np.unique(np.concatenate([rng.integers(0, M, 2_000_000)] +
                                   [np.arange(s, s + SPAN) for s in starts]))
    Qs = Q[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    yield Q, polys, idx, Qs
    del Q
    torch.cuda.empty_cache()


CASES = [("pip_voronoi", "voronoi", 8, None), ("pip_voronoi", "voronoi", 40, None),
         ("pip_voronoi", "voronoi", 40, "radial"), ("pip_sign_of_offset", "sign_of_offset", 40, None),
         ("pip_ray_crossing", "ray_crossing", 8, None)]


@pytest.mark.parametrize("fn,test,n,opt", CASES)
def test_beyond_2_31_points(P, oracle, cloud, fn, test, n, opt):
    Q, polys, idx, Qs = cloud
    V = polys[n]
    old = P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES)
    if opt == "radial":
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3)
    try:
        say(f"[case] large: {fn} n={n} {opt or 'default screen'} m={M}")
        st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        lab = getattr(P, fn)(torch.from_numpy(V).cuda(), Q, status=st)
        torch.cuda.synchronize()
    finally:
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, old)
    assert int(st.item()) == 0
    words = lab.cpu().numpy().view(np.uint32)
    del lab
    assert words.size == (M + 31) // 32
    assert words[-1] >> (M % 32) == 0  # bits past the last point
    got = ((words[idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(bool)
    want = getattr(oracle, test)(V, Qs)
    bad = np.nonzero(got != want)[0]
    say(f"[stat] large {fn} n={n}: {len(idx)} points checked, {len(bad)} mismatches, "
        f"inside fraction {got.mean():.4f}")
    assert len(bad) == 0, idx[bad[:10]]
