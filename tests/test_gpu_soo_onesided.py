"""The one-sided sign-of-offset screen (Section 2.2, Algorithm 2): each
polygon's rows are oriented so that the inner side of every edge is
positive, a point is decided inside when its smallest float32 offset clears
the band, and outside when that offset clears the band on the other side
and fl32(|X| + |Y|) is below the polygon's bound SO, which must guarantee
that some other edge's exact offset clears the band on the inner side (so
that Algorithm 2's binary64 comparisons disagree).

Checked here: that guarantee with exact rational arithmetic (the binary64
rounded edge vectors of Algorithm 2, the float32 local coordinates, the
stored band constants) on points with fl32(|X| + |Y|) just below SO and on
random points below it, for regular, irregular, clockwise, sliver, tiny and
far polygons; 0 < SO <= RQ / 2 (the frame of these screens is the vertex mean, so a
tiny polygon far from the origin, whose binary64 centroid can lie far from
it, keeps a usable bound); SO = 0 for a polygon without area; and the
labels of those polygons against the FP64 oracle on the vector and
matrix-core screens."""
from __future__ import annotations

import sys
from fractions import Fraction as Fr

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


def polygons():
    rng = np.random.default_rng(88)
    out = [("square", np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)),
           ("square cw", np.array([[0, 0], [0, 1], [1, 1], [1, 0]], float)),
           ("sliver", np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 1e-7]])),
           ("sliver cw far", np.array([[1e4, 3e3], [1e4 + 0.5, 3e3 + 1e-6], [1e4 + 1.0, 3e3]])),
           ("tiny far", W.circle_polygon(8, 1e-4, (1e4, -2e4), rng)),
           ("needle", placed_convex(rng, 12, 1e4, 10.0, 0.0)),
           ("tiny very far", W.circle_polygon(16, 1e-3, (3e6, -1e6), rng)),
           ("far needle", placed_convex(rng, 24, 1e3, 1e-2, 1e6))]
    for n in (3, 5, 16, 33, 64):
        out.append((f"circle {n}", W.circle_polygon(n, 1.0, (0.03, -0.02), rng)))
        out.append((f"irregular {n}", placed_convex(rng, n, 30.0, 100.0, 1e3)))
    return out


def orientation(V):
    """Sign of C = -sum(V'_y dV_x - V'_x dV_y) over the binary64 rounded edge
    vectors of Algorithm 2, exactly (twice the signed area when the edge
    vectors close up); wherever the bound SO is positive, the preparation's
    binary64 value of C has this sign."""
    Vp = np.roll(V, 1, 0)
    d = V - Vp
    C = -sum(Fr(float(Vp[i, 1])) * Fr(float(d[i, 0])) - Fr(float(Vp[i, 0])) * Fr(float(d[i, 1]))
             for i in range(len(V)))
    return -1 if C < 0 else 1


def f32(x):
    return float(np.float32(x))


@pytest.mark.parametrize("matrix", [0, 1])
def test_outside_bound_is_sound(P, matrix):
    rng = np.random.default_rng(89 + matrix)
    for name, V in polygons():
        t = P.pip_screen_table(torch.from_numpy(V).cuda(), 1, matrix).cpu().numpy()
        ox, oy, KA, KB, KC, RQ, SO = (float(t[k]) for k in (0, 1, 3, 4, 5, 8, 9))
        assert int(t[7]) == 0, name
        assert 0.0 < SO <= 0.5 * RQ, (name, SO, RQ)
        KS = max(KA, KB)
        sg = orientation(V)
        n = len(V)
        Vp = np.roll(V, 1, 0)
        d = V - Vp  # binary64 rounded edge vectors of Algorithm 2
        # points: random directions at radii that put fl32(|X| + |Y|) just
        # below SO, and random points below it
        m = 300
        th = rng.uniform(0, 2 * np.pi, m)
        c, s = np.cos(th), np.sin(th)
        rad = np.where(np.arange(m) < m // 2, SO * (1 - 2.0 ** -22), SO * rng.random(m))
        rad = rad / (np.abs(c) + np.abs(s))
        Q = np.stack([ox + rad * c, oy + rad * s], 1).astype(np.float32)
        checked = 0
        for qx, qy in Q.astype(np.float64):
            X, Y = f32(np.float32(qx) - np.float32(ox)), f32(np.float32(qy) - np.float32(oy))
            sxy = f32(np.float32(abs(X)) + np.float32(abs(Y)))
            if not sxy < SO:
                continue
            checked += 1
            band = Fr(KS) * (abs(Fr(X)) + abs(Fr(Y))) + Fr(KC)
            best = max(sg * (Fr(float(d[i, 0])) * (Fr(qy) - Fr(float(Vp[i, 1])))
                             - Fr(float(d[i, 1])) * (Fr(qx) - Fr(float(Vp[i, 0]))))
                       for i in range(n))
            assert best > band, (name, qx, qy, float(best), float(band))
        assert checked > m // 2, (name, checked)
        say(f"[stat] one-sided bound {name} matrix={matrix}: SO = {SO:.4g}, RQ = {RQ:.4g}, "
            f"{checked} points checked exactly")


def test_no_area_no_bound(P):
    V = np.array([[0, 0], [1, 0], [2, 0]], float)
    t = P.pip_screen_table(torch.from_numpy(V).cuda(), 1, 0).cpu().numpy()
    assert int(t[7]) == 2 and float(t[9]) == 0.0


@pytest.mark.parametrize("mfma_min", [0, 3])
def test_labels(P, oracle, mfma_min):
    """Every polygon above, 40,000 float32 points over 4x its bounding box
    (most far outside, beyond SO for the small ones) plus points on and near
    its edges: labels bit-identical to the oracle."""
    old = P.get_option(P.PIP_OPT_MFMA_MIN_EDGES)
    P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, mfma_min)
    try:
        rng = np.random.default_rng(90)
        for name, V in polygons():
            lo, hi = V.min(0), V.max(0)
            span = np.maximum(hi - lo, 1e-3 * np.abs(V).max())
            Q = rng.uniform(lo - 1.5 * span, hi + 1.5 * span, size=(40000, 2))
            Vp = np.roll(V, 1, 0)
            e = V - Vp
            L = np.hypot(e[:, 0], e[:, 1])
            i = rng.integers(len(V), size=4000)
            tt = rng.random(4000)
            off = rng.choice([0.0, 1e-9, -1e-9, 1e-6, -1e-6], size=4000) * np.abs(V).max()
            Q[:4000, 0] = Vp[i, 0] + tt * e[i, 0] + off * e[i, 1] / L[i]
            Q[:4000, 1] = Vp[i, 1] + tt * e[i, 1] - off * e[i, 0] / L[i]
            Q = Q.astype(np.float32)
            st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
            w = P.pip_sign_of_offset(torch.from_numpy(V).cuda(), torch.from_numpy(Q).cuda(), status=st)
            torch.cuda.synchronize()
            got = w.cpu().numpy().view(np.uint32)
            want = pack_bits(oracle.sign_of_offset(V, Q.astype(np.float64)))
            assert int(st.item()) == 0, name
            if not np.array_equal(got, want):
                g, h = unpack_bits(got, len(Q)), unpack_bits(want, len(Q))
                bad = np.nonzero(g != h)[0]
                raise AssertionError(f"{name}: {len(bad)} mismatches, first {bad[:8]}")
    finally:
        P.set_option(P.PIP_OPT_MFMA_MIN_EDGES, old)
