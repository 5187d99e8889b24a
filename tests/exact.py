"""Exact rational arithmetic versions of the paper's algorithms (tests only).

Python ``fractions.Fraction`` evaluates the centroid (Section 3, Eq. 3-4),
the generators (Section 3, Eq. 8), the Voronoi predicate (Section 4, Eq. 1
with the squared norms of Eq. 10-11), sign of offset (Section 2.2) and ray
crossing (Section 2.1) with no rounding at all, so on small-integer or
dyadic inputs they give the mathematically exact answer against which the
float64 oracle is pinned.  ``convex_contains`` is the textbook closed
half-plane definition of a convex polygon, an independent route to the same
set as the Voronoi polygon.
"""
from __future__ import annotations

from fractions import Fraction as Fr


def _fr(v):
    return [(Fr(x), Fr(y)) for x, y in v]


def centroid(V):
    V = _fr(V)
    n = len(V)
    S = Sx = Sy = Fr(0)
    for i in range(n):
        vx, vy = V[i]
        wx, wy = V[i - 1]
        A = wx * vy - vx * wy
        S += A
        Sx += (vx + wx) * A
        Sy += (vy + wy) * A
    area = S / 2
    return (Sx / (6 * area), Sy / (6 * area)), area


def generators(V):
    """[(g0), g_0, ..., g_{n-1}] exactly: g_i = g0 reflected across the line
    through v_{i-1} and v_i (Eq. 6-8)."""
    (g0x, g0y), _ = centroid(V)
    V = _fr(V)
    out = [(g0x, g0y)]
    for i in range(len(V)):
        vx, vy = V[i]
        wx, wy = V[i - 1]
        a = vy - wy
        b = wx - vx
        c = -(a * vx + b * vy)
        den = a * a + b * b
        gx = ((b * b - a * a) * g0x - 2 * a * b * g0y - 2 * c * a) / den
        gy = (-2 * a * b * g0x + (a * a - b * b) * g0y - 2 * c * b) / den
        out.append((gx, gy))
    return out


def voronoi_margins(P, p):
    """m_i = |p - g0|^2 - |p - g_i|^2 for every outer generator (exact)."""
    px, py = Fr(p[0]), Fr(p[1])
    g0x, g0y = P[0]
    M0 = (px - g0x) ** 2 + (py - g0y) ** 2
    return [M0 - ((px - gx) ** 2 + (py - gy) ** 2) for gx, gy in P[1:]]


def voronoi(V, p, P=None):
    P = P if P is not None else generators(V)
    return all(mi <= 0 for mi in voronoi_margins(P, p))


def sign_of_offset(V, p):
    V = _fr(V)
    px, py = Fr(p[0]), Fr(p[1])
    n = len(V)
    cnt = 0
    for i in range(n):
        vx, vy = V[i]
        wx, wy = V[i - 1]
        dVx, dVy = vx - wx, vy - wy
        if py * dVx - px * dVy < wy * dVx - wx * dVy:
            cnt += 1
    return cnt % n == 0


def ray_crossing(V, p):
    V = _fr(V)
    px, py = Fr(p[0]), Fr(p[1])
    cnt = 0
    for i in range(len(V)):
        vx, vy = V[i]
        wx, wy = V[i - 1]
        in_range = (vy > py) != (wy > py)
        up = vy > wy
        dVx, dVy = vx - wx, vy - wy
        lhs = py * dVx - px * dVy
        rhs = wy * dVx - wx * dVy
        left = lhs > rhs if up else lhs < rhs
        if in_range and left:
            cnt += 1
    return cnt % 2 == 1


def convex_contains(V, p):
    """Closed convex polygon membership by exact orientation tests: p is on
    the inner closed side of every edge line (either orientation)."""
    V = _fr(V)
    px, py = Fr(p[0]), Fr(p[1])
    s = []
    for i in range(len(V)):
        vx, vy = V[i]
        wx, wy = V[i - 1]
        s.append((vx - wx) * (py - wy) - (vy - wy) * (px - wx))
    return all(x >= 0 for x in s) or all(x <= 0 for x in s)
