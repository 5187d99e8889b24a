"""Exact convex decomposition of simple polygons (tests only).

Ear clipping with exact rational orientation tests, then the greedy removal
of every diagonal whose two sides merge into a convex piece (Hertel and
Mehlhorn's rule).  Pieces are index lists into the polygon's vertices, in the
polygon's own cyclic order.  Independent of the library's decomposition
routine; the oracle's union-of-pieces test takes whatever decomposition it is
given, so this file only produces valid inputs and exact reference sets.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np


def orient(a, b, c) -> Fr:
    """Twice the signed area of triangle abc, exactly."""
    ax, ay = Fr(a[0]), Fr(a[1])
    return (Fr(b[0]) - ax) * (Fr(c[1]) - ay) - (Fr(b[1]) - ay) * (Fr(c[0]) - ax)


def signed_area2(V) -> Fr:
    s = Fr(0)
    for i in range(len(V)):
        x0, y0 = V[i - 1]
        x1, y1 = V[i]
        s += Fr(x0) * Fr(y1) - Fr(x1) * Fr(y0)
    return s


def on_segment(p, a, b) -> bool:
    if orient(a, b, p) != 0:
        return False
    return (min(Fr(a[0]), Fr(b[0])) <= Fr(p[0]) <= max(Fr(a[0]), Fr(b[0])) and
            min(Fr(a[1]), Fr(b[1])) <= Fr(p[1]) <= max(Fr(a[1]), Fr(b[1])))


def triangulate(V) -> list[tuple[int, int, int]]:
    """Ear clipping; triangles as vertex-index triples in the polygon's
    orientation.  Vertices collinear with both neighbours are dropped from
    the remaining chain (they lie on an edge of it)."""
    n = len(V)
    s = 1 if signed_area2(V) > 0 else -1
    idx = list(range(n))
    tris = []
    guard = 0
    while len(idx) > 3:
        guard += 1
        if guard > 4 * n * n:
            raise ValueError("polygon is not simple")
        m = len(idx)
        clipped = False
        for t in range(m):
            i0, i1, i2 = idx[t - 1], idx[t], idx[(t + 1) % m]
            o = s * orient(V[i0], V[i1], V[i2])
            if o == 0:
                if on_segment(V[i1], V[i0], V[i2]):
                    del idx[t]
                    clipped = True
                    break
                continue
            if o < 0:
                continue
            ear = True
            for j in idx:
                if j in (i0, i1, i2):
                    continue
                p = V[j]
                if (s * orient(V[i0], V[i1], p) >= 0 and s * orient(V[i1], V[i2], p) >= 0 and
                        s * orient(V[i2], V[i0], p) >= 0):
                    ear = False
                    break
            if ear:
                tris.append((i0, i1, i2))
                del idx[t]
                clipped = True
                break
        if not clipped:
            raise ValueError("no ear found: polygon is not simple")
    if len(idx) == 3 and orient(V[idx[0]], V[idx[1]], V[idx[2]]) != 0:
        tris.append(tuple(idx))
    return tris


def _convex(V, piece, s) -> bool:
    k = len(piece)
    for t in range(k):
        if s * orient(V[piece[t - 1]], V[piece[t]], V[piece[(t + 1) % k]]) < 0:
            return False
    return True


def merge(V, tris, max_n: int = 64) -> list[list[int]]:
    """Remove diagonals greedily while both sides merge into a convex piece
    of at most max_n vertices."""
    s = 1 if signed_area2(V) > 0 else -1
    pieces = [list(t) for t in tris]
    changed = True
    while changed:
        changed = False
        for a in range(len(pieces)):
            for b in range(a + 1, len(pieces)):
                pa, pb = pieces[a], pieces[b]
                shared = None
                for t in range(len(pa)):
                    u, v = pa[t], pa[(t + 1) % len(pa)]
                    for r in range(len(pb)):
                        if pb[r] == v and pb[(r + 1) % len(pb)] == u:
                            shared = (t, r)
                            break
                    if shared:
                        break
                if not shared:
                    continue
                t, r = shared
                # pa from its vertex after u..v: v, ..., u; then pb's vertices strictly between u and v
                la, lb = len(pa), len(pb)
                seq = [pa[(t + 1 + q) % la] for q in range(la)]      # v ... u
                mid = [pb[(r + 2 + q) % lb] for q in range(lb - 2)]  # after u ... before v
                cand = seq + mid
                if len(cand) <= max_n and _convex(V, cand, s):
                    pieces[a] = cand
                    del pieces[b]
                    changed = True
                    break
            if changed:
                break
    return pieces


def to_csr(pieces):
    off = np.concatenate([[0], np.cumsum([len(p) for p in pieces])]).astype(np.int64)
    idx = np.array([i for p in pieces for i in p], dtype=np.int64)
    return off, idx


def decompose(V, max_n: int = 64, merged: bool = True):
    """(piece_off, piece_idx) of a convex decomposition of simple polygon V."""
    Vl = [tuple(map(float, v)) for v in np.asarray(V, dtype=np.float64)]
    tris = triangulate(Vl)
    return to_csr(merge(Vl, tris, max_n) if merged else [list(t) for t in tris])


def closed_contains(V, p) -> bool:
    """Exact membership of p in the closed simple polygon V: on an edge, or
    an odd number of crossings of a ray towards +x (exact, half-open rule)."""
    n = len(V)
    for i in range(n):
        if on_segment(p, V[i - 1], V[i]):
            return True
    px, py = Fr(p[0]), Fr(p[1])
    c = 0
    for i in range(n):
        ax, ay = Fr(V[i - 1][0]), Fr(V[i - 1][1])
        bx, by = Fr(V[i][0]), Fr(V[i][1])
        if (ay > py) != (by > py):
            x = ax + (py - ay) * (bx - ax) / (by - ay)
            if x > px:
                c += 1
    return c % 2 == 1


def star_polygon(rng, n, r_lo=0.4, r_hi=1.0, center=(0.0, 0.0), integer_scale=None):
    """Simple polygon, star-shaped about `center`: increasing angles, one
    per sector of 2 pi / n (n >= 3, so every gap is below pi), random radii.  With integer_scale, integer
    vertices whose exact angular order is strictly increasing."""
    for _ in range(1000):
        # one angle per sector of 2 pi / n, away from the sector ends
        th = (np.arange(n) + rng.uniform(0.1, 0.9, n)) * (2 * np.pi / n) + rng.uniform(0, 2 * np.pi)
        r = rng.uniform(r_lo, r_hi, n)
        V = np.stack([center[0] + r * np.cos(th), center[1] + r * np.sin(th)], 1)
        if integer_scale is None:
            return V
        Vi = np.round((V - np.asarray(center)) * integer_scale)
        if _strict_angular(Vi):
            return Vi + np.round(np.asarray(center))
    raise RuntimeError("no polygon")


def _strict_angular(Vi) -> bool:
    """Consecutive vertices turn strictly counter-clockwise about the origin
    (cross product > 0) with every step below pi: a simple star polygon."""
    n = len(Vi)
    for i in range(n):
        a, b = Vi[i - 1], Vi[i]
        if a[0] == 0 and a[1] == 0:
            return False
        if a[0] * b[1] - a[1] * b[0] <= 0:
            return False
    return True
