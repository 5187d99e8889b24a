"""Host checks of the constants the point-location index relies on (no GPU).

The index widens each polygon's box by the distance within which binary64
rounding can call an outside point inside.  Part of that distance is the
rounding of the stored generators: the generator of edge i (Section 3,
Eq. 8, Algorithm 4) differs from the exact mirror image of the stored p_0
across the exact edge line by at most 64 v S, v = 2^-53, S the largest
coordinate magnitude of the vertices and p_0.  Here that bound is checked
with exact rational reflections on polygons whose coordinates mix very
small and very large magnitudes (the stored generators are the oracle's,
which the GPU reproduces bit for bit)."""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W

V53 = 2.0 ** -53


def _worst_ratio(oracle, V):
    P, rc = oracle.generators(V)
    if rc != 0:
        return None
    g0 = (Fr(P[0, 0]), Fr(P[0, 1]))
    S = max(float(np.abs(V).max()), float(np.abs(P[0]).max()))
    worst = 0.0
    for i in range(len(V)):
        vx, vy = Fr(V[i, 0]), Fr(V[i, 1])
        wx, wy = Fr(V[i - 1, 0]), Fr(V[i - 1, 1])
        ex, ey = vx - wx, vy - wy
        t = ((g0[0] - wx) * ex + (g0[1] - wy) * ey) / (ex * ex + ey * ey)
        rx, ry = 2 * (wx + t * ex) - g0[0], 2 * (wy + t * ey) - g0[1]
        dx, dy = Fr(P[i + 1, 0]) - rx, Fr(P[i + 1, 1]) - ry
        worst = max(worst, math.sqrt(float(dx * dx + dy * dy)) / (V53 * S))
    return worst


@pytest.mark.parametrize("kind", ["small_x_large_y", "large", "thin", "large_x_tiny"])
def test_generator_rounding_within_index_bound(oracle, kind):
    rng = np.random.default_rng({"small_x_large_y": 1, "large": 2, "thin": 3, "large_x_tiny": 4}[kind])
    ratios = []
    for _ in range(120):
        n = int(rng.integers(3, 17))
        if kind == "small_x_large_y":
            c = (rng.choice([-1, 1]) * 10 ** rng.uniform(-9, -3),
                 rng.choice([-1, 1]) * 10 ** rng.uniform(5, 7))
            r = 10 ** rng.uniform(-9, -3)
        elif kind == "large":
            c, r = rng.uniform(-1e7, 1e7, 2), 10 ** rng.uniform(-3, 3)
        elif kind == "thin":
            c, r = rng.uniform(-1e6, 1e6, 2), 10 ** rng.uniform(-6, 0)
        else:
            c, r = (10 ** rng.uniform(3, 7), 10 ** rng.uniform(-9, -6)), 10 ** rng.uniform(-9, -6)
        V = W.circle_polygon(n, r, c, rng)
        if kind == "thin":
            V[:, 1] = c[1] + (V[:, 1] - c[1]) * 1e-3
        x = _worst_ratio(oracle, V)
        if x is not None:
            ratios.append(x)
    assert len(ratios) > 60
    assert max(ratios) <= 64.0, max(ratios)
