"""Test-side shapes: random irregular convex polygons (no inclusion
arithmetic; the labels always come from the oracle)."""
from __future__ import annotations

import numpy as np


def random_convex(rng, n):
    """A random convex polygon with exactly n vertices, CCW, float64: n random
    x and n random y values, each sorted range split at random into two
    monotone chains whose successive differences (summing to zero) are
    paired at random and laid end to end in order of angle.  Irregular
    shapes: short and long edges, sharp and nearly flat vertices."""
    for _ in range(100):
        def steps(k):
            v = np.sort(rng.random(k))
            lo, hi = v[0], v[-1]
            a, b = lo, lo
            out = []
            for x in v[1:-1]:
                if rng.random() < 0.5:
                    out.append(x - a)
                    a = x
                else:
                    out.append(b - x)
                    b = x
            out += [hi - a, b - hi]
            return np.array(out)
        dx, dy = steps(n), rng.permutation(steps(n))
        ang = np.arctan2(dy, dx)
        o = np.argsort(ang)
        E = np.stack([dx[o], dy[o]], 1)
        V = np.cumsum(E, 0)
        V -= V.mean(0)
        x, y = V[:, 0], V[:, 1]
        nxt = np.roll(V, -1, 0) - V
        prv = V - np.roll(V, 1, 0)
        turn = prv[:, 0] * nxt[:, 1] - prv[:, 1] * nxt[:, 0]
        if np.all(turn > 1e-9 * np.abs(V).max() ** 2) and np.all(np.hypot(*prv.T) > 1e-6):
            return V
    raise AssertionError("no strictly convex polygon drawn")


def placed_convex(rng, n, stretch, size, centre):
    """random_convex stretched along x, rotated by a random angle, scaled to
    the given size (largest coordinate), moved to (centre, -0.7 centre) and
    reversed (clockwise) with probability 1/2."""
    V = random_convex(rng, n)
    V[:, 0] *= stretch
    th = rng.uniform(0, 2 * np.pi)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    V = V @ R.T
    V *= size / np.abs(V).max()
    V += np.array([centre, -0.7 * centre])
    if rng.random() < 0.5:
        V = V[::-1].copy()
    return V
