"""The library's convex decomposition (host routine, no GPU needed): every
piece is strictly convex with 3..max vertices in the polygon's orientation,
the pieces' exact areas sum to the polygon's, every polygon edge bounds
exactly one piece and every diagonal two, and bad input is refused."""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np
import pytest

import polydecomp


@pytest.fixture(scope="module")
def P():
    import paper_2007_15385_amd as P
    P.load_library()
    return P


def _check(V, off, idx, max_n, strict_edges=True):
    n = len(V)
    Vl = [tuple(v) for v in V.tolist()]
    s = 1 if polydecomp.signed_area2(Vl) > 0 else -1
    total = Fr(0)
    edges = {}
    assert off[0] == 0 and off[-1] == len(idx)
    for k in range(len(off) - 1):
        pc = [int(i) for i in idx[off[k]:off[k + 1]]]
        assert 3 <= len(pc) <= max_n
        assert all(0 <= i < n for i in pc) and len(set(pc)) == len(pc)
        piece = [Vl[i] for i in pc]
        for t in range(len(pc)):
            assert s * polydecomp.orient(piece[t - 1], piece[t], piece[(t + 1) % len(pc)]) > 0
            e = (pc[t - 1], pc[t])
            edges[e] = edges.get(e, 0) + 1
        total += polydecomp.signed_area2(piece)
    assert total == polydecomp.signed_area2(Vl)
    for (a, b), c in edges.items():
        assert c == 1
        if not strict_edges:
            continue
        boundary = (b - a) % n == 1
        if not boundary:
            assert (b, a) in edges, "a diagonal bounds two pieces"


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("max_n", [3, 8, 64])
def test_decompose_star_polygons(P, seed, max_n):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 300))
    V = polydecomp.star_polygon(rng, n, center=tuple(rng.uniform(-1e3, 1e3, 2)))
    if seed % 2:
        V = V[::-1].copy()
    off, idx = P.convex_decompose(V, max_n)
    _check(V, off, idx, max_n)
    if max_n == 3:
        assert len(off) - 1 == n - 2


def test_decompose_convex_is_one_piece(P):
    rng = np.random.default_rng(7)
    import workloads as W
    V = W.circle_polygon(40, 1.0, (0.1, 0.2), rng)
    off, idx = P.convex_decompose(V, 64)
    assert off.tolist() == [0, 40] and sorted(idx.tolist()) == list(range(40))


def test_decompose_l_shape_and_collinear(P):
    V = np.array([[0, 0], [4, 0], [4, 2], [2, 2], [2, 4], [0, 4], [0, 2]], dtype=np.float64)
    off, idx = P.convex_decompose(V, 64)
    _check(V, off, idx, 64, strict_edges=False)
    assert 2 <= len(off) - 1 <= 3


def test_decompose_errors(P):
    with pytest.raises(P.PipError):
        P.convex_decompose(np.array([[0, 0], [1, 0], [2, 0]], float))  # zero area
    with pytest.raises(P.PipError):
        P.convex_decompose(np.array([[0, 0], [1, 0], [np.nan, 1]], float))
    bowtie = np.array([[0, 0], [2, 2], [2, 0], [0, 2]], float)  # self-intersecting
    try:
        off, idx = P.convex_decompose(bowtie)
    except P.PipError:
        return
    # if it returns, it returns pieces of valid shape (no guarantee of meaning)
    assert off[-1] == len(idx)
