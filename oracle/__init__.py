"""FP64 CPU oracle (test infrastructure only).

Plain, slow, per-point loops in binary64 that follow the paper's algorithms
(Zengin & Sezer, arXiv:2007.15385): the centroid (Section 3, Eq. 3-4,
Algorithm 3), the generators (Section 3, Eq. 5-8, Algorithm 4), the Voronoi
test (Section 4, Eq. 1 and 9-11, Algorithm 5), sign of offset (Section 2.2,
Algorithm 2) and ray crossing (Section 2.1, Algorithm 1), plus the rigid
footprint placement and the collision cost built on the normalized margin.

Only the tests, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library:
the C source is compiled here with gcc (``-O2 -ffp-contract=off``) into
``liboracle.so`` and loaded with ctypes.

Inputs are widened to float64 before the call (float32 -> float64 is exact),
so a float32 point cloud is tested exactly as the GPU receives it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-std=c11", "-Wall", "-Wextra"]


def build(src: str = _SRC, out: str = _LIB, defines: tuple = ()) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    cmd = ["gcc", *GCC_FLAGS, *[f"-D{d}" for d in defines], "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    sig = {
        "oracle_num_threads": (ctypes.c_int, []),
        "oracle_set_num_threads": (None, [ctypes.c_int]),
        "oracle_centroid": (ctypes.c_int, [_D, _i64, _D, _D]),
        "oracle_generators": (ctypes.c_int, [_D, _i64, _D]),
        "oracle_voronoi": (ctypes.c_int, [_D, _i64, _D, _i64, _U8]),
        "oracle_voronoi_pieces": (ctypes.c_int, [_D, _i64, _I64, _i64, _I64, _D, _i64, _U8]),
        "oracle_locate": (ctypes.c_int, [_I64, _i64, _D, _D, _i64, _I32]),
        "oracle_voronoi_raster": (ctypes.c_int, [_D, _i64, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, _i64, _i64,
                                                 _U8]),
        "oracle_voronoi_max_margin": (None, [_D, _i64, _D, _i64, _D]),
        "oracle_sign_of_offset": (None, [_D, _i64, _D, _i64, _U8]),
        "oracle_ray_crossing": (None, [_D, _i64, _D, _i64, _U8]),
        "oracle_pose_polygon": (None, [_D, _i64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _D]),
        "oracle_allpairs": (None, [_D, _i64, _D, _D, _i64, _D, _i64, _U32, _I64]),
        "oracle_cost": (ctypes.c_int, [_D, _i64, _D, _i64, _D, _i64, _D]),
        "oracle_cost_state": (ctypes.c_int, [_D, _i64, _D, _D, _i64, _I32]),
        "oracle_cost_grad": (ctypes.c_int, [_D, _i64, _D, _i64, _D, _i64, _D, _D, _D, _D, _D]),
        "oracle_cost_with_hash": (ctypes.c_int, [_D, _i64, _D, _i64, _D, _i64, _D,
                                                 ctypes.POINTER(ctypes.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib_cache: dict = {}


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (building first if needed) the oracle library at ``path``."""
    path = path or _LIB
    if path in _lib_cache:
        return _lib_cache[path]
    if path == _LIB and (not os.path.exists(_LIB) or
                         os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build()
    lib = _bind(ctypes.CDLL(path))
    _lib_cache[path] = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray, t=_D):
    return a.ctypes.data_as(t)


class Oracle:
    """Thin numpy front end over one build of the C oracle."""

    def __init__(self, path: str | None = None):
        self.lib = load(path)

    # -- bookkeeping -----------------------------------------------------
    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, t: int) -> None:
        self.lib.oracle_set_num_threads(int(t))

    # -- Section 3 -------------------------------------------------------
    def centroid(self, V):
        V = _f64(V).reshape(-1, 2)
        g0 = np.zeros(2)
        area = np.zeros(1)
        rc = self.lib.oracle_centroid(_p(V), len(V), _p(g0), _p(area))
        return g0, float(area[0]), int(rc)

    def generators(self, V):
        """(n+1, 2) float64: row 0 = p_0, row 1+i = generator of edge i."""
        V = _f64(V).reshape(-1, 2)
        P = np.zeros((len(V) + 1, 2))
        rc = self.lib.oracle_generators(_p(V), len(V), _p(P))
        return P, int(rc)

    # -- the three tests ---------------------------------------------------
    def voronoi(self, V, Q) -> np.ndarray:
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        out = np.zeros(len(Q), dtype=np.uint8)
        self.lib.oracle_voronoi(_p(V), len(V), _p(Q), len(Q), _p(out, _U8))
        return out.astype(bool)

    def voronoi_pieces(self, V, piece_off, piece_idx, Q, with_status: bool = False):
        """Non-convex polygon V as the union of convex pieces (piece k is
        V[piece_idx[piece_off[k]:piece_off[k+1]]]): inside iff the closed
        Voronoi test of some piece says inside."""
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        off = np.ascontiguousarray(piece_off, dtype=np.int64)
        idx = np.ascontiguousarray(piece_idx, dtype=np.int64)
        if len(idx) == 0:
            idx = np.zeros(1, np.int64)
        out = np.zeros(len(Q), dtype=np.uint8)
        rc = self.lib.oracle_voronoi_pieces(_p(V), len(V), _p(off, _I64), len(off) - 1,
                                            _p(idx, _I64), _p(Q), len(Q), _p(out, _U8))
        if rc == -3:
            raise ValueError("a piece vertex index lies outside the polygon")
        return (out.astype(bool), int(rc)) if with_status else out.astype(bool)

    def voronoi_raster(self, V, x0, y0, dx, dy, width, height) -> np.ndarray:
        """[height, width] bool: pixel (i, j) is the point (x0 + i dx, y0 + j dy)."""
        V = _f64(V).reshape(-1, 2)
        out = np.zeros((height, width), dtype=np.uint8)
        self.lib.oracle_voronoi_raster(_p(V), len(V), float(x0), float(y0), float(dx), float(dy),
                                       int(width), int(height), _p(out, _U8))
        return out.astype(bool)

    def locate(self, vtx_off, V, Q) -> np.ndarray:
        """[m] int32: smallest k whose polygon V[vtx_off[k]:vtx_off[k+1]]
        contains point j (Voronoi test), or -1."""
        off = np.ascontiguousarray(vtx_off, dtype=np.int64)
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        ids = np.zeros(len(Q), dtype=np.int32)
        rc = self.lib.oracle_locate(_p(off, _I64), len(off) - 1, _p(V), _p(Q), len(Q),
                                    _p(ids, _I32))
        if rc != 0:
            raise MemoryError("oracle_locate")
        return ids

    def voronoi_max_margin(self, V, Q) -> np.ndarray:
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        out = np.zeros(len(Q))
        self.lib.oracle_voronoi_max_margin(_p(V), len(V), _p(Q), len(Q), _p(out))
        return out

    def sign_of_offset(self, V, Q) -> np.ndarray:
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        out = np.zeros(len(Q), dtype=np.uint8)
        self.lib.oracle_sign_of_offset(_p(V), len(V), _p(Q), len(Q), _p(out, _U8))
        return out.astype(bool)

    def ray_crossing(self, V, Q) -> np.ndarray:
        V = _f64(V).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        out = np.zeros(len(Q), dtype=np.uint8)
        self.lib.oracle_ray_crossing(_p(V), len(V), _p(Q), len(Q), _p(out, _U8))
        return out.astype(bool)

    # -- poses, all pairs, cost -------------------------------------------
    def pose_polygon(self, F, tx, ty, c, s) -> np.ndarray:
        F = _f64(F).reshape(-1, 2)
        W = np.zeros_like(F)
        self.lib.oracle_pose_polygon(_p(F), len(F), float(tx), float(ty), float(c), float(s),
                                     _p(W))
        return W

    def allpairs(self, F, poses_xy, cs, Q):
        """Packed labels [K][ceil(m/32)] uint32 and inside-counts [K]."""
        F = _f64(F).reshape(-1, 2)
        poses_xy = _f64(poses_xy).reshape(-1, 2)
        cs = _f64(cs).reshape(-1, 2)
        Q = _f64(Q).reshape(-1, 2)
        K, m = len(poses_xy), len(Q)
        bits = np.zeros((K, (m + 31) // 32), dtype=np.uint32)
        counts = np.zeros(K, dtype=np.int64)
        self.lib.oracle_allpairs(_p(F), len(F), _p(poses_xy), _p(cs), K, _p(Q), m,
                                 _p(bits, _U32), _p(counts, _I64))
        return bits, counts

    def cost(self, F, poses, Q) -> np.ndarray:
        F = _f64(F).reshape(-1, 2)
        poses = _f64(poses).reshape(-1, 3)
        Q = _f64(Q).reshape(-1, 2)
        out = np.zeros(len(poses))
        self.lib.oracle_cost(_p(F), len(F), _p(poses), len(poses), _p(Q), len(Q), _p(out))
        return out

    def cost_state(self, F, pose, Q) -> np.ndarray:
        F = _f64(F).reshape(-1, 2)
        pose = _f64(pose).reshape(3)
        Q = _f64(Q).reshape(-1, 2)
        st = np.zeros(len(Q), dtype=np.int32)
        self.lib.oracle_cost_state(_p(F), len(F), _p(pose), _p(Q), len(Q), _p(st, _I32))
        return st

    def cost_grad(self, F, poses, Q, w=None, with_scale=False):
        """Closed-form gradient of sum_k w_k C_k: ([K][3], [n][2]); with
        with_scale also the sums of |per-point contributions| (same shapes)."""
        F = _f64(F).reshape(-1, 2)
        poses = _f64(poses).reshape(-1, 3)
        Q = _f64(Q).reshape(-1, 2)
        K = len(poses)
        w = np.ones(K) if w is None else _f64(w).reshape(K)
        gp = np.zeros((K, 3))
        gF = np.zeros_like(F)
        ap = np.zeros((K, 3))
        aF = np.zeros_like(F)
        self.lib.oracle_cost_grad(_p(F), len(F), _p(poses), K, _p(Q), len(Q), _p(w), _p(gp),
                                  _p(gF), _p(ap), _p(aF))
        return (gp, gF, ap, aF) if with_scale else (gp, gF)

    def cost_with_hash(self, F, poses, Q):
        """Costs [K] and per-pose hashes of the per-point kink states."""
        F = _f64(F).reshape(-1, 2)
        poses = _f64(poses).reshape(-1, 3)
        Q = _f64(Q).reshape(-1, 2)
        K = len(poses)
        c = np.zeros(K)
        h = np.zeros(K, dtype=np.uint64)
        self.lib.oracle_cost_with_hash(_p(F), len(F), _p(poses), K, _p(Q), len(Q), _p(c),
                                       h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        return c, h


def pack_bits(b: np.ndarray) -> np.ndarray:
    """Booleans -> little-endian 32-bit words (bit k%32 of word k//32)."""
    b = np.asarray(b, dtype=bool).reshape(-1)
    m = len(b)
    pad = (-m) % 32
    bb = np.concatenate([b, np.zeros(pad, dtype=bool)]) if pad else b
    by = np.packbits(bb, bitorder="little")
    return by.view(np.uint32).copy() if len(by) else np.zeros(0, dtype=np.uint32)


def unpack_bits(words: np.ndarray, m: int) -> np.ndarray:
    """Inverse of :func:`pack_bits`."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint32)).reshape(-1)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:m].astype(bool)
