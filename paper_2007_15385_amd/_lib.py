"""ctypes loader for ``libpip_voronoi.so`` (no torch types cross this layer)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libpip_voronoi.so"

PIP_F32 = 0
PIP_F64 = 1
PIP_OPT_MFMA_MIN_EDGES = 1
PIP_OPT_ALLPAIRS_CULL = 2
PIP_OPT_COST_CULL = 3
PIP_OPT_ALLPAIRS_PAIR = 4
PIP_OPT_COST_PAIR = 5
PIP_OPT_RADIAL_MIN_EDGES = 6
PIP_OPT_EARLY_EXIT = 7
PIP_BATCHED_SCRATCH_BYTES = 32 << 20  # static scratch array of pip_voronoi_batched_noalloc

STATUS_NAMES = {
    0: "PIP_OK", 1: "PIP_EINVAL", 2: "PIP_EDEGENERATE", 3: "PIP_ENONCONVEX", 4: "PIP_EHIP",
    5: "PIP_ENOMEM", 6: "PIP_EUNSUPPORTED",
}


def status_name(s: int) -> str:
    return STATUS_NAMES.get(int(s), f"PIP_UNKNOWN({int(s)})")


class PipError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = int(status)
        super().__init__(f"{where}: {status_name(status)}: {detail}")


def lib_path() -> str:
    return os.environ.get("PIP_VORONOI_LIB", os.path.join(HERE, LIB_NAME))


_c = ctypes
_vp = _c.c_void_p
_i32 = _c.c_int32
_i64 = _c.c_int64
_int = _c.c_int

# name -> (restype, argtypes); pointers are passed as plain integers
SIGNATURES = {
    "pip_version": (_int, []),
    "pip_set_option": (_int, [_vp, _int, _i64]),
    "pip_get_option": (_int, [_vp, _int, _c.POINTER(_i64)]),
    "pip_create": (_int, [_int, _c.POINTER(_vp)]),
    "pip_destroy": (None, [_vp]),
    "pip_status_str": (_c.c_char_p, [_int]),
    "pip_last_error": (_c.c_char_p, [_vp]),
    "polygon_to_generators": (_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "pip_mfma_margin_probe": (_int, [_vp, _vp, _i64, _vp, _vp]),
    "pip_voronoi": (_int, [_vp, _vp, _i32, _vp, _int, _i64, _vp, _vp, _vp]),
    "pip_voronoi_radial_bounds": (_int, [_vp, _vp, _i32, _vp, _vp]),
    "pip_screen_table": (_int, [_vp, _i32, _i32, _vp, _i32, _vp, _vp]),
    "pip_sign_of_offset": (_int, [_vp, _vp, _i32, _vp, _int, _i64, _vp, _vp, _vp]),
    "pip_ray_crossing": (_int, [_vp, _vp, _i32, _vp, _int, _i64, _vp, _vp, _vp]),
    "pip_voronoi_fp32_plain": (_int, [_vp, _vp, _i32, _vp, _int, _i64, _vp, _vp, _vp]),
    "pip_voronoi_max_margin": (_int, [_vp, _vp, _i32, _vp, _int, _i64, _vp, _vp, _vp]),
    "pip_index_create": (_int, [_vp, _i32, _vp, _vp, _i64, _i64, _vp, _vp, _c.POINTER(_vp)]),
    "pip_index_locate": (_int, [_vp, _vp, _i64, _vp, _vp]),
    "pip_index_info": (_int, [_vp, _c.POINTER(_i64), _c.POINTER(_i64)]),
    "pip_index_locate_workspace_bytes": (_c.c_size_t, [_vp, _i64]),
    "pip_index_locate_binned": (_int, [_vp, _vp, _i64, _vp, _vp, _c.c_size_t, _vp]),
    "pip_index_destroy": (None, [_vp]),
    "pip_voronoi_raster": (_int, [_vp, _vp, _i32, _c.c_double, _c.c_double, _c.c_double,
                                  _c.c_double, _i64, _i64, _vp, _vp, _vp]),
    "pip_voronoi_batched_workspace_bytes": (_c.c_size_t, [_i32, _i64, _i64]),
    "pip_voronoi_batched": (_int, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                                   _c.c_size_t, _vp, _vp]),
    "pip_voronoi_batched_noalloc": (_int, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp,
                                           _vp, _vp, _vp]),
    "pip_convex_decompose": (_int, [_vp, _i32, _i32, _vp, _vp, _c.POINTER(_i32), _c.POINTER(_i64)]),
    "pip_voronoi_pieces_workspace_bytes": (_c.c_size_t, [_i32, _i64]),
    "pip_voronoi_pieces": (_int, [_vp, _vp, _i64, _i32, _vp, _vp, _i64, _vp, _int, _i64, _vp, _vp,
                                  _vp, _c.c_size_t, _vp]),
    "pip_plan_create_batched": (_int, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp,
                                       _c.POINTER(_vp)]),
    "pip_plan_autotune": (_int, [_vp, _i32, _vp]),
    "pip_plan_launch": (_int, [_vp, _vp]),
    "pip_plan_config": (_int, [_vp, _vp, _c.POINTER(_c.c_float)]),
    "pip_plan_set_config": (_int, [_vp, _vp]),
    "pip_plan_create_allpairs": (_int, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp,
                                        _c.POINTER(_vp)]),
    "pip_plan_variant": (_int, [_vp, _vp, _c.POINTER(_c.c_float)]),
    "pip_plan_create_cost": (_int, [_vp, _i32, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp,
                                    _vp, _c.POINTER(_vp)]),
    "pip_plan_create": (_int, [_vp, _i32, _vp, _c.POINTER(_vp)]),
    "pip_plan_set_variant": (_int, [_vp, _vp]),
    "pip_plan_destroy": (None, [_vp]),
    "pip_poses_to_polygons": (_int, [_vp, _vp, _i32, _vp, _vp, _i64, _vp, _vp]),
    "pip_voronoi_allpairs_workspace_bytes": (_c.c_size_t, [_i32, _i32]),
    "pip_voronoi_allpairs": (_int, [_vp, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                                    _c.c_size_t, _vp]),
    "pip_voronoi_allpairs_csr_workspace_bytes": (_c.c_size_t, [_i32, _i64]),
    "pip_voronoi_allpairs_csr": (_int, [_vp, _i32, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp,
                                        _c.c_size_t, _vp]),
    "pip_cost_workspace_bytes": (_c.c_size_t, [_i32, _i64, _i64]),
    "pip_cost_fwd": (_int, [_vp, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _c.c_size_t, _vp]),
    "pip_cost_bwd": (_int, [_vp, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                            _c.c_size_t, _vp]),
}


class BatchedConfig(ctypes.Structure):
    _fields_ = [("chunks_per_tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class VariantConfig(ctypes.Structure):
    _fields_ = [("cull", ctypes.c_int32), ("pair", ctypes.c_int32)]


# pip_plan_create: kinds and descriptors (the typed creators' arguments)
PIP_PLAN_BATCHED = 0
PIP_PLAN_ALLPAIRS = 1
PIP_PLAN_COST_FWD = 2
PIP_PLAN_COST_BWD = 3


class BatchedDesc(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("vtx_off", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("total_vertices", ctypes.c_int64), ("pt_off", ctypes.c_void_p),
                ("Q", ctypes.c_void_p), ("total_points", ctypes.c_int64),
                ("lbl_word_off", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class AllpairsDesc(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("n", ctypes.c_int32), ("V", ctypes.c_void_p),
                ("Q", ctypes.c_void_p), ("m", ctypes.c_int64), ("labels", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class CostDesc(ctypes.Structure):
    _fields_ = [("footprint", ctypes.c_void_p), ("n", ctypes.c_int32), ("pose", ctypes.c_void_p),
                ("K", ctypes.c_int64), ("Q", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("cost", ctypes.c_void_p), ("grad_cost", ctypes.c_void_p),
                ("grad_pose", ctypes.c_void_p), ("grad_footprint", ctypes.c_void_p),
                ("residual", ctypes.c_void_p)]

_lock = threading.Lock()
_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load the HIP library (import torch first so that its HIP runtime is
    the one the library binds to).  Raises if the library is missing."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or lib_path()
        if not os.path.exists(p):
            raise ImportError(
                f"{p} not found: build the HIP library first "
                "(python -m paper_2007_15385_amd.build); there is no CPU fallback")
        lib = ctypes.CDLL(p)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if path is None:
            _lib = lib
        return lib


def num_label_words(m: int) -> int:
    return (int(m) + 31) // 32
