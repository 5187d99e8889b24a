"""Python binding of the MI355X point-inclusion library (``libpip_voronoi.so``).

Argument marshalling only: every function takes torch tensors that already
live on a ROCm device, checks their dtype/shape/contiguity, and passes the
raw device pointers plus the current HIP stream to the C ABI declared in
``include/pip_voronoi.h``.  Every step of every test runs in the library's
HIP kernels; there is no CPU fallback.  If the library has not been built,
or no GPU is present, the calls raise.

The functions carry the C names: :func:`polygon_to_generators`,
:func:`pip_voronoi`, :func:`pip_sign_of_offset`, :func:`pip_ray_crossing`,
:func:`pip_voronoi_fp32_plain`, :func:`pip_voronoi_max_margin`.
"""
from __future__ import annotations

from ._lib import (PIP_BATCHED_SCRATCH_BYTES, PIP_F32, PIP_F64, PIP_OPT_ALLPAIRS_CULL, PIP_OPT_ALLPAIRS_PAIR, PIP_OPT_COST_CULL, PIP_OPT_COST_PAIR, PIP_OPT_MFMA_MIN_EDGES, PIP_OPT_RADIAL_MIN_EDGES, PIP_OPT_EARLY_EXIT, PipError, lib_path, load_library,
                   num_label_words, status_name, PIP_PLAN_BATCHED, PIP_PLAN_ALLPAIRS,
                   PIP_PLAN_COST_FWD, PIP_PLAN_COST_BWD, BatchedDesc, AllpairsDesc, CostDesc)
from .api import get_option, set_option, pip_plan_create
from .api import (AllpairsPlan, BatchedPlan, LocateIndex, allpairs_workspace_bytes, batched_workspace_bytes,
                  convex_decompose, pieces_workspace_bytes, pip_voronoi_pieces,
                  allpairs_csr_workspace_bytes, pip_voronoi_allpairs_csr, pip_mfma_margin_probe, label_word_offsets, pip_poses_to_polygons,
                  pip_ray_crossing, pip_sign_of_offset, pip_voronoi, pip_voronoi_allpairs,
                  pip_voronoi_batched, pip_voronoi_batched_noalloc, pip_voronoi_fp32_plain, pip_voronoi_max_margin, pip_voronoi_radial_bounds, pip_voronoi_raster,
                  pip_screen_table,
                  polygon_to_generators, unpack_labels)
from .autograd import CollisionCost, CostPlan, collision_cost, pip_cost_bwd, pip_cost_fwd

__all__ = [
    "PIP_F32", "PIP_F64", "PipError", "lib_path", "load_library", "num_label_words",
    "status_name", "polygon_to_generators", "pip_voronoi", "pip_sign_of_offset",
    "pip_ray_crossing", "pip_voronoi_fp32_plain", "pip_voronoi_max_margin", "pip_voronoi_radial_bounds", "pip_voronoi_raster", "unpack_labels",
    "pip_screen_table",
    "pip_voronoi_batched", "pip_voronoi_batched_noalloc", "PIP_BATCHED_SCRATCH_BYTES",
    "batched_workspace_bytes", "label_word_offsets", "BatchedPlan",
    "LocateIndex", "AllpairsPlan", "convex_decompose", "pieces_workspace_bytes",
    "pip_voronoi_pieces", "allpairs_csr_workspace_bytes", "pip_voronoi_allpairs_csr", "pip_mfma_margin_probe",
    "pip_poses_to_polygons", "pip_voronoi_allpairs", "allpairs_workspace_bytes", "pip_cost_fwd", "pip_cost_bwd",
    "CollisionCost", "CostPlan", "collision_cost", "PIP_OPT_MFMA_MIN_EDGES", "PIP_OPT_ALLPAIRS_CULL", "PIP_OPT_ALLPAIRS_PAIR", "PIP_OPT_COST_CULL", "PIP_OPT_COST_PAIR", "PIP_OPT_RADIAL_MIN_EDGES", "PIP_OPT_EARLY_EXIT", "set_option", "get_option",
    "pip_plan_create", "PIP_PLAN_BATCHED", "PIP_PLAN_ALLPAIRS", "PIP_PLAN_COST_FWD",
    "PIP_PLAN_COST_BWD", "BatchedDesc", "AllpairsDesc", "CostDesc",
]
