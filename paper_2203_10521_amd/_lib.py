"""ctypes loader of libobbv.so and the C structs of include/obbv.h.

torch is imported first so that its HIP runtime (libamdhip64) is the one the
library binds to: device pointers and streams from torch are then valid
arguments.  A missing library raises; there is no fallback path.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libobbv.so")

c_int32 = ctypes.c_int32
c_uint32 = ctypes.c_uint32
c_uint64 = ctypes.c_uint64
c_void_p = ctypes.c_void_p
c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_uint32_p = ctypes.POINTER(ctypes.c_uint32)


class ObbvMesh(ctypes.Structure):
    _fields_ = [("vertices", c_void_p), ("triangles", c_void_p),
                ("n_vertices", c_int32), ("n_triangles", c_int32)]


class ObbvOvParams(ctypes.Structure):
    _fields_ = [("R", c_int32), ("axis_mask", c_uint32), ("seed", c_uint64),
                ("block_rays", c_int32), ("flags", c_uint32)]


class ObbvLloydParams(ctypes.Structure):
    _fields_ = [("R", c_int32), ("block_rays", c_int32), ("seed", c_uint64), ("pops_per_round", c_int32),
                ("reserved", c_int32), ("delta", ctypes.c_double)]


class ObbvSurrogate(ctypes.Structure):
    _fields_ = [("mlp_params", c_void_p), ("volume", c_void_p), ("frame", c_void_p), ("N", c_int32),
                ("verify_top", c_int32), ("max_error", ctypes.c_float), ("judge_every", c_int32)]


class ObbvHierParams(ctypes.Structure):
    _fields_ = [("levels", c_int32), ("branching", c_int32), ("iters", c_int32), ("sweeps", c_int32),
                ("R", c_int32), ("block_rays", c_int32), ("pops_per_round", c_int32), ("reserved", c_int32),
                ("seed", c_uint64), ("delta", ctypes.c_double), ("surrogate", ctypes.POINTER(ObbvSurrogate))]


# name -> (restype, argtypes); every symbol declared in include/obbv.h
SIGNATURES = {
    "obbv_version": (ctypes.c_char_p, []),
    "obbv_last_error": (ctypes.c_char_p, []),
    "obbv_status": (c_int32, [c_void_p, c_uint32_p]),
    "obbv_release": (c_int32, []),
    "obbv_validate_mesh": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32_p, c_double_p, c_void_p]),
    "obbv_outer_volume": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_void_p, c_void_p, c_void_p,
                                    c_int32, ctypes.POINTER(ObbvOvParams), c_void_p, c_void_p]),
    "obbv_outer_volume_ex": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_void_p, c_void_p, c_void_p,
                                       c_int32, ctypes.POINTER(ObbvOvParams), c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
    "obbv_outer_volume_grouped": (c_int32, [ctypes.POINTER(ObbvMesh), c_void_p, c_void_p, c_int32,
                                            ctypes.POINTER(ObbvOvParams), c_void_p, c_void_p, c_int32, c_void_p,
                                            c_void_p]),
    "obbv_outer_volume_noalloc": (c_int32, [ctypes.POINTER(ObbvMesh), c_void_p, c_void_p, c_int32,
                                            ctypes.POINTER(ObbvOvParams), c_void_p, c_void_p, c_void_p]),
    "obbv_ov_plan_create": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                      ctypes.POINTER(ObbvOvParams), c_void_p, ctypes.c_double, c_void_p,
                                      ctypes.POINTER(c_void_p)]),
    "obbv_ov_plan_launch": (c_int32, [c_void_p, c_void_p]),
    "obbv_ov_plan_info": (c_int32, [c_void_p, c_int32_p, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_float)]),
    "obbv_ov_plan_destroy": (c_int32, [c_void_p]),
    "obbv_profile_enable": (c_int32, [c_int32]),
    "obbv_collision_queries": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                         c_void_p, c_void_p]),
    "obbv_outer_volume_central": (c_int32, [ctypes.POINTER(ObbvMesh), c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "obbv_outer_volume_exact": (c_int32, [ctypes.POINTER(ObbvMesh), c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "obbv_profile_read": (c_int32, [c_double_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64), c_double_p]),
    "obbv_fit": (c_int32, [ctypes.POINTER(ObbvMesh), c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "obbv_box_features": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                    c_uint64, c_void_p, c_void_p]),
    "obbv_occupancy_volume": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_void_p, c_uint64, c_void_p, c_void_p]),
    "obbv_sample_features": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "obbv_mlp_param_count": (ctypes.c_int64, []),
    "obbv_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "obbv_mlp_rank_boxes": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "obbv_mlp_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_int32,
                                      ctypes.c_float, c_void_p, c_void_p, c_void_p]),
    "obbv_lloyd_create": (c_int32, [ctypes.POINTER(ObbvMesh), ctypes.POINTER(ObbvLloydParams),
                                    ctypes.POINTER(c_void_p)]),
    "obbv_lloyd_set_groups": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "obbv_lloyd_step": (c_int32, [c_void_p, c_void_p]),
    "obbv_lloyd_adjust": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "obbv_lloyd_set_surrogate": (c_int32, [c_void_p, ctypes.POINTER(ObbvSurrogate)]),
    "obbv_lloyd_get": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double_p,
                                 ctypes.POINTER(ctypes.c_int64)]),
    "obbv_lloyd_record": (c_int32, [c_void_p, ctypes.c_int64]),
    "obbv_lloyd_take_records": (c_int32, [c_void_p, ctypes.c_int64, c_void_p, c_void_p,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "obbv_lloyd_destroy": (c_int32, [c_void_p]),
    "obbv_build_obb_tree": (c_int32, [ctypes.POINTER(ObbvMesh), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                      c_void_p]),
    "obbv_build_hierarchy": (c_int32, [ctypes.POINTER(ObbvMesh), ctypes.POINTER(ObbvHierParams), c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_10521_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
