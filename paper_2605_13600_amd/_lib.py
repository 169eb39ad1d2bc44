"""ctypes declarations of the libscoup C ABI (include/scoup.h); marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscoup.so")

OK, E_ARG, E_WORKSPACE, E_HIP, E_UNSUPPORTED, E_DATA = 0, -1, -2, -3, -4, -5
F32, BF16, FP8_E4M3 = 0, 1, 2


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacities", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("near_z", C.c_float)]


class Views(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("cams", C.POINTER(Camera)), ("region_maps", C.c_void_p),
                ("map_offsets", C.POINTER(C.c_int64)), ("region_base", C.POINTER(C.c_int64)),
                ("code_idx", C.c_void_p), ("code_val", C.c_void_p), ("k_code", C.c_int32),
                ("m_atoms", C.c_int32)]


# every exported symbol of include/scoup.h with its signature
SIGNATURES = {
    "scoup_uplift_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Views), C.c_int64, C.c_int32]),
    "scoup_required_pair_capacity": (C.c_int64, []),
    "scoup_uplift_accumulate": (C.c_int, [C.POINTER(Gaussians), C.POINTER(Views), C.c_void_p, C.c_int32,
                                          C.c_int64, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                          C.c_void_p]),
    "scoup_uplift_levels_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int32, C.POINTER(Views), C.c_int64,
                                                         C.c_int32]),
    "scoup_uplift_levels": (C.c_int, [C.POINTER(Gaussians), C.c_int32, C.POINTER(Views), C.c_int32,
                                      C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_void_p), C.c_int64, C.c_int32, C.c_void_p, C.c_size_t,
                                      C.c_void_p, C.c_void_p]),
    "scoup_uplift_dense_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Views), C.c_int32, C.c_int64,
                                                        C.c_int32]),
    "scoup_uplift_dense": (C.c_int, [C.POINTER(Gaussians), C.POINTER(Views), C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.c_void_p]),
    "scoup_entropy": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]),
    "scoup_topk": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    "scoup_uplift": (C.c_int, [C.POINTER(Gaussians), C.POINTER(Views), C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                               C.c_void_p]),
    "scoup_render_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Camera), C.c_int64]),
    "scoup_render_coeff": (C.c_int, [C.POINTER(Gaussians), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                     C.POINTER(Camera), C.c_void_p, C.c_int, C.c_float, C.c_void_p,
                                     C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "scoup_render_decode_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Camera), C.c_int32, C.c_int32,
                                                         C.c_int, C.c_int64]),
    "scoup_render": (C.c_int, [C.POINTER(Gaussians), C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Camera),
                               C.c_void_p, C.c_int32, C.c_int32, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "scoup_render_views_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Camera), C.c_int32, C.c_int32,
                                                        C.c_int32, C.c_int, C.c_int64]),
    "scoup_render_views": (C.c_int, [C.POINTER(Gaussians), C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Camera),
                                     C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int, C.c_void_p, C.c_int,
                                     C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "scoup_decode_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int]),
    "scoup_decode": (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_int64, C.c_int32, C.c_void_p, C.c_int32,
                               C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "scoup_decode_noalloc_max_bytes": (C.c_size_t, []),
    "scoup_decode_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_int64, C.c_int32, C.c_void_p,
                                       C.c_int32, C.c_void_p, C.c_int, C.c_void_p]),
    "scoup_relevancy_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int]),
    "scoup_relevancy": (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_int64, C.c_int32, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_float, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
    "scoup_render_backward_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Camera), C.c_int32, C.c_int32,
                                                           C.c_int64]),
    "scoup_render_backward": (C.c_int, [C.POINTER(Gaussians), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(Camera), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "scoup_stage_timing": (None, [C.c_int32]),
    "scoup_stage_stats": (C.c_int32, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "scoup_set_views_in_flight": (None, [C.c_int32]),
    "scoup_views_in_flight": (C.c_int32, []),
    "scoup_set_deferred_entry_limit": (None, [C.c_int64]),
    "scoup_uplift_touch_stats": (None, [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64)]),
    "scoup_last_error": (C.c_char_p, []),
    "scoup_version": (C.c_char_p, []),
}

_lib = None


def load() -> C.CDLL:
    """Load libscoup.so (once).  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
