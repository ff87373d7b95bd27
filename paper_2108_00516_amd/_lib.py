"""ctypes declarations of the C ABI in include/posegraph.h.

Loading fails loudly when libposegraph.so has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libposegraph.so")

PG_OK = 0
PG_ERR_INVALID_ARG = -1
PG_ERR_NO_DEVICE = -2
PG_ERR_OUT_OF_MEMORY = -3
PG_ERR_CAPACITY = -4
PG_ERR_SINGULAR = -5
PG_ERR_NONFINITE = -6
PG_ERR_HIP = -7
STATUS_NAMES = {0: "PG_OK", -1: "PG_ERR_INVALID_ARG", -2: "PG_ERR_NO_DEVICE", -3: "PG_ERR_OUT_OF_MEMORY",
                -4: "PG_ERR_CAPACITY", -5: "PG_ERR_SINGULAR", -6: "PG_ERR_NONFINITE", -7: "PG_ERR_HIP"}

(PG_SOLVER_AUTO, PG_SOLVER_PCG, PG_SOLVER_CHOLESKY, PG_SOLVER_GAUSS_JORDAN, PG_SOLVER_LDL,
 PG_SOLVER_PCG_MATRIX_FREE) = 0, 1, 2, 3, 4, 5
PG_WEIGHT_HUBER, PG_WEIGHT_LEARNED = 0, 1
PG_PREC_FP32, PG_PREC_BF16X3 = 0, 1
PG_MAX_FRAMES_LIMIT = 32
PG_MAX_ITERS = 32


class pg_camera(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class pg_config(C.Structure):
    _fields_ = [("max_frames", C.c_int), ("gn_iters", C.c_int),
                ("lambda_f", C.c_double), ("lambda_g", C.c_double),
                ("huber_f_m", C.c_double), ("huber_g_m", C.c_double),
                ("gate_dist_m", C.c_double), ("gate_normal_rad", C.c_double),
                ("solver", C.c_int), ("pcg_max_iters", C.c_int), ("pcg_rel_tol", C.c_double),
                ("weighting", C.c_int), ("precision", C.c_int), ("use_graph", C.c_int), ("timing", C.c_int),
                ("tile_pixels", C.c_int), ("prune_frac", C.c_double), ("persistent", C.c_int)]


class pg_stats(C.Structure):
    _fields_ = [("iters_done", C.c_int),
                ("energy_f", C.c_double * PG_MAX_ITERS), ("energy_g", C.c_double * PG_MAX_ITERS),
                ("n_valid_g", C.c_longlong * PG_MAX_ITERS), ("n_valid_f", C.c_longlong * PG_MAX_ITERS),
                ("status_bits", C.c_int), ("src_pixels", C.c_longlong), ("n_assoc_launches", C.c_int),
                ("ms_assoc", C.c_float), ("ms_feature", C.c_float), ("ms_reduce", C.c_float),
                ("ms_solve", C.c_float), ("ms_total", C.c_float),
                ("n_target_reads", C.c_longlong * PG_MAX_ITERS), ("pcg_iters", C.c_int * PG_MAX_ITERS)]


# entry point -> (restype, argtypes)
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
SIGNATURES = {
    "pg_config_default": (None, [C.POINTER(pg_config)]),
    "pose_graph_create": (C.c_int, [C.POINTER(pg_config), C.POINTER(pg_camera), _vp, C.POINTER(_vp)]),
    "pose_graph_add_frame": (C.c_int, [_vp, _vp, _vp, _dp, C.c_int, C.POINTER(C.c_int)]),
    "pose_graph_add_matches": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, C.c_int]),
    "pose_graph_set_pose": (C.c_int, [_vp, C.c_int, _dp]),
    "pose_graph_get_pose": (C.c_int, [_vp, C.c_int, _dp]),
    "pose_graph_set_poses": (C.c_int, [_vp, C.c_int, _dp]),
    "pose_graph_optimize": (C.c_int, [_vp, C.POINTER(pg_stats)]),
    "pose_graph_optimize_batch": (C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(pg_stats)]),
    "pose_graph_linearize": (C.c_int, [_vp, _dp, _dp, C.POINTER(pg_stats)]),
    "pose_graph_associate": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_float),
                                       C.POINTER(C.c_float)]),
    "pose_graph_frame_info": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int)]),
    "pose_graph_set_mlp": (C.c_int, [_vp, _vp, C.c_size_t]),
    "pose_graph_pair_features": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp]),
    "pose_graph_prune": (C.c_int, [_vp, _vp, _vp]),
    "pose_graph_time_assoc": (C.c_int, [_vp, C.c_int, _dp]),
    "pg_set_tile_table": (C.c_int, [_vp, C.c_int]),
    "pg_mlp_create": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "pg_mlp_destroy": (None, [_vp]),
    "pg_mlp_set_params": (C.c_int, [_vp, _vp]),
    "pg_mlp_get_params": (C.c_int, [_vp, _vp, _vp]),
    "pg_mlp_loss_grad": (C.c_int, [_vp, _vp, _vp, C.c_int, _dp, _dp]),
    "pg_mlp_adam_step": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, _dp]),
    "pg_mlp_forward": (C.c_int, [_vp, _vp, C.c_int, _vp]),
    "pg_mlp_last_error": (C.c_char_p, [_vp]),
    "pose_graph_num_frames": (C.c_int, [_vp]),
    "pose_graph_last_error": (C.c_char_p, [_vp]),
    "pose_graph_destroy": (None, [_vp]),
    "pg_match_descriptors": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp, _vp, C.c_int, C.c_double, _vp, _vp, _vp,
                                       _vp]),
    "pg_match_descriptors_noalloc": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp, _vp, C.c_int, C.c_double, _vp,
                                               _vp, _vp, _vp]),
    "pg_frontend_last_error": (C.c_char_p, []),
    "pg_select_keyframes": (C.c_int, [_vp, C.c_int, _vp, C.c_int, C.c_double, _vp, _vp, _vp, _vp, _vp]),
    "pose_graph_ransac": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp, C.c_int, _vp, C.c_double, C.c_double,
                                    C.c_int, _vp, _vp, _vp, _vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libposegraph.so and declare its entry points."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch supplies device memory and streams; its HIP runtime has the same
        # soname as the one this library links, so load it first and let the
        # process use a single runtime whatever the import order
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()' or python paper_2108_00516_amd/build.py)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    # the tuned association tiles shipped with the package
    from . import autotune
    table = autotune.load(autotune.TABLE_PATH)
    if table:
        autotune.apply(table, lib)
    return lib
