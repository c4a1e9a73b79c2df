"""ctypes declarations of the C ABI in include/hgmm.h (marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgmm.so")

P = C.c_void_p
I64 = C.c_int64
D = C.c_double


class BuildParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("build_iters", C.c_int32), ("reg_eps", D), ("min_mass", D)]


class Tuning(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("block64_max", "block256_max", "block512_max", "min_tile", "target_tiles",
                                          "max_tile", "reg_tile", "reg_chunk", "reg_graph", "reg_sort", "tile_threads", "reg_lds_levels",
                                          "build_graph", "reg_atomics", "fold_tiles")]


class RegParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("max_levels", C.c_int32), ("lambda_c", D), ("tol_rot", D),
                ("tol_trans_rel", D)]


class TreeHost(C.Structure):
    _fields_ = [("levels", C.c_int32), ("pad_", C.c_int32), ("n_points", I64), ("origin", D * 3), ("extent", D),
                ("live", P), ("has_children", P), ("count", P), ("pi", P), ("pig", P), ("mu", P), ("cov", P),
                ("lam", P), ("evec", P), ("kappa", P)]


# name -> (restype, argtypes)
SIGNATURES = {
    "hgmm_last_error": (C.c_char_p, []),
    "hgmm_params_default": (C.c_int, [P, P]),
    "hgmm_tree_nodes": (I64, [C.c_int]),
    "hgmm_level_offset": (I64, [C.c_int]),
    "hgmm_build_graph_stats": (C.c_int, [P, P, P, P]),
    "hgmm_build_workspace_bytes": (C.c_size_t, [I64, C.c_int]),
    "hgmm_register_workspace_bytes": (C.c_size_t, [I64, C.c_int]),
    "hgmm_build": (C.c_int, [P, I64, P, P, C.c_size_t, P, P]),
    "hgmm_register": (C.c_int, [P, P, I64, P, P, P, P, C.c_size_t, P, P, P, P, P]),
    "hgmm_estep": (C.c_int, [P, P, I64, P, P, D, P, C.c_size_t, P, P, P, P, P]),
    "hgmm_noalloc_scratch_bytes": (C.c_size_t, []),
    "hgmm_register_noalloc": (C.c_int, [P, P, I64, P, P, P, P, P, P, P, P]),
    "hgmm_register_flat": (C.c_int, [P, P, I64, C.c_int, P, P, P, P, C.c_size_t, P, P, P, P, P]),
    "hgmm_estep_flat": (C.c_int, [P, P, I64, C.c_int, P, P, P, C.c_size_t, P, P, P, P, P]),
    "hgmm_register_soft": (C.c_int, [P, P, I64, D, P, P, P, P, C.c_size_t, P, P, P, P, P]),
    "hgmm_point_loglik": (C.c_int, [P, P, I64, P, P, D, P, C.c_size_t, P, P, P]),
    "hgmm_estep_soft": (C.c_int, [P, P, I64, D, P, P, D, P, C.c_size_t, P, P, P, P]),
    "hgmm_normal_equations": (C.c_int, [P, P, I64, P, C.c_size_t, P, P, P]),
    "hgmm_tree_export": (C.c_int, [P, C.c_int, P]),
    "hgmm_tree_labels": (C.c_int, [P, C.c_int, P, P]),
    "hgmm_tree_import": (C.c_int, [P, P, P]),
    "hgmm_tree_info": (C.c_int, [P, C.c_int, P, P, P, P]),
    "hgmm_tree_destroy": (None, [P]),
    "hgmm_set_tuning": (C.c_int, [P]),
    "hgmm_get_tuning": (C.c_int, [P]),
    "hgmm_autotune_workspace_bytes": (C.c_size_t, [P, P, P, C.c_int]),
    "hgmm_autotune": (C.c_int, [P, P, P, C.c_int, P, P, P, P, P, C.c_size_t, P, C.c_int, C.c_int, P, P, P]),
    "hgmm_build_batch_workspace_bytes": (C.c_size_t, [P, P, C.c_int]),
    "hgmm_build_batch": (C.c_int, [P, P, P, C.c_int, P, P, C.c_size_t, P, P]),
    "hgmm_register_batch_workspace_bytes": (C.c_size_t, [P, P, C.c_int]),
    "hgmm_register_batch": (C.c_int, [P, P, P, C.c_int, P, P, P, P, P, C.c_size_t, P, P, P, P, P, P]),
    "hgmm_register_warm_batch": (C.c_int, [P, P, P, C.c_int, P, C.c_int, C.c_int, P, P, P, C.c_size_t, P, P, P, P, P,
                                           P, P]),
    "hgmm_odometry_workspace_bytes": (C.c_size_t, [P, C.c_int, C.c_int]),
    "hgmm_odometry": (C.c_int, [P, P, C.c_int, P, P, P, P, C.c_int, P, C.c_size_t, P, P, P, P, P, P, P, P]),
    "hgmm_estep_batch": (C.c_int, [P, P, P, C.c_int, P, P, D, P, C.c_size_t, P, P, P]),
    "hgmm_mlp_param_count": (I64, []),
    "hgmm_mlp_create": (C.c_int, [C.c_uint64, P]),
    "hgmm_mlp_destroy": (None, [P]),
    "hgmm_mlp_get_params": (C.c_int, [P, P]),
    "hgmm_mlp_set_params": (C.c_int, [P, P]),
    "hgmm_mlp_forward": (C.c_int, [P, P, C.c_int, P, P]),
    "hgmm_mlp_train_step": (C.c_int, [P, P, P, C.c_int, C.c_float, C.c_float, P, P]),
    "hgmm_mlp_backward": (C.c_int, [P, P, P, C.c_int, C.c_float, P, P, P]),
    "hgmm_warm_features": (C.c_int, [P, P, C.c_int, D, P, P, P]),
    "hgmm_warm_head_pose": (C.c_int, [P, P, P, C.c_int, P, P, P]),
    "hgmm_warm_head_target": (C.c_int, [P, P, P, P, C.c_int, P, P]),
    "hgmm_gemm_bf16": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, C.c_int, P, C.c_int, P,
                                 C.c_int, P]),
    "hgmm_profile": (C.c_int, [C.c_int]),
    "hgmm_profile_reset": (None, []),
    "hgmm_profile_read": (C.c_int, [C.c_int, P, P, P]),
    "hgmm_profile_work": (C.c_int, [C.c_int, P, P]),
}

_lib = None


def load() -> C.CDLL:
    """Load libhgmm.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(the library has no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if not hasattr(lib, name):
                continue
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error() -> str:
    return load().hgmm_last_error().decode(errors="replace")


class HgmmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with status {code}: {last_error()}")
        self.code = code


def check(code: int, what: str) -> int:
    if code != 0:
        raise HgmmError(code, what)
    return code
