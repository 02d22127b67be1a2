"""ctypes loader for libradonlp.so: argument marshalling only.

Every declaration mirrors include/radonlp.h.  Loading the library touches no device.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libradonlp.so")

RL_OK = 0
RL_ERR_INVALID_ARG, RL_ERR_GEOMETRY, RL_ERR_WORKSPACE, RL_ERR_HIP = 1, 2, 3, 4
STATUS_NAMES = {
    0: "RL_OK",
    1: "RL_ERR_INVALID_ARG",
    2: "RL_ERR_GEOMETRY",
    3: "RL_ERR_WORKSPACE",
    4: "RL_ERR_HIP",
    5: "RL_ERR_UNSUPPORTED_ARCH",
    6: "RL_ERR_INTERNAL",
}
RL_OP_FWD, RL_OP_ADJ, RL_OP_FBP, RL_OP_EM, RL_OP_BP_LP, RL_OP_FBP_LP = 0, 1, 2, 3, 4, 5
RL_FILTER_RAMLAK = 0
RL_FILTER_COSINE = 1
RL_FILTER_SHEPP_LOGAN = 2
FILTERS = {"ramlak": RL_FILTER_RAMLAK, "cosine": RL_FILTER_COSINE, "shepp-logan": RL_FILTER_SHEPP_LOGAN}
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024  # RL_NOALLOC_SCRATCH_BYTES
RL_STAGE_PREFILTER, RL_STAGE_LOGPOLAR, RL_STAGE_CONV, RL_STAGE_KERNEL = 0, 1, 2, 3

# Every function declared in include/radonlp.h.
EXPORTED = (
    "rl_geom_default",
    "rl_plan_create",
    "rl_plan_destroy",
    "rl_plan_geometry",
    "rl_plan_rows",
    "rl_plan_get_tuning",
    "rl_plan_set_tuning",
    "rl_tune_workspace_bytes",
    "rl_plan_autotune",
    "rl_workspace_bytes",
    "rl_plan_samples",
    "radon_fwd",
    "radon_adj",
    "radon_transpose",
    "radon_adj_transpose",
    "radon_fwd_noalloc",
    "fbp",
    "radon_bp_lp",
    "fbp_lp",
    "rl_last_error",
    "rl_debug_stage",
    "rl_profile_start",
    "rl_profile_stop",
    "rl_profile_count",
    "rl_profile_record",
    "rl_batch_create",
    "rl_batch_workspace_bytes",
    "rl_batch_fwd",
    "rl_batch_adj",
    "rl_batch_bp_lp",
    "rl_batch_destroy",
    "rl_em_norm",
    "rl_em",
)


class RlGeom(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("n_theta", ctypes.c_int32),
        ("n_s", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("n_rho", ctypes.c_int32),
        ("k_theta", ctypes.c_int32),
        ("r_dec", ctypes.c_int32),
        ("dec_filter", ctypes.c_int32),
        ("q_theta", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class RlTune(ctypes.Structure):
    _fields_ = [
        ("theta_cols", ctypes.c_int32),
        ("theta_xcd_order", ctypes.c_int32),
        ("prefilter_rows", ctypes.c_int32),
        ("fwd_patch_split", ctypes.c_int32),
        ("fwd_xcd_order", ctypes.c_int32),
        ("adj_walk", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class RadonLibError(RuntimeError):
    def __init__(self, func, status, message):
        super().__init__(f"{func} failed with {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libradonlp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: the HIP library has not been built "
            "(run `python -m paper_1506_00014_amd.build`)"
        )
    lib = ctypes.CDLL(path)
    c_int32, c_size_t, c_void_p = ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p
    lib.rl_geom_default.argtypes = [c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, ctypes.POINTER(RlGeom)]
    lib.rl_geom_default.restype = c_int32
    lib.rl_plan_create.argtypes = [ctypes.POINTER(RlGeom), ctypes.POINTER(c_void_p)]
    lib.rl_plan_create.restype = c_int32
    lib.rl_plan_destroy.argtypes = [c_void_p]
    lib.rl_plan_destroy.restype = None
    lib.rl_plan_geometry.argtypes = [c_void_p, ctypes.POINTER(RlGeom)]
    lib.rl_plan_geometry.restype = c_int32
    lib.rl_workspace_bytes.argtypes = [c_void_p, c_int32, c_int32]
    lib.rl_workspace_bytes.restype = c_size_t
    lib.rl_plan_samples.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.rl_plan_samples.restype = c_int32
    lib.rl_plan_rows.argtypes = [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]
    lib.rl_plan_rows.restype = c_int32
    lib.rl_plan_get_tuning.argtypes = [c_void_p, ctypes.POINTER(RlTune)]
    lib.rl_plan_get_tuning.restype = c_int32
    lib.rl_plan_set_tuning.argtypes = [c_void_p, ctypes.POINTER(RlTune)]
    lib.rl_plan_set_tuning.restype = c_int32
    lib.rl_tune_workspace_bytes.argtypes = [c_void_p, c_int32]
    lib.rl_tune_workspace_bytes.restype = c_size_t
    lib.rl_plan_autotune.argtypes = [c_void_p, c_int32, c_void_p, c_size_t, c_void_p, ctypes.c_char_p]
    lib.rl_plan_autotune.restype = c_int32
    for name in ("radon_fwd", "radon_adj", "radon_transpose", "radon_adj_transpose", "radon_bp_lp"):
        f = getattr(lib, name)
        f.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]
        f.restype = c_int32
    lib.radon_fwd_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.radon_fwd_noalloc.restype = c_int32
    for name in ("fbp", "fbp_lp"):
        f = getattr(lib, name)
        f.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_size_t, c_void_p]
        f.restype = c_int32
    lib.rl_last_error.argtypes = []
    lib.rl_last_error.restype = ctypes.c_char_p
    lib.rl_debug_stage.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]
    lib.rl_debug_stage.restype = c_int32
    lib.rl_profile_start.argtypes = [c_int32]
    lib.rl_profile_start.restype = c_int32
    lib.rl_profile_stop.argtypes = []
    lib.rl_profile_stop.restype = c_int32
    lib.rl_profile_count.argtypes = []
    lib.rl_profile_count.restype = c_int32
    lib.rl_profile_record.argtypes = [c_int32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float)]
    lib.rl_profile_record.restype = c_int32
    lib.rl_batch_create.argtypes = [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(c_int32),
                                    ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int32, ctypes.c_char_p,
                                    ctypes.POINTER(c_void_p)]
    lib.rl_batch_create.restype = c_int32
    lib.rl_batch_workspace_bytes.argtypes = [c_void_p, c_int32]
    lib.rl_batch_workspace_bytes.restype = c_size_t
    for name in ("rl_batch_fwd", "rl_batch_adj", "rl_batch_bp_lp"):
        f = getattr(lib, name)
        f.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
        f.restype = c_int32
    lib.rl_batch_destroy.argtypes = [c_void_p]
    lib.rl_batch_destroy.restype = None
    lib.rl_em_norm.argtypes = [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.rl_em_norm.restype = c_int32
    lib.rl_em.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_size_t, c_void_p]
    lib.rl_em.restype = c_int32
    _lib = lib
    return lib


def check(func: str, status: int):
    if status != RL_OK:
        msg = _lib.rl_last_error().decode() if _lib is not None else ""
        raise RadonLibError(func, status, msg)


def geom_default(n, n_theta, n_s, m=4, q_theta=1, smooth=0) -> RlGeom:
    lib = load()
    g = RlGeom()
    check("rl_geom_default", lib.rl_geom_default(n, n_theta, n_s, m, q_theta, smooth, ctypes.byref(g)))
    return g
