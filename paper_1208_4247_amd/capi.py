"""ctypes binding of libgmg.so (the C ABI declared in include/gmg.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmg.so")

GMG_OK = 0
GMG_NOT_CONVERGED = 1
GMG_ERR_INVALID_ARG = -1
GMG_ERR_WORKSPACE = -2
GMG_ERR_NONFINITE = -3
GMG_ERR_DIVERGED = -4
GMG_ERR_HIP = -5
GMG_ERR_UNSUPPORTED = -6

GMG_SMOOTH_RBGS = 0
GMG_SMOOTH_WJ = 1
GMG_SMOOTH_MCGS = 2
GMG_FP64 = 0
GMG_MIXED_FP32_IR = 1
GMG_F64 = 0
GMG_F32 = 1

GMG_USE_GRAPH = 0x1
GMG_AUTOTUNE = 0x2
GMG_PROFILE = 0x4
GMG_POST_FORWARD = 0x8
GMG_NO_TEMPORAL_BLOCKING = 0x10
GMG_NO_FUSED_COARSE = 0x20
GMG_NO_FUSED_RESTRICT = 0x40
GMG_FE_TRANSFER = 0x80
GMG_COARSE_RELAX = 0x100
GMG_NO_CROSS_CYCLE = 0x200
GMG_BATCH_ONE_STREAM = 0x400
GMG_SCRATCH_BYTES = 64 << 20

EXPORTED = [
    "gmg_config_default", "gmg_setup", "gmg_vcycle", "gmg_solve", "gmg_batch_solve",
    "gmg_destroy", "gmg_status_string", "gmg_plan_workspace_bytes", "gmg_level_side",
    "gmg_op_smooth", "gmg_op_restrict_residual", "gmg_op_residual", "gmg_op_prolong_add",
    "gmg_profile_count",
    "gmg_profile_get", "gmg_profile_reset", "gmg_tile_variant_count", "gmg_plan_set_tile",
    "gmg_profile_set_mask", "gmg_plan_get_tile", "gmg_fmg", "gmg_dst_setup", "gmg_dst_solve",
    "gmg_dst_destroy", "gmg_tune_cache_check", "gmg_plan_set_tile_order", "gmg_solve_scratch",
]


class GmgConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("nu1", ctypes.c_int),
        ("nu2", ctypes.c_int),
        ("omega", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("flags", ctypes.c_uint),
    ]


class GmgKernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_longlong),
        ("total_ms", ctypes.c_double),
        ("alg_bytes", ctypes.c_double),
    ]


class GmgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s" % (where, status_string(status)))


_lib = None


def lib():
    """Load libgmg.so (raises if it is missing: build it with
    ``python -m paper_1208_4247_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgmg.so is not built (%s); run python -m paper_1208_4247_amd.build"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    cfgp = ctypes.POINTER(GmgConfig)
    L.gmg_config_default.argtypes = [cfgp, i, i]
    L.gmg_setup.argtypes = [cfgp, i, ip, ip, vp, ctypes.POINTER(sz), vp, ctypes.POINTER(vp)]
    L.gmg_vcycle.argtypes = [vp, vp, vp]
    L.gmg_fmg.argtypes = [vp, vp, vp]
    L.gmg_solve.argtypes = [vp, vp, vp, d, i, dp, ip, dp]
    L.gmg_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), d, i, ip, dp, ip]
    L.gmg_destroy.argtypes = [vp]
    L.gmg_status_string.argtypes = [i]
    L.gmg_status_string.restype = ctypes.c_char_p
    L.gmg_plan_workspace_bytes.argtypes = [vp]
    L.gmg_plan_workspace_bytes.restype = sz
    L.gmg_level_side.argtypes = [vp, i, i]
    L.gmg_op_smooth.argtypes = [vp, i, i, i, i, vp, vp, vp, vp, dp]
    L.gmg_op_restrict_residual.argtypes = [vp, i, i, vp, vp, vp]
    L.gmg_op_residual.argtypes = [vp, i, i, vp, vp, vp, dp]
    L.gmg_op_prolong_add.argtypes = [vp, i, i, vp, vp, vp]
    L.gmg_dst_setup.argtypes = [i, i, vp, ctypes.POINTER(sz), vp, ctypes.POINTER(vp)]
    L.gmg_dst_solve.argtypes = [vp, vp, vp]
    L.gmg_dst_destroy.argtypes = [vp]
    L.gmg_profile_count.argtypes = [vp]
    L.gmg_profile_get.argtypes = [vp, i, ctypes.POINTER(GmgKernelStat)]
    L.gmg_profile_reset.argtypes = [vp]
    L.gmg_tile_variant_count.argtypes = [i, i, i]
    L.gmg_plan_set_tile.argtypes = [vp, i, i, i, i]
    L.gmg_profile_set_mask.argtypes = [vp, ctypes.c_uint]
    ip = ctypes.POINTER(ctypes.c_int)
    L.gmg_plan_get_tile.argtypes = [vp, i, i, ip, ip, ip]
    L.gmg_tune_cache_check.argtypes = [ctypes.c_char_p, ip, ip]
    L.gmg_plan_set_tile_order.argtypes = [vp, i, i, i]
    L.gmg_solve_scratch.argtypes = [cfgp, vp, vp, d, i, dp, ip, dp, vp]
    for name in EXPORTED:
        if name not in ("gmg_status_string", "gmg_plan_workspace_bytes", "gmg_level_side",
                        "gmg_profile_count", "gmg_tile_variant_count"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().gmg_status_string(int(s)).decode()


def check(s: int, where: str) -> int:
    if s < 0:
        raise GmgError(s, where)
    return s


def tune_cache_check(path: str) -> tuple[int, int]:
    """(usable, skipped) line counts of an autotuner cache file."""
    nv, ni = ctypes.c_int(0), ctypes.c_int(0)
    check(lib().gmg_tune_cache_check(path.encode(), ctypes.byref(nv), ctypes.byref(ni)),
          "gmg_tune_cache_check")
    return nv.value, ni.value


def config_default(dim: int, levels: int) -> GmgConfig:
    c = GmgConfig()
    lib().gmg_config_default(ctypes.byref(c), int(dim), int(levels))
    return c


def workspace_bytes(cfg: GmgConfig, nproblems: int = 1, dims=None, levels=None) -> tuple[int, int]:
    """(status, bytes) of the two-phase setup's size query."""
    n = ctypes.c_size_t(0)
    da = (ctypes.c_int * len(dims))(*dims) if dims is not None else None
    la = (ctypes.c_int * len(levels))(*levels) if levels is not None else None
    s = lib().gmg_setup(ctypes.byref(cfg), int(nproblems), da, la, None, ctypes.byref(n), None,
                        None)
    return s, n.value
