"""ctypes declarations of librpca_mi355x.so (the C ABI in include/rpca.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpca_mi355x.so")

RPCA_OK = 0
RPCA_NOT_CONVERGED = 1
RPCA_ERR_ARG = -1
RPCA_ERR_NOMEM = -2
RPCA_ERR_DEVICE = -3
RPCA_ERR_NONFINITE = -4
RPCA_ERR_UNSUPPORTED = -5
RPCA_ERR_TIMEOUT = -6
RPCA_F64 = 0
RPCA_F32 = 1
RPCA_GRAM_DEFAULT = 0
RPCA_GRAM_BF16X3 = 1
RPCA_GRAM_BF16X6 = 2
RPCA_N_MAX = 144
RPCA_N_MAX_F64 = 128
RPCA_KNOB_EIG_THREADS = 1
RPCA_KNOB_STREAM_KERNEL = 2
RPCA_KNOB_TILE_ROWS = 3
RPCA_KNOB_REG_TILES = 4
RPCA_SERVER_SIMULATE = 1
RPCA_SERVER_STAGE_INIT = 1
RPCA_NOALLOC_MAX_BYTES = 192 << 20

EXPORTS = (
    "rpca_solve_f64", "rpca_solve_f32", "rpca_solve_many", "rpca_solve_ex", "rpca_solve_noalloc",
    "rpca_footprint_bytes", "rpca_strerror", "rpca_version",
    "rpca_profile_enable", "rpca_profile_read", "rpca_last_error",
    "rpca_tune_set", "rpca_tune_get",
    "rpca_server_create", "rpca_server_submit", "rpca_server_step", "rpca_server_pending",
    "rpca_server_peak_bytes", "rpca_server_request_bytes", "rpca_server_destroy",
    "rpca_server_set_timeout", "rpca_server_inject_failure",
    "rpca_autotune", "rpca_autotune_save", "rpca_autotune_load",
    "rpca_frame_correlation", "rpca_frame_keep", "rpca_frame_select", "rpca_moving_average",
    "rpca_dice", "rpca_rmse", "rpca_masked_mean",
)


class RpcaProblem(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lam", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int32),
        ("L", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("iterations", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("residual", ctypes.c_double),
        ("S0", ctypes.c_void_p),
        ("Y0", ctypes.c_void_p),
        ("Y", ctypes.c_void_p),
    ]


class RpcaProfile(ctypes.Structure):
    _fields_ = [
        ("init_ms", ctypes.c_double),
        ("eig_ms", ctypes.c_double),
        ("update_ms", ctypes.c_double),
        ("finalize_ms", ctypes.c_double),
        ("eig_launches", ctypes.c_int64),
        ("update_launches", ctypes.c_int64),
        ("update_bytes", ctypes.c_double),
        ("solves", ctypes.c_int64),
        ("iterations", ctypes.c_int64),
    ]


class RpcaCompletion(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("residual", ctypes.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library once; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own copy of the HIP runtime under the same soname.  Load
    # torch first so the library binds to that one runtime instead of bringing
    # a second copy into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(
            f"librpca_mi355x.so not found at {path}; build it with "
            "`python -m paper_2506_10257_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    for name in ("rpca_solve_f64", "rpca_solve_f32"):
        f = getattr(lib, name)
        f.argtypes = [vp, i64, i64, dbl, dbl, dbl, i32, vp, vp, ctypes.POINTER(i32), vp]
        f.restype = ctypes.c_int
    lib.rpca_solve_noalloc.argtypes = [vp, i64, i64, i32, dbl, dbl, dbl, i32, vp, vp,
                                        ctypes.POINTER(i32), vp]
    lib.rpca_solve_noalloc.restype = ctypes.c_int
    lib.rpca_solve_many.argtypes = [ctypes.POINTER(RpcaProblem), i32, i32, i32, vp]
    lib.rpca_solve_many.restype = ctypes.c_int
    lib.rpca_solve_ex.argtypes = [ctypes.POINTER(RpcaProblem), i32, i32, vp]
    lib.rpca_solve_ex.restype = ctypes.c_int
    lib.rpca_footprint_bytes.argtypes = [i64, i64, i32]
    lib.rpca_footprint_bytes.restype = ctypes.c_size_t
    lib.rpca_strerror.argtypes = [ctypes.c_int]
    lib.rpca_strerror.restype = ctypes.c_char_p
    lib.rpca_last_error.argtypes = []
    lib.rpca_last_error.restype = ctypes.c_char_p
    lib.rpca_version.argtypes = []
    lib.rpca_version.restype = ctypes.c_char_p
    lib.rpca_profile_enable.argtypes = [ctypes.c_int]
    lib.rpca_profile_enable.restype = None
    lib.rpca_profile_read.argtypes = [ctypes.POINTER(RpcaProfile), ctypes.c_int]
    lib.rpca_profile_read.restype = ctypes.c_int
    lib.rpca_tune_set.argtypes = [i32, i32, i32, i32]
    lib.rpca_tune_set.restype = ctypes.c_int
    lib.rpca_tune_get.argtypes = [i32, i32, i32]
    lib.rpca_tune_get.restype = ctypes.c_int
    sz = ctypes.c_size_t
    lib.rpca_server_create.argtypes = [i32, i32, sz, i32, i32, i32, vp]
    lib.rpca_server_create.restype = vp
    lib.rpca_server_submit.argtypes = [vp, ctypes.POINTER(RpcaProblem), i64]
    lib.rpca_server_submit.restype = ctypes.c_int
    lib.rpca_server_step.argtypes = [vp, ctypes.POINTER(RpcaCompletion), i32, ctypes.POINTER(i32)]
    lib.rpca_server_step.restype = ctypes.c_int
    lib.rpca_server_pending.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz)]
    lib.rpca_server_pending.restype = ctypes.c_int
    lib.rpca_server_peak_bytes.argtypes = [vp]
    lib.rpca_server_peak_bytes.restype = sz
    lib.rpca_server_request_bytes.argtypes = [i64, i64, i32]
    lib.rpca_server_request_bytes.restype = sz
    lib.rpca_server_destroy.argtypes = [vp]
    lib.rpca_server_destroy.restype = None
    lib.rpca_server_set_timeout.argtypes = [vp, dbl]
    lib.rpca_server_set_timeout.restype = ctypes.c_int
    lib.rpca_server_inject_failure.argtypes = [vp, i32, i32]
    lib.rpca_server_inject_failure.restype = ctypes.c_int
    lib.rpca_autotune.argtypes = [i32, i64, vp]
    lib.rpca_autotune.restype = ctypes.c_int
    lib.rpca_autotune_save.argtypes = [ctypes.c_char_p]
    lib.rpca_autotune_save.restype = ctypes.c_int
    lib.rpca_autotune_load.argtypes = [ctypes.c_char_p]
    lib.rpca_autotune_load.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    lib.rpca_frame_correlation.argtypes = [vp, i64, i64, i32, dp, vp]
    lib.rpca_frame_keep.argtypes = [dp, i64, dbl, ip]
    lib.rpca_frame_select.argtypes = [vp, i64, i64, i32, ip, vp, vp]
    lib.rpca_moving_average.argtypes = [vp, i64, i64, i32, i32, vp, vp]
    lib.rpca_dice.argtypes = [vp, dbl, vp, dbl, i64, i32, lp, dp, vp]
    lib.rpca_rmse.argtypes = [vp, vp, i64, i32, dp, vp]
    lib.rpca_masked_mean.argtypes = [vp, vp, i64, i32, dp, vp]
    for name in ("rpca_frame_correlation", "rpca_frame_keep", "rpca_frame_select",
                 "rpca_moving_average", "rpca_dice", "rpca_rmse", "rpca_masked_mean"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib
