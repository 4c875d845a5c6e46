"""Binding of the processing steps around the solve (rpca_frame_correlation,
rpca_frame_keep, rpca_frame_select, rpca_moving_average, rpca_dice, rpca_rmse,
rpca_masked_mean in include/rpca.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes

from . import _lib, casorati_shape, _dtype_code, _stream_ptr


def _check(rc: int, name: str) -> int:
    if rc < 0:
        raise RuntimeError(f"{name} failed ({rc}): {_lib.load().rpca_last_error().decode()}")
    return rc


def frame_correlation(M):
    """Correlations of consecutive frames of the device Casorati tensor M."""
    import numpy as np
    m, n = casorati_shape(M)
    rho = np.zeros(max(n - 1, 1))
    _check(_lib.load().rpca_frame_correlation(
        M.data_ptr(), m, n, _dtype_code(M), rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        _stream_ptr(M)), "rpca_frame_correlation")
    return rho[: n - 1]


def frame_keep(rho, threshold: float = 0.8):
    import numpy as np
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    keep = np.zeros(len(rho) + 1, dtype=np.int32)
    _check(_lib.load().rpca_frame_keep(rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       len(rho) + 1, float(threshold),
                                       keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "rpca_frame_keep")
    return keep.astype(bool)


def frame_select(M, keep):
    """The kept frames of M as a new (m, kept) column-major tensor."""
    import numpy as np
    import torch
    m, n = casorati_shape(M)
    k = np.ascontiguousarray(np.asarray(keep, dtype=np.int32))
    out = torch.empty((int(k.sum()), m), dtype=M.dtype, device=M.device).t()
    _check(_lib.load().rpca_frame_select(M.data_ptr(), m, n, _dtype_code(M),
                                         k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         out.data_ptr(), _stream_ptr(M)), "rpca_frame_select")
    return out


def moving_average(M, W: int = 20):
    import torch
    m, n = casorati_shape(M)
    out = torch.empty((n - W + 1, m), dtype=M.dtype, device=M.device).t()
    _check(_lib.load().rpca_moving_average(M.data_ptr(), m, n, int(W), _dtype_code(M),
                                           out.data_ptr(), _stream_ptr(M)), "rpca_moving_average")
    return out


def dice(A, thr_a: float, B, thr_b: float):
    """(Dice, (|A & B|, |A|, |B|)) of the binarised tensors A >= thr_a, B >= thr_b."""
    counts = (ctypes.c_int64 * 3)()
    d = ctypes.c_double(0.0)
    _check(_lib.load().rpca_dice(A.data_ptr(), float(thr_a), B.data_ptr(), float(thr_b), A.numel(),
                                 _dtype_code(A), counts, ctypes.byref(d), _stream_ptr(A)), "rpca_dice")
    return d.value, tuple(int(c) for c in counts)


def rmse(A, B) -> float:
    out = ctypes.c_double(0.0)
    _check(_lib.load().rpca_rmse(A.data_ptr(), B.data_ptr(), A.numel(), _dtype_code(A),
                                 ctypes.byref(out), _stream_ptr(A)), "rpca_rmse")
    return out.value


def masked_mean(A, mask) -> float:
    """Mean of A where the uint8 device mask is nonzero."""
    out = ctypes.c_double(0.0)
    _check(_lib.load().rpca_masked_mean(A.data_ptr(), mask.data_ptr(), A.numel(), _dtype_code(A),
                                        ctypes.byref(out), _stream_ptr(A)), "rpca_masked_mean")
    return out.value
