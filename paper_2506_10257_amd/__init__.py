"""MI355X RPCA: Python binding of librpca_mi355x.so.

The functions named like the C ABI (``rpca_solve_f32``, ``rpca_solve_f64``,
``rpca_solve_many``, ...) marshal torch tensors to device pointers and call
the library; ``solve`` / ``solve_many`` are the same calls with outputs
allocated for the caller.  torch supplies device memory and the current HIP
stream only.

Matrix arguments are the Casorati matrix (pixels x frames) of paper Sec. II-A,
column-major with leading dimension m: either a 2-D (m, n) tensor with
strides (1, m) (the transpose of a contiguous (n, m) tensor), or a
C-contiguous (n, H, W) image stack (m = H*W).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

from . import _lib
from ._lib import (RPCA_OK, RPCA_NOT_CONVERGED, RPCA_ERR_ARG, RPCA_ERR_NOMEM,
                   RPCA_ERR_DEVICE, RPCA_ERR_NONFINITE, RPCA_ERR_UNSUPPORTED, RPCA_ERR_TIMEOUT,
                   RPCA_F32, RPCA_F64, RPCA_GRAM_DEFAULT, RPCA_GRAM_BF16X3, RPCA_GRAM_BF16X6, RPCA_N_MAX, RPCA_N_MAX_F64,
                   RPCA_KNOB_EIG_THREADS, RPCA_KNOB_STREAM_KERNEL, RPCA_KNOB_TILE_ROWS, RPCA_KNOB_REG_TILES, RpcaProblem,
                   RpcaProfile, RPCA_NOALLOC_MAX_BYTES)

__all__ = ["solve", "solve_many", "SolveResult", "casorati_shape", "rpca_solve_f32",
           "rpca_solve_f64", "rpca_solve_noalloc", "rpca_solve_many", "rpca_solve_ex", "rpca_footprint_bytes",
           "rpca_strerror", "rpca_version", "rpca_last_error", "rpca_profile_enable", "rpca_profile_read",
           "rpca_tune_set", "rpca_tune_get", "RPCA_KNOB_EIG_THREADS", "RPCA_KNOB_STREAM_KERNEL", "RPCA_KNOB_TILE_ROWS", "RPCA_KNOB_REG_TILES", "Server",
           "rpca_autotune", "rpca_autotune_save", "rpca_autotune_load", "tuning_choices",
           "RPCA_OK", "RPCA_NOT_CONVERGED", "RPCA_ERR_ARG", "RPCA_ERR_NOMEM",
           "RPCA_ERR_DEVICE", "RPCA_ERR_NONFINITE", "RPCA_ERR_UNSUPPORTED", "RPCA_ERR_TIMEOUT", "RPCA_F32",
           "RPCA_F64", "RPCA_GRAM_DEFAULT", "RPCA_GRAM_BF16X3", "RPCA_GRAM_BF16X6", "RPCA_N_MAX", "RPCA_N_MAX_F64"]


def _stream_ptr(t) -> int:
    import torch
    return int(torch.cuda.current_stream(t.device).cuda_stream)


def casorati_shape(t) -> tuple[int, int]:
    """(m, n) of a Casorati tensor in either accepted layout; raises otherwise."""
    if t.dim() == 2:
        m, n = int(t.shape[0]), int(t.shape[1])
        if n == 1 or m == 1:
            if t.is_contiguous() or t.t().is_contiguous():
                return m, n
        if t.stride(0) == 1 and t.stride(1) == m:
            return m, n
        raise ValueError("2-D input must be column-major (strides (1, m))")
    if t.dim() == 3:
        if not t.is_contiguous():
            raise ValueError("3-D input must be a C-contiguous (n, H, W) stack")
        return int(t.shape[1] * t.shape[2]), int(t.shape[0])
    raise ValueError("input must be (m, n) column-major or (n, H, W)")


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return RPCA_F32
    if t.dtype == torch.float64:
        return RPCA_F64
    raise TypeError("input must be float32 or float64")


def _check_device(*ts):
    dev = ts[0].device
    if dev.type != "cuda":
        raise ValueError("tensors must be on a HIP device (torch 'cuda')")
    for t in ts:
        if t.device != dev or t.dtype != ts[0].dtype:
            raise ValueError("all tensors must share device and dtype")


def rpca_solve_f32(M, m: int, n: int, lam: float, mu: float, tol: float, maxit: int, L, S,
                   stream: Optional[int] = None) -> tuple[int, int]:
    """C ``rpca_solve_f32`` on torch tensors (or raw device addresses as int)."""
    return _solve_raw(_lib.load().rpca_solve_f32, M, m, n, lam, mu, tol, maxit, L, S, stream)


def rpca_solve_f64(M, m: int, n: int, lam: float, mu: float, tol: float, maxit: int, L, S,
                   stream: Optional[int] = None) -> tuple[int, int]:
    """C ``rpca_solve_f64`` on torch tensors (or raw device addresses as int)."""
    return _solve_raw(_lib.load().rpca_solve_f64, M, m, n, lam, mu, tol, maxit, L, S, stream)


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _solve_raw(fn, M, m, n, lam, mu, tol, maxit, L, S, stream):
    if stream is None:
        stream = _stream_ptr(M) if hasattr(M, "device") else 0
    it = ctypes.c_int32(0)
    rc = fn(_ptr(M), int(m), int(n), float(lam), float(mu), float(tol), int(maxit),
            _ptr(L), _ptr(S), ctypes.byref(it), stream)
    return int(rc), int(it.value)


def rpca_solve_noalloc(M, m: int, n: int, dtype: int, lam: float, mu: float, tol: float,
                       maxit: int, L, S, stream: Optional[int] = None) -> tuple[int, int]:
    """C ``rpca_solve_noalloc``: the solve of rpca_solve_f32 / rpca_solve_f64
    with its workspace in the library's static device array (no allocation
    during the call).  Returns (status, iterations)."""
    if stream is None:
        stream = _stream_ptr(M) if hasattr(M, "device") else 0
    it = ctypes.c_int32(0)
    rc = _lib.load().rpca_solve_noalloc(_ptr(M), int(m), int(n), int(dtype), float(lam), float(mu),
                                        float(tol), int(maxit), _ptr(L), _ptr(S), ctypes.byref(it),
                                        stream)
    return int(rc), int(it.value)


def rpca_solve_many(problems: Sequence[RpcaProblem], dtype: int, gram_mode: int = RPCA_GRAM_DEFAULT,
                    stream: int = 0) -> int:
    arr = (RpcaProblem * len(problems))(*problems)
    rc = _lib.load().rpca_solve_many(arr, len(problems), int(dtype), int(gram_mode), stream)
    for i, p in enumerate(problems):
        p.iterations, p.status, p.residual = arr[i].iterations, arr[i].status, arr[i].residual
    return int(rc)


def rpca_solve_ex(problem: RpcaProblem, dtype: int, gram_mode: int, stream: int = 0) -> int:
    return int(_lib.load().rpca_solve_ex(ctypes.byref(problem), int(dtype), int(gram_mode), stream))


def rpca_footprint_bytes(m: int, n: int, dtype: int) -> int:
    return int(_lib.load().rpca_footprint_bytes(int(m), int(n), int(dtype)))


def rpca_strerror(code: int) -> str:
    return _lib.load().rpca_strerror(int(code)).decode()


def rpca_last_error() -> str:
    return _lib.load().rpca_last_error().decode()


def rpca_version() -> str:
    return _lib.load().rpca_version().decode()


def rpca_profile_enable(on: bool) -> None:
    _lib.load().rpca_profile_enable(1 if on else 0)


def rpca_profile_read(reset: bool = True) -> dict:
    p = RpcaProfile()
    _lib.load().rpca_profile_read(ctypes.byref(p), 1 if reset else 0)
    return {name: getattr(p, name) for name, _ in RpcaProfile._fields_}


def rpca_tune_set(knob: int, dtype: int, cls: int, value: int) -> int:
    return int(_lib.load().rpca_tune_set(int(knob), int(dtype), int(cls), int(value)))


def rpca_tune_get(knob: int, dtype: int, cls: int) -> int:
    return int(_lib.load().rpca_tune_get(int(knob), int(dtype), int(cls)))


def rpca_autotune(dtype: int, rows: int = 262144, stream: Optional[int] = None) -> int:
    """Time every tuning variant on this device and keep the fastest."""
    if stream is None:
        import torch
        stream = int(torch.cuda.current_stream().cuda_stream)
    return int(_lib.load().rpca_autotune(int(dtype), int(rows), stream))


def rpca_autotune_save(path: str) -> int:
    return int(_lib.load().rpca_autotune_save(str(path).encode()))


def rpca_autotune_load(path: str) -> int:
    return int(_lib.load().rpca_autotune_load(str(path).encode()))


def tuning_choices() -> dict:
    """Current knob values: {"eig_threads": {(dtype, cls): v}, "stream_kernel": {cls: v},
    "tile_rows": {nb: rows}, "reg_tiles": {(dtype, cls): tiles}}."""
    out = {"eig_threads": {}, "stream_kernel": {}, "tile_rows": {}}
    for dt in (RPCA_F64, RPCA_F32):
        for cls in (16, 32, 64):
            out["eig_threads"][(dt, cls)] = rpca_tune_get(RPCA_KNOB_EIG_THREADS, dt, cls)
    for cls in (4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60, 64):
        out["stream_kernel"][cls] = rpca_tune_get(RPCA_KNOB_STREAM_KERNEL, RPCA_F32, cls)
    for nb in range(16, 145, 16):
        out["tile_rows"][nb] = rpca_tune_get(RPCA_KNOB_TILE_ROWS, RPCA_F32, nb)
    out["reg_tiles"] = {}
    for cls in (4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60, 64):
        out["reg_tiles"][(RPCA_F32, cls)] = rpca_tune_get(RPCA_KNOB_REG_TILES, RPCA_F32, cls)
    for cls in (4, 8, 10, 12, 16, 20, 24, 28, 32):
        out["reg_tiles"][(RPCA_F64, cls)] = rpca_tune_get(RPCA_KNOB_REG_TILES, RPCA_F64, cls)
    return out


@dataclass
class SolveResult:
    L: object
    S: object
    iterations: int
    status: int
    residual: float
    Y: object = None  # the final dual variable, when asked for


def _problem(M, L, S, lam, mu, tol, maxit, S0=None, Y0=None, Y=None) -> RpcaProblem:
    m, n = casorati_shape(M)
    p = RpcaProblem()
    p.M, p.m, p.n = M.data_ptr(), m, n
    p.lam = -1.0 if lam is None else float(lam)
    p.mu = -1.0 if mu is None else float(mu)
    p.tol, p.maxit = float(tol), int(maxit)
    p.L, p.S = L.data_ptr(), S.data_ptr()
    for name, t in (("S0", S0), ("Y0", Y0)):
        if t is not None:
            if t.shape != M.shape or t.stride() != M.stride() or t.dtype != M.dtype or t.device != M.device:
                raise ValueError(f"{name} must have M's shape, layout, dtype and device")
            setattr(p, name, t.data_ptr())
    if Y is not None:
        p.Y = Y.data_ptr()
    return p


def solve(M, lam: Optional[float] = None, mu: Optional[float] = None, tol: float = 1e-7,
          maxit: int = 500, gram_mode: int = RPCA_GRAM_DEFAULT, S0=None, Y0=None,
          return_Y: bool = False) -> SolveResult:
    """One RPCA solve of M; L and S are returned in M's layout.  S0, Y0
    (optional, M's layout) start the iteration from a given S and Y instead
    of zero; return_Y also returns the final dual Y.  A negative status
    raises RuntimeError."""
    import torch
    _check_device(M)
    dt = _dtype_code(M)
    L = torch.empty_like(M)
    S = torch.empty_like(M)
    Y = torch.empty_like(M) if return_Y else None
    p = _problem(M, L, S, lam, mu, tol, maxit, S0, Y0, Y)
    rc = rpca_solve_ex(p, dt, gram_mode, _stream_ptr(M))
    if rc < 0:
        raise RuntimeError(f"rpca solve failed: {rpca_strerror(rc)} ({rc}) {rpca_last_error()}")
    return SolveResult(L, S, int(p.iterations), int(p.status), float(p.residual), Y)


def solve_many(Ms: Sequence, lam: Optional[float] = None, mu: Optional[float] = None,
               tol: float = 1e-7, maxit: int = 500,
               gram_mode: int = RPCA_GRAM_DEFAULT) -> list[SolveResult]:
    """Batched solve (one set of launches per iteration for all problems)."""
    import torch
    if len(Ms) == 0:
        return []
    _check_device(*Ms)
    dt = _dtype_code(Ms[0])
    outs = [(torch.empty_like(M), torch.empty_like(M)) for M in Ms]
    probs = [_problem(M, L, S, lam, mu, tol, maxit) for M, (L, S) in zip(Ms, outs)]
    rc = rpca_solve_many(probs, dt, gram_mode, _stream_ptr(Ms[0]))
    if rc < 0:
        raise RuntimeError(f"rpca batch failed: {rpca_strerror(rc)} ({rc}) {rpca_last_error()}")
    return [SolveResult(L, S, int(p.iterations), int(p.status), float(p.residual))
            for (L, S), p in zip(outs, probs)]


from .server import Server  # noqa: E402
