"""Python binding of the continuous-batching server (rpca_server_* in
include/rpca.h).  Argument marshalling only: admission, scheduling and every
iteration run in the library.

    srv = Server(dtype=RPCA_F32, hbm_budget=64 << 30, max_active=64, quantum=16)
    srv.submit(M, tag=7, tol=1e-6, maxit=1000)   # M: device Casorati tensor
    for c in srv.step():                         # one quantum of iterations
        c.tag, c.status, c.iterations, c.L, c.S

or, with futures and a background thread that steps the server:

    srv = Server(dtype=RPCA_F32, background=True)
    fut = srv.submit_async(frames)               # (n, H, W) stack or (m, n)
    c = fut.result()                             # Completion with L and S
"""
from __future__ import annotations

import ctypes
import itertools
import threading
from concurrent.futures import Future
from dataclasses import dataclass
from typing import Optional

from . import _lib
from ._lib import (RPCA_F32, RPCA_F64, RPCA_GRAM_DEFAULT, RPCA_SERVER_SIMULATE,
                   RPCA_SERVER_STAGE_INIT, RpcaCompletion)


@dataclass
class Completion:
    tag: int
    status: int
    iterations: int
    residual: float
    L: object = None
    S: object = None


def request_bytes(m: int, n: int, dtype: int) -> int:
    """Admission footprint of one request (workspace + M, L and S)."""
    return int(_lib.load().rpca_server_request_bytes(int(m), int(n), int(dtype)))


class Server:
    """Requests are admitted FIFO by footprint; each step runs `quantum`
    iterations of every active solve together on the device."""

    def __init__(self, dtype: int = RPCA_F32, hbm_budget: int = 64 << 30, max_active: int = 64,
                 quantum: int = 16, simulate: bool = False, stream: Optional[int] = None,
                 background: bool = False):
        lib = _lib.load()
        if stream is None and not simulate:
            import torch
            stream = int(torch.cuda.current_stream().cuda_stream)
        self._lib = lib
        self._dtype = int(dtype)
        self._h = lib.rpca_server_create(self._dtype, RPCA_GRAM_DEFAULT, int(hbm_budget),
                                         int(max_active), int(quantum),
                                         RPCA_SERVER_SIMULATE if simulate else 0, stream or 0)
        if not self._h:
            raise ValueError("rpca_server_create rejected the arguments")
        self._cap = max(int(max_active), 1) * 4
        self._buf = (RpcaCompletion * self._cap)()
        self._live = {}  # tag -> (M, L, S) kept alive until completion
        self._timeout = 0.0
        self._futures = {}  # tag -> Future of submit_async
        self._mu = threading.RLock()
        self._tags = itertools.count(1 << 62)  # tags of submit_async
        self._wake = threading.Event()
        self._stop = False
        self._thread = None
        if background:
            self._thread = threading.Thread(target=self._loop, name="rpca-server", daemon=True)
            self._thread.start()

    def set_timeout(self, seconds: float) -> None:
        """Timeout given to the requests submitted from now on (0 = none)."""
        rc = self._lib.rpca_server_set_timeout(self._h, float(seconds))
        if rc != 0:
            raise ValueError(f"invalid timeout {seconds!r}")
        self._timeout = float(seconds)

    def inject_failure(self, code: int, stage: int = RPCA_SERVER_STAGE_INIT) -> int:
        """Make the next set-up of admitted requests fail with `code` (tests)."""
        return int(self._lib.rpca_server_inject_failure(self._h, int(stage), int(code)))

    def submit_raw(self, problem, tag: int, keep=None) -> int:
        """Queue an rpca_problem whose device buffers the caller owns.  The
        library rejects a tag that names a request not yet reported."""
        with self._mu:
            rc = self._lib.rpca_server_submit(self._h, ctypes.byref(problem), int(tag))
            if rc == 0:
                self._live[int(tag)] = keep
        return int(rc)

    def submit(self, M, tag: int, lam: Optional[float] = None, mu: Optional[float] = None,
               tol: float = 1e-6, maxit: int = 1000, timeout: Optional[float] = None) -> None:
        """Queue a solve of the device tensor M; L and S are allocated here and
        returned with the completion.  M must be a device tensor of the
        server's dtype; `tag` must not name a request not yet reported.
        `timeout` (seconds) overrides the server's timeout for this request."""
        import torch
        from . import _problem, _check_device, _dtype_code
        with self._mu:
            if int(tag) in self._live:
                raise ValueError(f"tag {tag} names a request that has not been reported")
        if _dtype_code(M) != self._dtype:
            raise ValueError("M's dtype differs from the server's dtype")
        _check_device(M)
        L = torch.empty_like(M)
        S = torch.empty_like(M)
        p = _problem(M, L, S, lam, mu, tol, maxit)
        if timeout is not None:
            self.set_timeout(timeout)
        try:
            rc = self.submit_raw(p, tag, keep=(M, L, S))
        finally:
            if timeout is not None:
                self.set_timeout(self._timeout)
        if rc != 0:
            raise ValueError(f"request rejected: {rc}")

    def submit_async(self, frames, lam: Optional[float] = None, mu: Optional[float] = None,
                     tol: float = 1e-6, maxit: int = 1000, timeout: Optional[float] = None) -> Future:
        """Queue a window (an (n, H, W) frame stack or an (m, n) Casorati
        tensor on the device) and return a Future that step() (or the
        background thread) resolves with its Completion."""
        fut = Future()
        with self._mu:
            tag = next(self._tags)
            self._futures[tag] = fut
            try:
                self.submit(frames, tag, lam=lam, mu=mu, tol=tol, maxit=maxit, timeout=timeout)
            except BaseException:
                self._futures.pop(tag, None)
                raise
        self._wake.set()
        return fut

    def step(self) -> list:
        with self._mu:
            n = ctypes.c_int32(0)
            rc = self._lib.rpca_server_step(self._h, self._buf, self._cap, ctypes.byref(n))
            out = []
            for i in range(n.value):
                c = self._buf[i]
                keep = self._live.pop(int(c.tag), None)
                L = S = None
                if keep is not None and len(keep) == 3:
                    L, S = keep[1], keep[2]
                out.append(Completion(int(c.tag), int(c.status), int(c.iterations), float(c.residual), L, S))
            err = None
            if rc < 0:
                err = RuntimeError(f"server step failed ({rc}): {self._lib.rpca_last_error().decode()}")
            futs, plain = [], []
            for c in out:
                f = self._futures.pop(c.tag, None)
                (plain if f is None else futs).append(c if f is None else (f, c))
        for fut, c in futs:
            fut.set_result(c)
        if err is not None:
            raise err
        return plain

    def _loop(self):
        """Background stepping: run quanta while requests are pending, sleep
        until the next submit_async otherwise."""
        while not self._stop:
            try:
                left = self.pending()[0]
            except Exception:
                break
            if left == 0:
                self._wake.wait(0.05)
                self._wake.clear()
                continue
            try:
                self.step()
            except Exception as e:  # a device failure: fail every waiting future
                with self._mu:
                    futs = list(self._futures.values())
                    self._futures.clear()
                for f in futs:
                    f.set_exception(e)
                break

    def pending(self) -> tuple[int, int, int, int]:
        """(not yet reported, queued, active, admitted bytes)."""
        q, a, b = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_size_t(0)
        left = self._lib.rpca_server_pending(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b))
        return int(left), int(q.value), int(a.value), int(b.value)

    def peak_bytes(self) -> int:
        return int(self._lib.rpca_server_peak_bytes(self._h))

    def close(self) -> None:
        self._stop = True
        self._wake.set()
        if self._thread is not None and self._thread is not threading.current_thread():
            self._thread.join()
        self._thread = None
        with self._mu:
            if self._h:
                self._lib.rpca_server_destroy(self._h)
                self._h = None
                self._live.clear()
            futs = list(self._futures.values())
            self._futures.clear()
        for f in futs:
            if not f.done():
                f.cancel()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
