"""Helpers for the GPU tests: move seeded inputs to the device in the
Casorati layout and call the library through its C-ABI names."""
import numpy as np

import paper_2506_10257_amd as rp


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(X: np.ndarray, dtype):
    """(m, n) numpy array -> column-major (m, n) device tensor (strides (1, m))."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(X, dtype=dtype).T))
    return t.to(device()).t()


def to_host(t) -> np.ndarray:
    return t.t().contiguous().cpu().numpy().T.astype(np.float64)


def gpu_solve(X: np.ndarray, dtype=np.float64, lam=-1.0, mu=-1.0, tol=1e-7, maxit=500):
    """Run rpca_solve_f64 / rpca_solve_f32 on X; returns (L, S, iters, status)."""
    import torch
    M = to_dev(X, dtype)
    L = torch.empty_like(M)
    S = torch.empty_like(M)
    m, n = X.shape
    fn = rp.rpca_solve_f64 if dtype == np.float64 else rp.rpca_solve_f32
    rc, it = fn(M, m, n, lam, mu, tol, maxit, L, S)
    torch.cuda.synchronize()
    return L, S, it, rc, M


def report(name, **kw):
    """Print a one-line record of a GPU check (read from the run log)."""
    items = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items())
    print(f"[parity] {name} {items}", flush=True)
