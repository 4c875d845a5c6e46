"""rpca_solve_noalloc (workspace in the library's static device array) against
the allocating entry points rpca_solve_f32 / rpca_solve_f64, through the C
ABI: bitwise the same L, S, status and iteration count on two calls in a
row, the second with a smaller input, and the oracle's bar on the small one."""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro
from synth import window_512x512x20, planted_low_rank_sparse, batch_window
from tests.gpu_helpers import to_dev, to_host, report, device

pytestmark = pytest.mark.gpu


def _inputs(dtype):
    w = window_512x512x20()
    big = (w.X().astype(dtype), dict(lam=1.0 / 512, tol=1e-6, maxit=60))
    L0, S0 = planted_low_rank_sparse(3001, 13, 2, 0.05, 77)
    rng = np.random.default_rng(78)
    Xs = np.asfortranarray(L0 + S0 + 1e-3 * rng.standard_normal(L0.shape)).astype(dtype)
    small = (Xs, dict(lam=-1.0, tol=1e-6, maxit=300))
    return [big, small]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_equals_allocating_call(dtype):
    import torch
    device()
    code = rp.RPCA_F32 if dtype == np.float32 else rp.RPCA_F64
    alloc_fn = rp.rpca_solve_f32 if dtype == np.float32 else rp.rpca_solve_f64
    for X, kw in _inputs(dtype):
        m, n = X.shape
        M = to_dev(X, dtype)
        L1, S1 = torch.empty_like(M), torch.empty_like(M)
        rc1, it1 = alloc_fn(M, m, n, kw["lam"], -1.0, kw["tol"], kw["maxit"], L1, S1)
        L2 = torch.full_like(M, float("nan"))
        S2 = torch.full_like(M, float("nan"))
        torch.cuda.synchronize()
        rc2, it2 = rp.rpca_solve_noalloc(M, m, n, code, kw["lam"], -1.0, kw["tol"], kw["maxit"],
                                         L2, S2)
        torch.cuda.synchronize()
        same = torch.equal(L1, L2) and torch.equal(S1, S2)
        report(f"noalloc {m}x{n}", dtype=np.dtype(dtype).name, rc=rc2, rc_alloc=rc1, it=it2,
               it_alloc=it1, bitwise=int(same))
        assert rc2 == rc1 and it2 == it1
        assert same
    # the second (smaller) solve also meets the oracle's bar
    ref = rpca(X.astype(np.float64), lam=kw["lam"], tol=kw["tol"], maxit=kw["maxit"])
    bar = 1e-10 if dtype == np.float64 else 1e-4
    relL, relS = rel_fro(to_host(L2), ref.L), rel_fro(to_host(S2), ref.S)
    report("noalloc small vs oracle", relL=relL, relS=relS, it=it2, it_ref=ref.iterations)
    assert relL <= bar and relS <= bar
    assert abs(it2 - ref.iterations) <= (0 if dtype == np.float64 else 1)


# Wide windows: the in-place eigensolver with V in the workspace (and, for
# FP32 solves of 113-136 frames, its FP32 increment path and scratch), two
# calls in a row, the second smaller.
@pytest.mark.parametrize("dtype,shapes", [
    (np.float32, [(48, 40, 132), (40, 40, 100)]),
    (np.float64, [(40, 40, 128), (36, 40, 100)]),
])
def test_noalloc_wide_classes_equal_allocating_call(dtype, shapes):
    import torch
    device()
    code = rp.RPCA_F32 if dtype == np.float32 else rp.RPCA_F64
    alloc_fn = rp.rpca_solve_f32 if dtype == np.float32 else rp.rpca_solve_f64
    tol = 1e-6 if dtype == np.float32 else 1e-9
    for H, W, n in shapes:
        X = batch_window(H, W, n, 8100 + n).X().astype(dtype)
        m = X.shape[0]
        M = to_dev(X, dtype)
        L1, S1 = torch.empty_like(M), torch.empty_like(M)
        rc1, it1 = alloc_fn(M, m, n, -1.0, -1.0, tol, 80, L1, S1)
        L2 = torch.full_like(M, float("nan"))
        S2 = torch.full_like(M, float("nan"))
        torch.cuda.synchronize()
        rc2, it2 = rp.rpca_solve_noalloc(M, m, n, code, -1.0, -1.0, tol, 80, L2, S2)
        torch.cuda.synchronize()
        same = torch.equal(L1, L2) and torch.equal(S1, S2)
        report(f"noalloc wide {H}x{W}x{n}", dtype=np.dtype(dtype).name, rc=rc2, rc_alloc=rc1,
               it=it2, it_alloc=it1, bitwise=int(same))
        assert rc2 == rc1 and it2 == it1
        assert same


def test_noalloc_too_large_is_rejected():
    import torch
    device()
    m, n = 1 << 22, 20
    M = torch.zeros((n, m), dtype=torch.float32, device="cuda:0").t()
    L = torch.empty_like(M)
    S = torch.empty_like(M)
    rc, it = rp.rpca_solve_noalloc(M, m, n, rp.RPCA_F32, -1.0, -1.0, 1e-6, 10, L, S)
    assert rc == rp.RPCA_ERR_ARG and it == 0
    assert "RPCA_NOALLOC_MAX_BYTES" in rp.rpca_last_error()
