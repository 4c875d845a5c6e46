"""Solves started from a given S0 / Y0 (sliding-window warm start) and the
final-Y output, against the FP64 oracle run from the same start.

Bars as for cold starts: FP64 relative Frobenius error <= 1e-10 with the same
iteration count, FP32 <= 1e-4 with the count within one.
"""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro
from synth import make_window, batch_window
from tests.gpu_helpers import device, to_dev, to_host, report

pytestmark = pytest.mark.gpu


def _sliding(H, W, n, step, seed):
    """Window 2 of a sliding pair and its start: window 1's oracle S and Y
    shifted by `step` frames, zeros for the new frames."""
    w = make_window(H, W, n + step, max(1, H * W // 1300), max(1, 2 * H * W // 1300), 3, 20.0, seed)
    X = w.X()
    prev = rpca(X[:, :n], tol=1e-7, maxit=2000)
    S0 = np.zeros((X.shape[0], n))
    Y0 = np.zeros((X.shape[0], n))
    S0[:, : n - step] = prev.S[:, step:]
    Y0[:, : n - step] = prev.Y[:, step:]
    return np.asfortranarray(X[:, step:]), S0, Y0


def _gpu(X, dtype, S0=None, Y0=None, tol=1e-7, maxit=2000, gram_mode=rp.RPCA_GRAM_DEFAULT):
    M = to_dev(X, dtype)
    s0 = to_dev(S0, dtype) if S0 is not None else None
    y0 = to_dev(Y0, dtype) if Y0 is not None else None
    r = rp.solve(M, tol=tol, maxit=maxit, S0=s0, Y0=y0, return_Y=True, gram_mode=gram_mode)
    return r


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("which", ["both", "S0", "Y0"])
def test_warm_start_matches_oracle(dtype, which):
    device()
    X, S0, Y0 = _sliding(48, 48, 20, 5, 9000)
    s0 = S0 if which in ("both", "S0") else None
    y0 = Y0 if which in ("both", "Y0") else None
    tol = 1e-7 if dtype == np.float64 else 1e-6
    ref = rpca(X, tol=tol, maxit=2000, S0=s0, Y0=y0)
    r = _gpu(X, dtype, s0, y0, tol=tol)
    L, S, Y = to_host(r.L), to_host(r.S), to_host(r.Y)
    eL, eS, eY = rel_fro(L, ref.L), rel_fro(S, ref.S), rel_fro(Y, ref.Y)
    report(f"warm {which} {np.dtype(dtype).name}", it=r.iterations, it_ref=ref.iterations,
           relL=eL, relS=eS, relY=eY)
    bar = 1e-10 if dtype == np.float64 else 1e-4
    assert eL <= bar and eS <= bar and eY <= bar
    if dtype == np.float64:
        assert r.iterations == ref.iterations and r.status == ref.status
    else:
        assert abs(r.iterations - ref.iterations) <= 1


@pytest.mark.parametrize("n,gram_mode", [(40, rp.RPCA_GRAM_DEFAULT), (100, rp.RPCA_GRAM_DEFAULT),
                                         (132, rp.RPCA_GRAM_DEFAULT), (20, rp.RPCA_GRAM_BF16X6)])
def test_warm_start_tile_kernel_classes(n, gram_mode):
    """Warm starts through the MFMA tile kernel (40, 100, 132 frames; BF16x6);
    at 132 frames the eigensolver's FP32 increment path from the second
    iteration on."""
    device()
    X, S0, Y0 = _sliding(40, 44, n, 10, 9100 + n)
    ref = rpca(X, tol=1e-6, maxit=2000, S0=S0, Y0=Y0)
    r = _gpu(X, np.float32, S0, Y0, tol=1e-6, gram_mode=gram_mode)
    eL, eS = rel_fro(to_host(r.L), ref.L), rel_fro(to_host(r.S), ref.S)
    eY = rel_fro(to_host(r.Y), ref.Y)
    report(f"warm tile n={n} mode={gram_mode}", it=r.iterations, it_ref=ref.iterations,
           relL=eL, relS=eS, relY=eY)
    assert eL <= 1e-4 and eS <= 1e-4 and eY <= 1e-4
    assert abs(r.iterations - ref.iterations) <= 1


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cold_final_Y_matches_oracle(dtype):
    device()
    X = batch_window(48, 40, 12, 9200).X()
    ref = rpca(X, tol=1e-7, maxit=1000)
    r = _gpu(X, dtype, tol=1e-7, maxit=1000)
    eY = rel_fro(to_host(r.Y), ref.Y)
    report(f"cold Y {np.dtype(dtype).name}", it=r.iterations, it_ref=ref.iterations, relY=eY)
    if dtype == np.float64:
        assert r.iterations == ref.iterations
    else:
        assert abs(r.iterations - ref.iterations) <= 1
    assert eY <= (1e-10 if dtype == np.float64 else 1e-4)


def test_warm_mixed_batch_bitwise_equals_alone():
    import torch
    device()
    cases = [_sliding(40, 40, 20, 5, 9300), _sliding(36, 44, 40, 10, 9301)]
    probs_dev, alone = [], []
    for X, S0, Y0 in cases:
        M, s0, y0 = to_dev(X, np.float32), to_dev(S0, np.float32), to_dev(Y0, np.float32)
        probs_dev.append((M, s0, y0))
        alone.append(rp.solve(M, tol=1e-6, maxit=500, S0=s0, Y0=y0, return_Y=True))
    cold = to_dev(batch_window(40, 40, 20, 9302).X(), np.float32)
    cold_alone = rp.solve(cold, tol=1e-6, maxit=500)
    outs, probs = [], []
    for M, s0, y0 in probs_dev:
        L, S, Y = torch.empty_like(M), torch.empty_like(M), torch.empty_like(M)
        outs.append((L, S, Y))
        probs.append(rp._problem(M, L, S, None, None, 1e-6, 500, s0, y0, Y))
    Lc, Sc = torch.empty_like(cold), torch.empty_like(cold)
    probs.append(rp._problem(cold, Lc, Sc, None, None, 1e-6, 500))
    rc = rp.rpca_solve_many(probs, rp.RPCA_F32, rp.RPCA_GRAM_DEFAULT,
                            int(torch.cuda.current_stream().cuda_stream))
    assert rc >= 0
    torch.cuda.synchronize()
    for (L, S, Y), a, p in zip(outs, alone, probs):
        assert p.iterations == a.iterations
        assert torch.equal(L, a.L) and torch.equal(S, a.S) and torch.equal(Y, a.Y)
    assert torch.equal(Lc, cold_alone.L) and torch.equal(Sc, cold_alone.S)


def test_warm_zero_input():
    import torch
    device()
    M = torch.zeros((20, 2000), device="cuda", dtype=torch.float32).t()
    S0 = torch.ones_like(M)
    r = rp.solve(M, tol=1e-6, maxit=20, S0=S0, Y0=S0, return_Y=True)
    assert r.status == rp.RPCA_OK and r.iterations == 0
    assert bool((r.L == 0).all()) and bool((r.S == 0).all()) and bool((r.Y == 0).all())
