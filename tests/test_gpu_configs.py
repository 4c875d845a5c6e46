"""GPU parity at the sizes of the benchmark workloads, element-wise against the
FP64 oracle run live (whole-matrix relative Frobenius error of L and S).

* 512x512 x 20 (262144 x 20): the full 1000-iteration solve at tol 1e-6 in
  FP64 (<= 1e-10, same iteration count and status) and FP32 (<= 1e-4,
  iterations +-1), bound-bubble mask Dice >= 0.999 in both.
* the 64-window batch: one window for every (image size x frame count) cell
  of the batch set, all 16 in one rpca_solve_many call, at iterate level
  (tol = 0, k = 10) against the oracle, then each window's full solve
  (tol 1e-6, maxit 1000) bitwise equal alone and inside the batch.
* 1024x1024 x 40 (1048576 x 40, 15 dB): iterate level k = 5 for FP32 and the
  three-way split BF16 mode (<= 1e-4), and the two-way split BF16 mode
  against its error budget (tests/bf16_budget.py).
* 512x512 x 132 (262144 x 132, the 132-frame workload's window): iterate
  level k = 3 in FP32 (<= 1e-4, the FP32 bar; relS is about 1e-5 at this
  size from the first iterate on); iterations 2 and 3 run the eigensolver's
  warm start, which for 113-136 frames accumulates its rotations as an
  FP32 increment.
"""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro, dice, bound_threshold
from synth import window_512x512x20, window_1024x1024x40, batch_window, BATCH_SIZES, BATCH_FRAMES
from tests.bf16_budget import bf16x3_budget
from tests.gpu_helpers import gpu_solve, to_dev, to_host, report, device

pytestmark = pytest.mark.gpu


# ------------------------------------------------- 512x512 x 20, full solve
@pytest.fixture(scope="module")
def cfg2():
    w = window_512x512x20()
    X = w.X()
    print("[configs] oracle: 512x512x20 full solve (1000 FP64 SVD iterations)", flush=True)

    def progress(k, L, S, Y):
        if k % 100 == 0:
            print(f"[configs] oracle 512x512x20: iteration {k}", flush=True)

    ref = rpca(X, lam=1.0 / 512, tol=1e-6, maxit=1000, callback=progress)
    theta = bound_threshold(w.L_gt, w.bound_mask)
    return X, ref, theta


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_512x512x20_full_solve_elementwise(cfg2, dtype):
    X, ref, theta = cfg2
    L, S, it, rc, _ = gpu_solve(X.astype(dtype), dtype, lam=1.0 / 512, tol=1e-6, maxit=1000)
    Lh, Sh = to_host(L), to_host(S)
    relL, relS = rel_fro(Lh, ref.L), rel_fro(Sh, ref.S)
    d = dice(Lh >= theta, ref.L >= theta)
    report("512x512x20 full", dtype=np.dtype(dtype).name, it=it, it_ref=ref.iterations, rc=rc,
           rc_ref=ref.status, relL=relL, relS=relS, dice=d)
    if dtype == np.float64:
        assert it == ref.iterations and rc == ref.status
        assert relL <= 1e-10 and relS <= 1e-10
    else:
        assert abs(it - ref.iterations) <= 1
        assert relL <= 1e-4 and relS <= 1e-4
    assert d >= 0.999


# ------------------------------------------------- the 64-window batch cells
def _cell_windows():
    cells = [(H, W, n) for (H, W) in BATCH_SIZES for n in BATCH_FRAMES]
    return [(H, W, n, batch_window(H, W, n, 3100 + i)) for i, (H, W, n) in enumerate(cells)]


@pytest.fixture(scope="module")
def cfg3():
    return _cell_windows()


@pytest.mark.timeout(1200)
def test_batch_cells_iterate_parity(cfg3):
    """Every (size x frames) cell in one batched call, k = 10 iterations."""
    import torch
    device()
    K = 10
    Xs = [w.X().astype(np.float32) for (_, _, _, w) in cfg3]
    res = rp.solve_many([to_dev(X, np.float32) for X in Xs], tol=0.0, maxit=K)
    torch.cuda.synchronize()
    worst = 0.0
    for (H, W, n, _), X, r in zip(cfg3, Xs, res):
        ref = rpca(X.astype(np.float64), tol=0.0, maxit=K)
        relL, relS = rel_fro(to_host(r.L), ref.L), rel_fro(to_host(r.S), ref.S)
        report(f"batch cell {H}x{W}x{n} k={K}", it=r.iterations, relL=relL, relS=relS)
        assert r.iterations == K and r.status == rp.RPCA_NOT_CONVERGED
        assert relL <= 1e-4 and relS <= 1e-4
        worst = max(worst, relL, relS)
    report("batch cells", worst=worst)


@pytest.mark.timeout(900)
def test_batch_cells_full_solve_bitwise_alone(cfg3):
    """Full solves (tol 1e-6, maxit 1000): each window's result inside the
    batch is bitwise the one it gets alone."""
    import torch
    device()
    Ms = [to_dev(w.X(), np.float32) for (_, _, _, w) in cfg3]
    many = rp.solve_many(Ms, tol=1e-6, maxit=1000)
    torch.cuda.synchronize()
    for (H, W, n, _), M, b in zip(cfg3, Ms, many):
        a = rp.solve(M, tol=1e-6, maxit=1000)
        torch.cuda.synchronize()
        same = torch.equal(a.L, b.L) and torch.equal(a.S, b.S)
        report(f"batch cell {H}x{W}x{n} full", it=b.iterations, it_alone=a.iterations,
               bitwise=int(same))
        assert a.iterations == b.iterations and a.status == b.status
        assert same


# -------------------------------------------------- 1024x1024 x 40 precision
@pytest.fixture(scope="module")
def cfg4():
    w = window_1024x1024x40()
    X = w.X()
    K = 5
    print("[configs] oracle: 1024x1024x40, 5 FP64 SVD iterations", flush=True)
    ref = rpca(X, tol=0.0, maxit=K)
    theta = bound_threshold(w.L_gt, w.bound_mask)
    return X, ref, theta, K


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["f32", "bf16x6", "bf16x3"])
def test_1024x1024x40_iterate_parity(cfg4, mode):
    import torch
    device()
    X, ref, theta, K = cfg4
    gm = {"f32": rp.RPCA_GRAM_DEFAULT, "bf16x6": rp.RPCA_GRAM_BF16X6,
          "bf16x3": rp.RPCA_GRAM_BF16X3}[mode]
    M = to_dev(X, np.float32)
    r = rp.solve(M, tol=0.0, maxit=K, gram_mode=gm)
    torch.cuda.synchronize()
    Lh, Sh = to_host(r.L), to_host(r.S)
    relL, relS = rel_fro(Lh, ref.L), rel_fro(Sh, ref.S)
    d = dice(Lh >= theta, ref.L >= theta)
    if mode == "bf16x3":
        barL, barS = bf16x3_budget(K, ref.L, ref.S)
    else:
        barL = barS = 1e-4
    report(f"1024x1024x40 {mode} k={K}", relL=relL, relS=relS, barL=barL, barS=barS, dice=d)
    assert r.iterations == K
    assert relL <= barL and relS <= barS
    assert d >= 0.999


# ------------------------------------------------- 512x512 x 132, iterate level
@pytest.mark.timeout(900)
def test_512x512x132_iterate_parity():
    import torch
    from synth.device import device_window
    dev = device()
    K = 3
    M = device_window(512, 512, 132, 132, dev).view(132, 512 * 512).t()
    X = to_host(M)
    print("[configs] oracle: 512x512x132, 3 FP64 SVD iterations", flush=True)
    ref = rpca(X, tol=0.0, maxit=K)
    r = rp.solve(M, tol=0.0, maxit=K)
    torch.cuda.synchronize()
    relL, relS = rel_fro(to_host(r.L), ref.L), rel_fro(to_host(r.S), ref.S)
    report(f"512x512x132 k={K}", relL=relL, relS=relS)
    assert r.iterations == K and r.status == rp.RPCA_NOT_CONVERGED
    assert relL <= 1e-4 and relS <= 1e-4
