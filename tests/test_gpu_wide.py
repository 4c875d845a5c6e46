"""Windows of 65-144 frames (MFMA tile streaming kernel and the in-place
eigensolver; above 112 frames its eigenvectors stay in device memory), the
tile kernel on the smaller frame classes, and the split-BF16 precision
variants, against the FP64 oracle.

Bars as for the other FP32 paths: relative Frobenius error <= 1e-4 in L and
S, iterations within one, Dice >= 0.999 on the bound-bubble mask.  The
two-way split-BF16 mode carries a larger contraction error; it is held to the
error budget derived from its arithmetic (tests/bf16_budget.py).
"""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro, dice, bound_threshold
from synth import batch_window
from tests.bf16_budget import bf16x3_budget
from tests.gpu_helpers import device, to_dev, to_host, report

pytestmark = pytest.mark.gpu


def _solve(X, gram_mode=rp.RPCA_GRAM_DEFAULT, tol=1e-6, maxit=300):
    M = to_dev(X, np.float32)
    r = rp.solve(M, tol=tol, maxit=maxit, gram_mode=gram_mode)
    return to_host(r.L), to_host(r.S), r.iterations, r.status


def _check(name, w, ref, L, S, it, bar=1e-4, it_slack=1):
    theta = bound_threshold(w.L_gt, w.bound_mask)
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    d = dice(L >= theta, ref.L >= theta)
    report(name, it=it, it_ref=ref.iterations, relL=eL, relS=eS, dice=d)
    assert abs(it - ref.iterations) <= it_slack
    assert eL <= bar and eS <= bar
    assert d >= 0.999
    return eL, eS, d


# (H, W, n): ragged row counts (not a multiple of the 64-row tile), odd and
# even frame counts, every wide class (80, 96, 112, 128, 144) and its edges;
# 113-144 frames run the eigensolver with V in device memory (113-136 with
# the rotations accumulated as an FP32 increment in LDS, 137-144 rotating V
# in place), 132 is the paper's reference window length.
WIDE = [(48, 48, 65), (50, 47, 80), (40, 60, 81), (48, 49, 99), (44, 50, 100), (40, 52, 112),
        (40, 41, 113), (36, 40, 120), (32, 40, 128), (40, 40, 129), (44, 40, 132), (38, 40, 136),
        (36, 38, 137), (40, 37, 144)]


@pytest.mark.parametrize("H,W,n", WIDE)
def test_wide_fp32_matches_oracle(H, W, n):
    device()
    w = batch_window(H, W, n, 7000 + n)
    X = w.X()
    ref = rpca(X, tol=1e-6, maxit=300)
    L, S, it, rc = _solve(X)
    _check(f"wide {H}x{W}x{n}", w, ref, L, S, it)


@pytest.mark.parametrize("n", [100, 132, 140])
@pytest.mark.parametrize("k", [1, 2, 7, 60])
def test_wide_iterate_parity(n, k):
    """Fixed iteration counts (tol = 0): the k-th iterate against the oracle's
    (k >= 2 runs the eigensolver's warm start; k = 60 checks that the
    rounding of the eigenvector updates does not build up over the warm
    starts)."""
    device()
    w = batch_window(40, 40, n, 7101 + n)
    X = w.X()
    ref = rpca(X, tol=0.0, maxit=k)
    L, S, it, rc = _solve(X, tol=0.0, maxit=k)
    assert it == k and rc == rp.RPCA_NOT_CONVERGED
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    report(f"wide iterate n={n} k={k}", relL=eL, relS=eS)
    assert eL <= 1e-5 and eS <= 1e-5


@pytest.mark.parametrize("n", [10, 20, 40, 64])
def test_tile_kernel_on_register_classes(n):
    """The MFMA tile kernel selected for a class the register kernel also serves."""
    device()
    K = rp.RPCA_KNOB_STREAM_KERNEL
    cls = next(c for c in (4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60, 64) if c >= n)
    w = batch_window(64, 72, n, 7200 + n)
    X = w.X()
    ref = rpca(X, tol=1e-6, maxit=300)
    old = rp.rpca_tune_get(K, rp.RPCA_F32, cls)
    try:
        assert rp.rpca_tune_set(K, rp.RPCA_F32, cls, 1) == rp.RPCA_OK
        L, S, it, rc = _solve(X)
    finally:
        rp.rpca_tune_set(K, rp.RPCA_F32, cls, old)
    _check(f"tile kernel n={n}", w, ref, L, S, it)


def test_zero_input_wide():
    import torch
    device()
    M = torch.zeros((100, 3000), device="cuda").t()
    r = rp.solve(M, tol=1e-6, maxit=10)
    assert r.status == rp.RPCA_OK and r.iterations == 0
    assert bool((r.L == 0).all()) and bool((r.S == 0).all())


def test_wide_batch_bitwise_equals_alone():
    import torch
    device()
    # 113 and 132 frames take the eigensolver's FP32 increment path, 140 the
    # in-place path, in the same 144-frame eigensolve launch
    shapes = [(40, 40, 100), (32, 48, 20), (48, 40, 80), (30, 30, 112), (64, 64, 10), (40, 44, 132),
              (36, 36, 113), (36, 40, 140)]
    Ms = [to_dev(batch_window(H, W, n, 7300 + i).X(), np.float32) for i, (H, W, n) in enumerate(shapes)]
    alone = [rp.solve(M, tol=1e-6, maxit=200) for M in Ms]
    many = rp.solve_many(Ms, tol=1e-6, maxit=200)
    torch.cuda.synchronize()
    for a, b in zip(alone, many):
        assert a.iterations == b.iterations
        assert torch.equal(a.L, b.L) and torch.equal(a.S, b.S)


@pytest.mark.parametrize("H,W,n", [(64, 64, 40), (48, 50, 100), (44, 40, 132)])
def test_bf16x3_within_budget(H, W, n):
    """Two-way split BF16 contractions against the error budget derived from
    the split (tests/bf16_budget.py): at iterate level k = 5, and for the full
    solve with k = its iteration count."""
    device()
    w = batch_window(H, W, n, 7400 + n)
    X = w.X()
    theta = bound_threshold(w.L_gt, w.bound_mask)
    K = 5
    ref = rpca(X, tol=0.0, maxit=K)
    L, S, it, rc = _solve(X, gram_mode=rp.RPCA_GRAM_BF16X3, tol=0.0, maxit=K)
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    bL, bS = bf16x3_budget(K, ref.L, ref.S)
    report(f"bf16x3 {H}x{W}x{n} k={K}", relL=eL, relS=eS, budgetL=bL, budgetS=bS)
    assert it == K and eL <= bL and eS <= bS
    ref = rpca(X, tol=1e-6, maxit=300)
    L, S, it, rc = _solve(X, gram_mode=rp.RPCA_GRAM_BF16X3)
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    bL, bS = bf16x3_budget(max(it, ref.iterations), ref.L, ref.S)
    d = dice(L >= theta, ref.L >= theta)
    report(f"bf16x3 {H}x{W}x{n}", it=it, it_ref=ref.iterations, relL=eL, relS=eS,
           budgetL=bL, budgetS=bS, dice=d)
    assert eL <= bL and eS <= bS


def test_precision_window_fp32_and_bf16x3():
    """A scaled-down window of the 1024x1024x40 precision workload (same
    density and 15 dB SNR): FP32 within the bar, split-BF16 within its
    budget."""
    from synth import make_window, density_counts
    device()
    nb, nf, nv = density_counts(128, 128)
    w = make_window(128, 128, 40, nb, nf, nv, 15.0, 7501)
    X = w.X()
    ref = rpca(X, tol=1e-6, maxit=1000)
    L, S, it, rc = _solve(X, tol=1e-6, maxit=1000)
    _check("precision 128x128x40 f32", w, ref, L, S, it)
    L, S, it, rc = _solve(X, gram_mode=rp.RPCA_GRAM_BF16X3, tol=1e-6, maxit=1000)
    theta = bound_threshold(w.L_gt, w.bound_mask)
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    bL, bS = bf16x3_budget(max(it, ref.iterations), ref.L, ref.S)
    d = dice(L >= theta, ref.L >= theta)
    report("precision 128x128x40 bf16x3", it=it, it_ref=ref.iterations, relL=eL, relS=eS,
           budgetL=bL, budgetS=bS, dice=d)
    assert eL <= bL and eS <= bS and d >= 0.999


@pytest.mark.parametrize("H,W,n", [(128, 128, 40), (48, 50, 100), (64, 72, 20), (44, 40, 132)])
def test_bf16x6_meets_fp32_bar(H, W, n):
    """Three-way split BF16 contractions (six products): held to the FP32 bar."""
    from synth import make_window, density_counts
    device()
    nb, nf, nv = density_counts(H, W)
    w = make_window(H, W, n, nb, nf, nv, 15.0, 7600 + n)
    X = w.X()
    ref = rpca(X, tol=1e-6, maxit=1000)
    L, S, it, rc = _solve(X, gram_mode=rp.RPCA_GRAM_BF16X6, tol=1e-6, maxit=1000)
    _check(f"bf16x6 {H}x{W}x{n}", w, ref, L, S, it)


# FP64 solves of 33 to 128 frames: the FP64 tile kernel (both contractions on
# the f64 matrix cores) and, above 64 frames, the in-place eigensolver with a
# Newton-Schulz re-orthonormalisation of its warm start.  Held to the FP64
# bar: 1e-10 in L and S with the same iteration count and status.
FP64_WIDE = [(40, 38, 33), (48, 50, 40), (40, 41, 60), (36, 30, 64), (40, 44, 65), (36, 44, 81),
             (40, 40, 96), (38, 40, 97), (44, 50, 100), (40, 37, 112), (36, 40, 113), (32, 41, 128)]


def _solve64(X, tol=1e-7, maxit=300):
    M = to_dev(X, np.float64)
    r = rp.solve(M, tol=tol, maxit=maxit)
    return to_host(r.L), to_host(r.S), r.iterations, r.status


@pytest.mark.parametrize("H,W,n", FP64_WIDE)
def test_wide_fp64_matches_oracle(H, W, n):
    device()
    w = batch_window(H, W, n, 7700 + n)
    X = w.X()
    ref = rpca(X, tol=1e-7, maxit=300)
    L, S, it, rc = _solve64(X)
    _check(f"wide fp64 {H}x{W}x{n}", w, ref, L, S, it, bar=1e-10, it_slack=0)
    assert rc == ref.status


@pytest.mark.parametrize("n", [33, 60, 96, 100, 128])
@pytest.mark.parametrize("k", [1, 2, 7])
def test_wide_fp64_iterate_parity(n, k):
    """k-th iterate (tol = 0); k >= 2 runs the warm start with the
    Newton-Schulz step."""
    device()
    X = batch_window(40, 44, n, 7800 + n).X()
    ref = rpca(X, tol=0.0, maxit=k)
    L, S, it, rc = _solve64(X, tol=0.0, maxit=k)
    eL, eS = rel_fro(L, ref.L), rel_fro(S, ref.S)
    report(f"wide fp64 iterate n={n} k={k}", relL=eL, relS=eS)
    assert it == k and eL <= 1e-10 and eS <= 1e-10


def test_wide_fp64_batch_bitwise_equals_alone():
    import torch
    device()
    shapes = [(40, 40, 100), (32, 48, 20), (48, 40, 40), (30, 30, 128), (64, 64, 10), (36, 36, 70)]
    Ms = [to_dev(batch_window(H, W, n, 7900 + i).X(), np.float64) for i, (H, W, n) in enumerate(shapes)]
    alone = [rp.solve(M, tol=1e-7, maxit=200) for M in Ms]
    many = rp.solve_many(Ms, tol=1e-7, maxit=200)
    torch.cuda.synchronize()
    for a, b in zip(alone, many):
        assert a.iterations == b.iterations
        assert torch.equal(a.L, b.L) and torch.equal(a.S, b.S)


def test_fp64_above_128_frames_unsupported():
    import torch
    device()
    M = torch.ones((129, 64), dtype=torch.float64, device="cuda:0").t()
    L, S = torch.empty_like(M), torch.empty_like(M)
    rc, it = rp.rpca_solve_f64(M, 64, 129, -1.0, -1.0, 1e-7, 10, L, S)
    assert rc == rp.RPCA_ERR_UNSUPPORTED and it == 0
