"""Processing steps around the solve on the device, against the oracle:
frame correlation and rejection, frame selection, moving average, masked
mean, Dice and RMSE.  Counts and keep masks are compared bit for bit; sums
within FP64 rounding of the summation order (FP32 inputs are converted
exactly to FP64 on both sides)."""
import numpy as np
import pytest

from oracle import (frame_correlations, frame_keep, moving_average, masked_mean, dice, rmse,
                    rpca, bound_threshold)
from synth import make_window, batch_window
from tests.gpu_helpers import device, to_dev, to_host, report

pytestmark = pytest.mark.gpu


def _seq(seed, n=40, H=64, W=70, free=8, snr=20.0):
    """A sequence with two motion frames (shifted images, as in respiratory
    motion) among the first 40."""
    w = make_window(H, W, n, 4, free, 3, snr, seed)
    F = w.frames.copy()
    for t in (9, 27):
        if t < n:
            F[t] = np.roll(F[t], (7, -5), axis=(0, 1))
    return F.reshape(n, -1).T.copy(order="F")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_frame_correlation_and_keep(dtype):
    import paper_2506_10257_amd.postproc as pp
    device()
    # no free bubbles, 30 dB: consecutive frames correlate near 1 except the
    # two shifted frames
    X = _seq(8100, free=0, snr=30.0).astype(dtype)
    rho_ref = frame_correlations(X)
    rho = pp.frame_correlation(to_dev(X, dtype))
    err = float(np.max(np.abs(rho - rho_ref)))
    report(f"frame corr {np.dtype(dtype).name}", maxabs=err)
    assert err <= 1e-12
    keep = pp.frame_keep(rho, 0.8)
    assert keep.tolist() == frame_keep(rho_ref, 0.8).tolist()
    assert not keep[9] and not keep[27] and keep.sum() == 38


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_frame_select(dtype):
    import torch
    import paper_2506_10257_amd.postproc as pp
    device()
    X = _seq(8101, n=12).astype(dtype)
    keep = np.ones(12, dtype=bool)
    keep[[0, 5, 11]] = False
    out = pp.frame_select(to_dev(X, dtype), keep)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), X[:, keep].astype(np.float64))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("W", [1, 5, 20])
def test_moving_average(dtype, W):
    import paper_2506_10257_amd.postproc as pp
    device()
    X = _seq(8102 + W, n=45).astype(dtype)
    ref = moving_average(X, W)
    out = to_host(pp.moving_average(to_dev(X, dtype), W))
    err = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
    report(f"moving average W={W} {np.dtype(dtype).name}", rel=err)
    assert err <= (1e-13 if dtype == np.float64 else 2e-7)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dice_rmse_masked_mean_on_a_solve(dtype):
    """The paper's evaluation of an RPCA result (Sec. II-F): threshold = mean
    of the ground-truth L at the bound bubbles, Dice of the binarised L
    series, RMSE of L and S."""
    import torch
    import paper_2506_10257_amd as rp
    import paper_2506_10257_amd.postproc as pp
    device()
    w = batch_window(64, 64, 20, 8200)
    X = w.X()
    r = rp.solve(to_dev(X, dtype), tol=1e-6, maxit=500)
    L, S = to_host(r.L), to_host(r.S)
    Lgt, Sgt = w.X() * 0 + w.L_gt.reshape(20, -1).T, w.S_gt.reshape(20, -1).T
    mask = np.repeat(w.bound_mask.reshape(1, -1), 20, axis=0).T
    theta_ref = bound_threshold(w.L_gt, w.bound_mask)
    theta = pp.masked_mean(to_dev(Lgt, dtype),
                           torch.from_numpy(np.ascontiguousarray(mask.T.astype(np.uint8))).cuda().t())
    assert theta == pytest.approx(masked_mean(Lgt.astype(dtype), mask), rel=1e-12)
    report(f"threshold {np.dtype(dtype).name}", theta=theta, theta_ref=theta_ref)
    Ld, Lgtd = to_dev(L, dtype), to_dev(Lgt, dtype)
    d, counts = pp.dice(Ld, theta, Lgtd, theta)
    a = L.astype(dtype).astype(np.float64) >= theta
    b = Lgt.astype(dtype).astype(np.float64) >= theta
    assert counts == (int((a & b).sum()), int(a.sum()), int(b.sum()))
    assert d == dice(a, b)
    e = pp.rmse(to_dev(S, dtype), to_dev(Sgt, dtype))
    e_ref = rmse(S.astype(dtype), Sgt.astype(dtype))
    report(f"dice/rmse {np.dtype(dtype).name}", dice=d, rmse=e)
    assert e == pytest.approx(e_ref, rel=1e-12)
