"""Pins for the evaluation metrics (paper Sec. II-F, Eqs. 7 and 8)."""
import numpy as np
import pytest

from oracle import dice, rmse, bound_threshold, rel_fro


def test_dice_hand_examples():
    a = np.array([1, 1, 0, 0, 1], bool)
    b = np.array([1, 0, 0, 1, 1], bool)
    # |A & B| = 2, |A| = 3, |B| = 3 -> 4/6
    assert dice(a, b) == pytest.approx(2 / 3)
    assert dice(a, a) == 1.0
    assert dice(a, ~a) == 0.0
    assert dice(np.zeros(4, bool), np.zeros(4, bool)) == 1.0


def test_rmse_hand_example():
    # differences 1, -1, 2, 0 -> mean square 6/4
    assert rmse(np.array([1.0, 2, 5, 4]), np.array([0.0, 3, 3, 4])) == pytest.approx(np.sqrt(1.5))


def test_bound_threshold_is_mean_over_mask_all_frames():
    L = np.arange(2 * 2 * 3, dtype=float).reshape(3, 2, 2)   # frames of 2x2
    mask = np.array([[True, False], [False, True]])
    # entries (0,0) and (1,1) of each frame: 0,3,4,7,8,11 -> mean 5.5
    assert bound_threshold(L, mask) == pytest.approx(5.5)


def test_rel_fro():
    assert rel_fro(np.array([3.0, 4.0]), np.array([3.0, 4.0])) == 0.0
    assert rel_fro(np.array([3.0, 5.0]), np.array([3.0, 4.0])) == pytest.approx(0.2)


def test_frame_correlations_closed_forms():
    """Affine copies correlate +-1 exactly; orthogonal zero-mean frames 0."""
    from oracle import frame_correlations
    rng = np.random.default_rng(5)
    a = rng.standard_normal(50)
    b = np.where(np.arange(50) % 2 == 0, 1.0, -1.0)
    b = b - b.mean()
    a0 = a - a.mean()
    c = b - a0 * (np.dot(a0, b) / np.dot(a0, a0))       # zero mean, orthogonal to a0
    X = np.stack([a, 3.0 * a + 2.0, -0.5 * a + 7.0, c + 4.0], axis=1)
    rho = frame_correlations(X)
    assert rho[0] == pytest.approx(1.0, abs=1e-14)
    assert rho[1] == pytest.approx(-1.0, abs=1e-14)
    assert rho[2] == pytest.approx(0.0, abs=1e-14)
    const = np.stack([a, np.full(50, 3.0)], axis=1)
    assert frame_correlations(const)[0] == 0.0


def test_frame_keep_reading():
    from oracle import frame_keep
    # a single jumping frame (index 2) correlates badly with both neighbours
    rho = np.array([0.95, 0.3, 0.2, 0.97])
    assert frame_keep(rho, 0.8).tolist() == [True, True, False, True, True]
    assert frame_keep(np.array([0.1]), 0.8).tolist() == [False, False]
    assert frame_keep(np.array([]), 0.8).tolist() == [True]


def test_moving_average_closed_forms():
    from oracle import moving_average
    m, n, W = 7, 30, 20
    t = np.arange(n, dtype=np.float64)
    ramp = np.tile(2.0 * t + 1.0, (m, 1))               # column t = 2t + 1
    out = moving_average(ramp, W)
    assert out.shape == (m, n - W + 1)
    # the mean of 2t+1 over t .. t+W-1 is 2t + W
    np.testing.assert_allclose(out, np.tile(2.0 * np.arange(n - W + 1) + W, (m, 1)), rtol=0, atol=1e-12)
    const = np.full((m, n), -3.5)
    np.testing.assert_allclose(moving_average(const, W), -3.5, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(moving_average(ramp, 1), ramp)


def test_masked_mean_hand_example():
    from oracle import masked_mean
    A = np.array([[1.0, 2.0], [3.0, 10.0]])
    M = np.array([[True, False], [True, True]])
    assert masked_mean(A, M) == pytest.approx((1 + 3 + 10) / 3)
