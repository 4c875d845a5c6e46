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
