"""The per-product constant of the split-BF16 error budget
(tests/bf16_budget.py), checked by emulating the split on the CPU."""
import numpy as np

from tests.bf16_budget import C2, EPS, to_bf16


def test_to_bf16_rounds_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -2.5], np.float32)
    got = to_bf16(x)
    assert list(got) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5]


def test_split_product_error_within_c2():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    y = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    hx = to_bf16(x)
    lx = to_bf16(x - hx)
    hy = to_bf16(y)
    ly = to_bf16(y - hy)
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    approx = (hx.astype(np.float64) * hy + hx.astype(np.float64) * ly + lx.astype(np.float64) * hy)
    rel = np.abs(xd * yd - approx) / (np.abs(xd) * np.abs(yd))
    assert rel.max() <= C2
    assert rel.max() >= C2 / 16        # the constant is not vacuous
    assert C2 <= EPS - 144 * 2.0 ** -24  # room for the FP32 accumulation
    # the three-way split with six products is about FP32 rounding
    mx = to_bf16(x - hx)
    rx = to_bf16(x - hx - mx)
    my = to_bf16(y - hy)
    ry = to_bf16(y - hy - my)
    six = (hx.astype(np.float64) * hy + hx.astype(np.float64) * my + mx.astype(np.float64) * hy
           + hx.astype(np.float64) * ry + mx.astype(np.float64) * my + rx.astype(np.float64) * hy)
    rel6 = np.abs(xd * yd - six) / (np.abs(xd) * np.abs(yd))
    assert rel6.max() <= 4 * 2.0 ** -24
