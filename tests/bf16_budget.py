"""Error budget of the split-BF16 contraction mode with two terms (BF16x3),
derived from its arithmetic.

Split: x = h + l + d with h = bf16(x), l = bf16(x - h) (round to nearest), so
|x - h| <= 2^-8 |x|, |d| <= 2^-8 |x - h| <= 2^-16 |x|.  The mode forms
h h' + h l' + l h' and drops l l' and the d terms:

    x y - (h h' + h l' + l h') = l l' + (h + l) d' + d (h' + l') + d d',

so one product is off by at most C2 |x||y| with
C2 = 2^-16 ((1 + 2^-8)^2 + 2 (1 + 2^-16) + 2^-16) ~ 3.008 * 2^-16.  The
products of BF16 values are exact in FP32; the FP32 accumulation over at most
K = 144 terms (the longest contraction: 64-row Gram tiles, rebuilds of up to
144 frames) adds at most K 2^-24 = 0.56 * 2^-16 relative to the sum of |terms|.
Per contraction the relative error is therefore below EPS = 2^-14 (4 * 2^-16).

Propagation (first order): the rebuild L = A P and the Gram A^T A of one
iteration each carry at most EPS relative to the sums of |terms|.  The ALM
iteration with a fixed penalty is non-expansive, so to first order the
perturbations of k iterations add up: ||dL||_F <= k EPS ||L||_F.  The shrink
of Eq. 5 is 1-Lipschitz, so ||dS||_F <= ||dL||_F, i.e.
relS <= k EPS ||L||_F / ||S||_F.  The budget ignores the amplification by the
thresholding's sensitivity to eigenvalues near tau and the cancellation in
sums of mixed signs; the measured errors stay well inside it.
"""
import numpy as np

C2 = 2.0 ** -16 * ((1 + 2.0 ** -8) ** 2 + 2 * (1 + 2.0 ** -16) + 2.0 ** -16)
EPS = 2.0 ** -14


def bf16x3_budget(k: int, L_ref: np.ndarray, S_ref: np.ndarray) -> tuple[float, float]:
    """(relL, relS) bounds after k iterations, from the oracle's L and S."""
    relL = k * EPS
    return relL, relL * float(np.linalg.norm(L_ref)) / float(np.linalg.norm(S_ref))


def to_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)
