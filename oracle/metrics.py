"""Evaluation metrics of the paper (Sec. II-F) and the comparison measures.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only tests, the smoke check
and the CPU-baseline leg of the benchmark use it.

* RMSE (Eq. 7): sqrt of the mean squared difference over all samples and frames.
* Dice (Eq. 8): 2 |C & C^| / (|C| + |C^|) of two binary masks.
* Binarisation (Sec. II-F): threshold = mean intensity of the ground-truth
  image at the bound-bubble locations.  No histogram matching is applied (the
  GPU result and the oracle are compared on the same threshold).
"""
from __future__ import annotations

import numpy as np


def rmse(est: np.ndarray, ref: np.ndarray) -> float:
    """Eq. 7 over every entry (all pixels, all frames)."""
    d = np.asarray(est, dtype=np.float64) - np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d)))


def dice(a: np.ndarray, b: np.ndarray) -> float:
    """Eq. 8.  Two empty masks agree perfectly (Dice 1)."""
    a = np.asarray(a, dtype=bool)
    b = np.asarray(b, dtype=bool)
    den = int(a.sum()) + int(b.sum())
    if den == 0:
        return 1.0
    return 2.0 * float(np.logical_and(a, b).sum()) / float(den)


def bound_threshold(L_gt_frames: np.ndarray, bound_mask: np.ndarray) -> float:
    """Mean of the ground-truth low-rank series over the bound-bubble pixels
    (all frames): the binarisation threshold of Sec. II-F."""
    sel = np.broadcast_to(bound_mask[None], L_gt_frames.shape)
    return float(L_gt_frames[sel].mean())


def bound_mask_series(L: np.ndarray, theta: float) -> np.ndarray:
    """Binary series: entries of L (any layout) at or above theta."""
    return np.asarray(L) >= theta


def rel_fro(est: np.ndarray, ref: np.ndarray) -> float:
    """||est - ref||_F / ||ref||_F (0/0 counts as 0)."""
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.linalg.norm(ref))
    num = float(np.linalg.norm(est - ref))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


# --------------------------------------------------- steps around the solve
def frame_correlations(X: np.ndarray) -> np.ndarray:
    """Pearson correlation of consecutive frames (columns) t, t+1 of the
    Casorati matrix X (m x n), t = 0 .. n-2; a frame with zero variance gives
    0.  Used to drop frames that correlate poorly with their neighbours
    (the paper's in vivo reference, Sec. III)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros(X.shape[1] - 1)
    for t in range(X.shape[1] - 1):
        a = X[:, t] - X[:, t].mean()
        b = X[:, t + 1] - X[:, t + 1].mean()
        den = np.sqrt(np.dot(a, a) * np.dot(b, b))
        out[t] = np.dot(a, b) / den if den > 0 else 0.0
    return out


def frame_keep(rho: np.ndarray, threshold: float = 0.8) -> np.ndarray:
    """Reading of the frame rejection: frame t is kept when it correlates at
    least `threshold` with one of its neighbours (the larger of rho[t-1] and
    rho[t] where they exist)."""
    n = len(rho) + 1
    keep = np.zeros(n, dtype=bool)
    for t in range(n):
        nb = []
        if t > 0:
            nb.append(rho[t - 1])
        if t + 1 < n:
            nb.append(rho[t])
        keep[t] = (not nb) or max(nb) >= threshold
    return keep


def moving_average(X: np.ndarray, W: int) -> np.ndarray:
    """Temporal moving average over W frames, 'valid' part: column t is the
    mean of columns t .. t+W-1 (Sec. III, 20-frame window)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]
    return np.stack([X[:, t:t + W].mean(axis=1) for t in range(n - W + 1)], axis=1)


def masked_mean(A: np.ndarray, mask: np.ndarray) -> float:
    """Mean of A over the entries where mask is set (binarisation threshold,
    Sec. II-F)."""
    A = np.asarray(A, dtype=np.float64)
    return float(A[np.asarray(mask, dtype=bool)].mean())
