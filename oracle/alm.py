"""Plain FP64 CPU oracle of the paper's RPCA solve (inexact ALM / ADMM on PCP).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product path never does; it shares no code with it.

Follows the paper, Sec. II-A:

* problem (Eq. 2): minimise ||L||_* + lam ||S||_1 subject to L + S = X;
* augmented Lagrangian (Eq. 3) minimised by repeating three steps:
  1. L-step (Eq. 4): L = D_{1/mu}(X - S + Y/mu), singular value thresholding
     D_tau(M) = U max(Lambda - tau, 0) V^*, here with a full thin LAPACK SVD;
  2. S-step (Eq. 5): S = shrink_{lam/mu}(X - L + Y/mu) with
     shrink_g(x) = sgn(x) max(|x| - g, 0);
  3. dual step (Eq. 6): Y = Y + mu (X - L - S), with the L and S just computed;
* penalty mu = n1 n2 / (4 ||X||_1), n1 n2 the number of entries of X and
  ||X||_1 the entrywise sum of |X_ij| (Sec. II-A, after Eq. 6), kept fixed;
* stop when ||X - L - S||_F < delta ||X||_F (Sec. II-A, after Eq. 6).

Readings where the paper is silent (stated once here, listed with the others
in the design notes): lam defaults to 1/sqrt(max(m, n)); S and Y start at 0;
the stopping test is strict and is made after the dual step; tol <= 0 runs
exactly maxit iterations; sgn(0) = 0; sum(|X|) == 0 returns L = S = 0 after 0
iterations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

OK = 0
NOT_CONVERGED = 1
ERR_ARG = -1
ERR_NONFINITE = -4


@dataclass
class Result:
    L: np.ndarray
    S: np.ndarray
    Y: np.ndarray
    iterations: int
    status: int
    residual: float          # ||X - L - S||_F / ||X||_F at return
    lam: float
    mu: float
    history: list = field(default_factory=list)   # relative residual per iteration


def shrink(x: np.ndarray, gamma: float) -> np.ndarray:
    """Eq. 5 shrinkage operator, entrywise: sgn(x) * max(|x| - gamma, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - gamma, 0.0)


def svt(M: np.ndarray, tau: float) -> np.ndarray:
    """Eq. 4 singular value thresholding D_tau(M) = U max(Lambda - tau, 0) V^*.

    Full thin SVD from LAPACK (gesdd, falling back to gesvd if it fails).
    """
    try:
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        U, s, Vt = scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")
    w = np.maximum(s - tau, 0.0)
    return (U * w) @ Vt


def default_lambda(m: int, n: int) -> float:
    """Sparsity weight 1/sqrt(max(m, n)) (the value used by the PCP work the
    paper cites for Eq. 2; the paper itself gives no number)."""
    return 1.0 / np.sqrt(float(max(m, n)))


def default_mu(X: np.ndarray) -> float:
    """mu = n1 n2 / (4 ||X||_1), ||X||_1 = sum_ij |X_ij| (Sec. II-A)."""
    m, n = X.shape
    return float(m) * float(n) / (4.0 * float(np.sum(np.abs(X))))


def l_step(X: np.ndarray, S: np.ndarray, Y: np.ndarray, mu: float) -> np.ndarray:
    """Step 1, Eq. 4: L = D_{1/mu}(X - S + Y/mu)."""
    return svt(X - S + Y / mu, 1.0 / mu)


def s_step(X: np.ndarray, L: np.ndarray, Y: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """Step 2, Eq. 5: S = shrink_{lam/mu}(X - L + Y/mu)."""
    return shrink(X - L + Y / mu, lam / mu)


def dual_step(Y: np.ndarray, X: np.ndarray, L: np.ndarray, S: np.ndarray, mu: float) -> np.ndarray:
    """Step 3, Eq. 6: Y + mu (X - L - S) with the L and S just computed."""
    return Y + mu * (X - L - S)


def converged(rel: float, tol: float) -> bool:
    """Stopping test after Eq. 6: ||X - L - S||_F < delta ||X||_F (strict)."""
    return rel < tol


def rpca(X: np.ndarray, lam: Optional[float] = None, mu: Optional[float] = None,
         tol: float = 1e-7, maxit: int = 500,
         S0: Optional[np.ndarray] = None, Y0: Optional[np.ndarray] = None,
         callback: Optional[Callable[[int, np.ndarray, np.ndarray, np.ndarray], None]] = None,
         ) -> Result:
    """Inexact-ALM RPCA of X (m x n) in float64, steps in the order of Sec. II-A.

    lam, mu: None or <= 0 selects the defaults.  tol <= 0: exactly maxit
    iterations.  S0, Y0: optional starting S and Y (default zero).
    callback(k, L, S, Y) is called after every iteration (for invariant tests).
    """
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] < 1 or X.shape[1] < 1 or maxit < 1:
        raise ValueError("X must be a non-empty 2-D matrix and maxit >= 1")
    m, n = X.shape
    if not np.all(np.isfinite(X)):
        z = np.zeros_like(X)
        return Result(z, z.copy(), z.copy(), 0, ERR_NONFINITE, float("nan"), float("nan"), float("nan"))
    if lam is None or lam <= 0:
        lam = default_lambda(m, n)
    nX1 = float(np.sum(np.abs(X)))
    nXF = float(np.linalg.norm(X, "fro"))
    if nX1 == 0.0:
        z = np.zeros_like(X)
        return Result(z, z.copy(), z.copy(), 0, OK, 0.0, float(lam), float("nan"))
    if mu is None or mu <= 0:
        mu = default_mu(X)
    lam = float(lam)
    mu = float(mu)

    S = np.zeros_like(X) if S0 is None else np.array(S0, dtype=np.float64)
    Y = np.zeros_like(X) if Y0 is None else np.array(Y0, dtype=np.float64)
    L = np.zeros_like(X)
    history = []
    for k in range(1, maxit + 1):
        L = l_step(X, S, Y, mu)                       # Eq. 4
        S = s_step(X, L, Y, lam, mu)                  # Eq. 5
        Y = dual_step(Y, X, L, S, mu)                 # Eq. 6, new L and S
        rel = float(np.linalg.norm(X - L - S, "fro")) / nXF
        history.append(rel)
        if callback is not None:
            callback(k, L, S, Y)
        if converged(rel, tol):                       # after the dual step
            return Result(L, S, Y, k, OK, rel, lam, mu, history)
    return Result(L, S, Y, maxit, NOT_CONVERGED, history[-1], lam, mu, history)
