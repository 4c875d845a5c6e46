"""Write tests/golden/oracle_512x512x20.npz: the FP64 oracle's full solve of
the seeded 512x512 x 20 window (lambda = 1/512, tol = 1e-6, maxit = 1000).

Calls only oracle/ and synth/.  The full solve takes minutes on the CPU, too
long to repeat inside a GPU test, so the test compares against this summary:
iteration count, status, residual, Frobenius norms, 8192 sampled entries of L
and S, and the complete thresholded bound-bubble mask of L (packed bits).

Run from the repository root:  python tests/golden/make_oracle_summaries.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rpca, bound_threshold          # noqa: E402
from synth import window_512x512x20                # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_512x512x20.npz")


def main():
    w = window_512x512x20()
    X = w.X()
    m, n = X.shape
    r = rpca(X, lam=1.0 / 512.0, tol=1e-6, maxit=1000)
    theta = bound_threshold(w.L_gt, w.bound_mask)
    mask = (r.L >= theta)
    rng = np.random.default_rng(0)
    idx = rng.choice(m * n, size=8192, replace=False)
    Lf = r.L.ravel(order="F")
    Sf = r.S.ravel(order="F")
    np.savez_compressed(
        OUT, iterations=r.iterations, status=r.status, residual=r.residual, mu=r.mu, lam=r.lam,
        L_fro=np.linalg.norm(r.L), S_fro=np.linalg.norm(r.S), theta=theta,
        sample_idx=idx, L_sample=Lf[idx], S_sample=Sf[idx],
        mask_bits=np.packbits(mask.ravel(order="F")), m=m, n=n,
        history=np.asarray(r.history))
    print(f"iterations {r.iterations} status {r.status} residual {r.residual:.3e} -> {OUT}")


if __name__ == "__main__":
    main()
