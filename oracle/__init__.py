"""CPU FP64 oracle of the RPCA hot path.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package.  It shares no code with the HIP path.
"""
from .alm import (OK, NOT_CONVERGED, ERR_ARG, ERR_NONFINITE, Result, shrink, svt,
                   default_lambda, default_mu, rpca)
from .metrics import (rmse, dice, bound_threshold, bound_mask_series, rel_fro,
                      frame_correlations, frame_keep, moving_average, masked_mean)

__all__ = ["OK", "NOT_CONVERGED", "ERR_ARG", "ERR_NONFINITE", "Result", "shrink", "svt",
           "default_lambda", "default_mu", "rpca", "rmse", "dice", "bound_threshold",
           "bound_mask_series", "rel_fro", "frame_correlations", "frame_keep",
           "moving_average", "masked_mean"]
