"""The oracle's pins must catch plausible mistakes.

Each mutant below plants one mistake in the oracle (on the CPU, by patching
a step of the loop); the fast pins of test_oracle_pins.py are then run against
the mutated oracle and at least one of them has to fail.
"""
import numpy as np
import pytest

import oracle.alm as O
from tests import test_oracle_pins as P

_orig = {name: getattr(O, name) for name in
         ("shrink", "svt", "l_step", "s_step", "dual_step", "converged",
          "default_mu", "default_lambda", "rpca")}


def _svt_no_clamp(M, tau):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    return (U * (s - tau)) @ Vt


def _svt_tau_squared(M, tau):
    return _orig["svt"](M, tau * tau)


def _svt_transposed(M, tau):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    w = np.maximum(s - tau, 0.0)
    return ((U * w) @ Vt).T.reshape(M.shape)


def _dual_stale():
    """Eq. 6 with the L and S of the previous iteration (zero before the
    first), instead of the ones just computed."""
    prev = {}

    def dual(Y, X, L, S, mu):
        Lp, Sp = prev.get("L"), prev.get("S")
        if Lp is None or Lp.shape != L.shape:
            Lp, Sp = np.zeros_like(L), np.zeros_like(S)
        prev["L"], prev["S"] = L, S
        return Y + mu * (X - Lp - Sp)
    return dual


def _iters_off_by_one(*args, **kw):
    """The iteration count reported one too high (counting from zero)."""
    r = _orig["rpca"](*args, **kw)
    if r.iterations > 0:
        r.iterations += 1
    return r


MUTANTS = {
    # Eq. 4
    "L_step_minus_Y": lambda X, S, Y, mu: _orig["svt"](X - S - Y / mu, 1.0 / mu),
    "L_step_tau_mu": lambda X, S, Y, mu: _orig["svt"](X - S + Y / mu, mu),
    "L_step_plus_S": lambda X, S, Y, mu: _orig["svt"](X + S + Y / mu, 1.0 / mu),
    "L_step_drop_Y": lambda X, S, Y, mu: _orig["svt"](X - S, 1.0 / mu),
    "svt_no_clamp": _svt_no_clamp,
    "svt_tau_squared": _svt_tau_squared,
    "svt_transposed": _svt_transposed,
    # Eq. 5
    "S_step_gamma_lam_mu": lambda X, L, Y, lam, mu: _orig["shrink"](X - L + Y / mu, lam * mu),
    "S_step_drop_Y": lambda X, L, Y, lam, mu: _orig["shrink"](X - L, lam / mu),
    "S_step_minus_Y": lambda X, L, Y, lam, mu: _orig["shrink"](X - L - Y / mu, lam / mu),
    "shrink_no_sign": lambda x, g: np.maximum(np.abs(x) - g, 0.0),
    "shrink_no_clamp": lambda x, g: np.sign(x) * (np.abs(x) - g),
    "shrink_hard_threshold": lambda x, g: np.where(np.abs(x) > g, x, 0.0),
    # Eq. 6
    "dual_minus": lambda Y, X, L, S, mu: Y - mu * (X - L - S),
    "dual_drop_S": lambda Y, X, L, S, mu: Y + mu * (X - L),
    "dual_over_mu": lambda Y, X, L, S, mu: Y + (X - L - S) / mu,
    "dual_stale_L_S": _dual_stale(),
    # stopping rule and defaults
    "stop_not_strict": lambda rel, tol: rel <= tol,
    "mu_frame_dims": lambda X: float(X.shape[0]) / (4.0 * float(np.sum(np.abs(X)))),
    "mu_fro_norm": lambda X: float(X.size) / (4.0 * float(np.linalg.norm(X))),
    "lambda_min_dim": lambda m, n: 1.0 / np.sqrt(float(min(m, n))),
    "iters_off_by_one": _iters_off_by_one,
}

TARGET = {
    "L_step": "l_step", "S_step": "s_step", "svt": "svt", "shrink": "shrink",
    "dual": "dual_step", "stop": "converged", "mu": "default_mu", "lambda": "default_lambda",
    "iters": "rpca",
}


def _pins(_unused):
    """The fast pins, as zero-argument callables."""
    return [
        P.test_shrink_special_values,
        P.test_default_mu_and_lambda_formulas,
        lambda: P.test_hand_worked_iterates("diag_2x2"),
        lambda: P.test_hand_worked_iterates("diag_2x2_mu2"),
        lambda: P.test_hand_worked_iterates("rank1_3x2"),
        P.test_hand_worked_stopping_iteration,
        P.test_tol_nonpositive_runs_exactly_maxit,
        P.test_shrink_matches_brute_force_4x3,
        lambda: P.test_svt_kkt_certificate_4x3(0.9),
        lambda: P.test_svt_kkt_certificate_4x3(2.5),
        P.test_svt_no_descent_direction,
        P.test_dual_bound_and_sign_invariant_every_iteration,
        lambda: P.test_planted_recovery(2000, 40, 1, 0.05, 7),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    prefix = next(k for k in TARGET if name.startswith(k))
    attr = TARGET[prefix]
    monkeypatch.setattr(O, attr, MUTANTS[name])
    if hasattr(P, attr):
        monkeypatch.setattr(P, attr, MUTANTS[name])
    caught = False
    for pin in _pins(None):          # cheapest first; one failure is enough
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, KeyError, ValueError, IndexError, np.linalg.LinAlgError):
            caught = True
            break
    assert caught, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_all_fast_pins():
    for pin in _pins(None):
        pin()
