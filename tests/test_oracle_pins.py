"""Pins for the CPU oracle: each check is fixed by the paper or by mathematics,
never by re-running the oracle's own formula.

Paper: Sec. II-A, Eqs. 2-6 and the mu / stopping paragraph after Eq. 6.
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

import oracle
from oracle import rpca, shrink, svt, default_lambda, default_mu, rel_fro
from synth import planted_low_rank_sparse, window_128x128x20

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


# ---------------------------------------------------------------- brute force
def _brute_scalar(fun, centre, width):
    """Minimise a 1-D convex function: dense grid, then bounded Brent."""
    grid = np.linspace(centre - width, centre + width, 4001)
    vals = np.array([fun(g) for g in grid])
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    if hi <= lo:
        return grid[i]
    r = minimize_scalar(fun, bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-13, "maxiter": 500})
    return r.x if r.fun <= vals[i] else grid[i]


def _nuclear(M):
    return float(np.sum(np.linalg.svd(M, compute_uv=False)))


def _bm_minimise(obj_of_L, m, n, rng, restarts=6):
    """Burer-Monteiro brute force: minimise g(L) + ||L||_* over L = P Q^T using
    ||L||_* = min (||P||^2 + ||Q||^2) / 2.  Returns the best L found."""
    k = min(m, n)
    best, best_val = None, np.inf

    def f(v):
        P = v[: m * k].reshape(m, k)
        Q = v[m * k:].reshape(n, k)
        return 0.5 * (np.sum(P * P) + np.sum(Q * Q)) + obj_of_L(P @ Q.T)

    for _ in range(restarts):
        v0 = rng.standard_normal(m * k + n * k)
        r = minimize(f, v0, method="BFGS", options={"gtol": 1e-12, "maxiter": 20000})
        if r.fun < best_val:
            best_val = r.fun
            P = r.x[: m * k].reshape(m, k)
            Q = r.x[m * k:].reshape(n, k)
            best = P @ Q.T
    return best


# ------------------------------------------------------------- Eq. 5 (prox l1)
def test_shrink_matches_brute_force_4x3():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((4, 3)) * 2.0
    X[0, 0] = 0.0
    X[1, 1] = 0.7            # exactly at the threshold below
    for g in (0.0, 0.3, 0.7, 1.5):
        ref = np.empty_like(X)
        for i in range(4):
            for j in range(3):
                x = X[i, j]
                ref[i, j] = _brute_scalar(lambda s: g * abs(s) + 0.5 * (s - x) ** 2, x, abs(x) + 2 * g + 1)
        np.testing.assert_allclose(shrink(X, g), ref, atol=1e-7, rtol=0)


def test_shrink_special_values():
    # sgn(0) = 0; |x| == gamma gives exactly 0; odd symmetry.
    assert shrink(np.array([0.0]), 1.0)[0] == 0.0
    assert shrink(np.array([2.0, -2.0]), 2.0).tolist() == [0.0, 0.0]
    assert shrink(np.array([5.0, -5.0]), 2.0).tolist() == [3.0, -3.0]


# ------------------------------------------------------------ Eq. 4 (prox nuc)
@pytest.mark.parametrize("tau", [0.2, 0.9, 2.5])
def test_svt_kkt_certificate_4x3(tau):
    """A - D_tau(A) = tau (U_r V_r^T + W) with U_r^T W = 0, W V_r = 0, ||W||_2 <= 1:
    the optimality condition of min tau ||L||_* + 1/2 ||L - A||_F^2."""
    rng = np.random.default_rng(int(tau * 100))
    A = rng.standard_normal((4, 3)) * 2.0
    D = svt(A, tau)
    U, s, Vt = np.linalg.svd(D, full_matrices=False)
    r = int(np.sum(s > 1e-12 * max(1.0, s[0])))
    Ur, Vr = U[:, :r], Vt[:r].T
    W = (A - D) / tau - Ur @ Vr.T
    assert np.abs(Ur.T @ W).max() < 1e-12
    assert np.abs(W @ Vr).max() < 1e-12
    assert np.linalg.norm(W, 2) <= 1.0 + 1e-12


@pytest.mark.parametrize("tau", [0.3, 1.1])
def test_svt_matches_burer_monteiro_brute_force(tau):
    rng = np.random.default_rng(7 + int(10 * tau))
    A = rng.standard_normal((4, 3)) * 2.0
    Lbf = _bm_minimise(lambda L: 0.5 / tau * np.sum((L - A) ** 2), 4, 3, rng)
    # objective is ||L||_* + (1/(2 tau))||L - A||^2  (same minimiser as tau ||L||_* + ...)
    np.testing.assert_allclose(svt(A, tau), Lbf, atol=2e-6)


def test_svt_no_descent_direction():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 3)) * 3.0
    tau = 1.3
    D = svt(A, tau)

    def F(L):
        return tau * _nuclear(L) + 0.5 * np.sum((L - A) ** 2)

    f0 = F(D)
    for _ in range(200):
        E = rng.standard_normal((4, 3))
        for eps in (1e-2, 1e-4):
            assert F(D + eps * E) >= f0 - 1e-12


# --------------------------------------------- Eqs. 4 and 5 minimise Eq. 3
def _augmented_lagrangian(L, S, Y, X, lam, mu):
    """Eq. 3 written out term by term."""
    R = X - L - S
    return _nuclear(L) + lam * np.sum(np.abs(S)) + np.sum(Y * R) + 0.5 * mu * np.sum(R * R)


def test_L_step_minimises_augmented_lagrangian():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((4, 3)) * 2.0
    S = rng.standard_normal((4, 3)) * 0.5
    Y = rng.standard_normal((4, 3)) * 0.3
    lam, mu = 0.4, 0.8

    def g(L):  # Eq. 3 without the nuclear norm (the BM helper adds it)
        R = X - L - S
        return lam * np.sum(np.abs(S)) + np.sum(Y * R) + 0.5 * mu * np.sum(R * R)

    Lbf = _bm_minimise(g, 4, 3, rng)
    Lstep = svt(X - S + Y / mu, 1.0 / mu)   # Eq. 4
    np.testing.assert_allclose(Lstep, Lbf, atol=2e-6)
    assert _augmented_lagrangian(Lstep, S, Y, X, lam, mu) <= \
        _augmented_lagrangian(Lbf, S, Y, X, lam, mu) + 1e-9


def test_S_step_minimises_augmented_lagrangian():
    rng = np.random.default_rng(22)
    X = rng.standard_normal((4, 3)) * 2.0
    L = rng.standard_normal((4, 3))
    Y = rng.standard_normal((4, 3)) * 0.3
    lam, mu = 0.6, 1.7
    Sbf = np.empty_like(X)
    for i in range(4):
        for j in range(3):
            x, l, y = X[i, j], L[i, j], Y[i, j]
            # the S-dependent part of Eq. 3 for one entry
            fun = lambda s: lam * abs(s) - y * s + 0.5 * mu * (x - l - s) ** 2
            Sbf[i, j] = _brute_scalar(fun, x - l, abs(x - l) + 5)
    np.testing.assert_allclose(shrink(X - L + Y / mu, lam / mu), Sbf, atol=1e-7)


# ------------------------------------------------------ defaults and golden
def test_default_mu_and_lambda_formulas():
    g = _golden()["defaults"]
    X = np.array(g["X"])
    assert default_mu(X) == pytest.approx(g["mu"], rel=1e-15)
    assert default_lambda(*X.shape) == pytest.approx(g["lam"], rel=1e-15)
    # tall and wide shapes: 1/sqrt of the larger dimension
    assert default_lambda(16384, 20) == 1.0 / 128.0
    assert default_lambda(20, 16384) == 1.0 / 128.0


@pytest.mark.parametrize("name", ["diag_2x2", "diag_2x2_mu2", "rank1_3x2"])
def test_hand_worked_iterates(name):
    g = _golden()[name]
    X = np.array(g["X"])
    for it in g["iterates"]:
        seen = {}

        def cb(k, L, S, Y):
            seen[k] = (L.copy(), S.copy(), Y.copy())

        rpca(X, lam=g["lam"], mu=g["mu"], tol=0.0, maxit=it["k"], callback=cb)
        L, S, Y = seen[it["k"]]
        np.testing.assert_allclose(L, np.array(it["L"]), atol=1e-12)
        np.testing.assert_allclose(S, np.array(it["S"]), atol=1e-12)
        np.testing.assert_allclose(Y, np.array(it["Y"]), atol=1e-12)
        assert np.linalg.norm(X - L - S) == pytest.approx(it["residual_fro"], abs=1e-12)


def test_hand_worked_stopping_iteration():
    g = _golden()["diag_2x2"]
    r = rpca(np.array(g["X"]), lam=g["lam"], mu=g["mu"], tol=1e-9, maxit=50)
    assert r.status == oracle.OK
    assert r.iterations == g["stops_at_k_with_positive_tol"]


# --------------------------------------------------------------- invariants
def test_dual_bound_and_sign_invariant_every_iteration():
    """S-step optimality with the new S in Eq. 6: |Y| <= lam everywhere and
    Y = lam sgn(S) on supp S, after every iteration."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((60, 12)) + np.outer(rng.standard_normal(60), rng.standard_normal(12)) * 3
    worst = [0.0, 0.0]

    def cb(k, L, S, Y):
        lam = default_lambda(*X.shape)
        worst[0] = max(worst[0], float(np.abs(Y).max() / lam - 1.0))
        nz = S != 0
        if nz.any():
            worst[1] = max(worst[1], float(np.abs(Y[nz] - lam * np.sign(S[nz])).max() / lam))

    rpca(X, tol=0.0, maxit=40, callback=cb)
    assert worst[0] <= 1e-12
    assert worst[1] <= 1e-12


def test_stopping_rule_is_first_crossing():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((80, 10)) + 2.0
    tol = 1e-5
    r = rpca(X, tol=tol, maxit=5000)
    assert r.status == oracle.OK
    # returned iterate satisfies the test, the previous one did not
    assert np.linalg.norm(X - r.L - r.S) / np.linalg.norm(X) < tol
    assert r.history[-1] < tol
    if r.iterations > 1:
        assert r.history[-2] >= tol
    # not converged within the cap: exactly maxit iterations and status 1
    r2 = rpca(X, tol=tol, maxit=r.iterations - 1)
    assert r2.status == oracle.NOT_CONVERGED and r2.iterations == r.iterations - 1


def test_tol_nonpositive_runs_exactly_maxit():
    X = np.random.default_rng(8).standard_normal((30, 5))
    r = rpca(X, tol=0.0, maxit=17)
    assert r.iterations == 17 and r.status == oracle.NOT_CONVERGED


def test_zero_and_nonfinite_inputs():
    r = rpca(np.zeros((10, 4)), tol=1e-7, maxit=10)
    assert r.status == oracle.OK and r.iterations == 0
    assert not r.L.any() and not r.S.any()
    X = np.ones((10, 4))
    X[3, 2] = np.nan
    assert rpca(X).status == oracle.ERR_NONFINITE
    X[3, 2] = np.inf
    assert rpca(X).status == oracle.ERR_NONFINITE


# ------------------------------------------------------- whole-loop pins
@pytest.mark.parametrize("m,n,rank,rho,seed", [(2000, 40, 1, 0.05, 7), (300, 300, 10, 0.05, 8),
                                               (500, 500, 25, 0.05, 9)])
def test_planted_recovery(m, n, rank, rho, seed):
    """PCP recovers a planted low-rank + sparse pair (Eq. 2); the iteration must
    get there to the stopping accuracy."""
    L0, S0 = planted_low_rank_sparse(m, n, rank, rho, seed)
    r = rpca(L0 + S0, tol=1e-10, maxit=3000)
    assert r.status == oracle.OK
    assert rel_fro(r.L, L0) <= 1e-6
    assert rel_fro(r.S, S0) <= 1e-6
    assert np.linalg.norm(L0 + S0 - r.L - r.S) <= 1e-10 * np.linalg.norm(L0 + S0)


def test_small_lambda_gives_all_sparse():
    """lam < 1/sqrt(mn): lam ||L||_1 < ||L||_* for L != 0, so (0, X) is the
    unique PCP solution."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((24, 8)) + np.outer(rng.standard_normal(24), rng.standard_normal(8))
    lam = 0.9 / np.sqrt(X.size)
    r = rpca(X, lam=lam, tol=1e-12, maxit=20000)
    assert r.status == oracle.OK
    assert np.linalg.norm(r.L) <= 1e-9 * np.linalg.norm(X)
    assert rel_fro(r.S, X) <= 1e-9


def test_large_lambda_gives_all_low_rank():
    """lam > 1: ||S||_* <= ||S||_1 < lam ||S||_1 for S != 0, so (X, 0) is the
    unique PCP solution."""
    rng = np.random.default_rng(10)
    X = rng.standard_normal((24, 8))
    r = rpca(X, lam=1.1, tol=1e-12, maxit=20000)
    assert r.status == oracle.OK
    assert rel_fro(r.L, X) <= 1e-9
    assert np.linalg.norm(r.S) <= 1e-9 * np.linalg.norm(X)


def test_converged_point_satisfies_pcp_optimality():
    """At convergence Y certifies optimality of Eq. 2: Y in lam d||S||_1 (exact
    by construction) and Y in d||L||_*, i.e. Y = U_r V_r^T + W with W orthogonal
    to the range of L and ||W||_2 <= 1."""
    L0, S0 = planted_low_rank_sparse(200, 40, 2, 0.05, 12)
    X = L0 + S0
    r = rpca(X, tol=1e-11, maxit=5000)
    U, s, Vt = np.linalg.svd(r.L, full_matrices=False)
    k = int(np.sum(s > 1e-8 * s[0]))
    Ur, Vr = U[:, :k], Vt[:k].T
    assert np.abs(Ur.T @ r.Y @ Vr - np.eye(k)).max() < 1e-6
    W = r.Y - Ur @ Vr.T
    assert np.linalg.norm(W, 2) <= 1.0 + 1e-6


# ------------------------------------------------------------- symmetries
@pytest.fixture(scope="module")
def small_us():
    w = window_128x128x20()
    X = w.X()[::8].copy(order="F")     # 2048 x 20 subsample of the ultrasound window
    return X


def test_scale_equivariance_powers_of_two(small_us):
    X = small_us
    a = rpca(X, tol=1e-6, maxit=300)
    b = rpca(X * 4.0, tol=1e-6, maxit=300)
    assert a.iterations == b.iterations
    assert rel_fro(b.L, 4.0 * a.L) <= 1e-14
    assert rel_fro(b.S, 4.0 * a.S) <= 1e-14


def test_transpose_equivariance(small_us):
    X = small_us[:400]
    a = rpca(X, tol=1e-6, maxit=300)
    b = rpca(X.T, tol=1e-6, maxit=300)
    assert a.iterations == b.iterations
    assert rel_fro(b.L, a.L.T) <= 1e-11
    assert rel_fro(b.S, a.S.T) <= 1e-11


def test_permutation_equivariance(small_us):
    X = small_us
    rng = np.random.default_rng(4)
    pr = rng.permutation(X.shape[0])
    pc = rng.permutation(X.shape[1])
    a = rpca(X, tol=1e-6, maxit=300)
    b = rpca(X[pr][:, pc], tol=1e-6, maxit=300)
    assert a.iterations == b.iterations
    assert rel_fro(b.L, a.L[pr][:, pc]) <= 1e-11
    assert rel_fro(b.S, a.S[pr][:, pc]) <= 1e-11


# ------------------------------------------------ iteration from a given start
def test_explicit_zero_start_is_the_default():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((30, 6))
    a = rpca(X, tol=1e-8, maxit=200)
    b = rpca(X, tol=1e-8, maxit=200, S0=np.zeros_like(X), Y0=np.zeros_like(X))
    assert a.iterations == b.iterations
    assert np.array_equal(a.L, b.L) and np.array_equal(a.S, b.S) and np.array_equal(a.Y, b.Y)


def test_dual_bound_holds_after_one_step_from_any_start():
    """|Y_1| <= lam whatever S0, Y0 (Eq. 5 makes X - L + Y/mu - S_1 a clamp
    to [-lam/mu, lam/mu], and Eq. 6 scales it by mu)."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((25, 7))
    S0 = 5.0 * rng.standard_normal(X.shape)
    Y0 = 10.0 * rng.standard_normal(X.shape)
    r = rpca(X, tol=0.0, maxit=1, S0=S0, Y0=Y0)
    assert np.max(np.abs(r.Y)) <= r.lam * (1 + 1e-12)


def test_converged_point_is_a_fixed_point_of_the_iteration():
    """Started from its own converged (S, Y), a solve stops after one step
    with the same decomposition."""
    L0, S0_ = planted_low_rank_sparse(120, 30, 3, 0.05, 13)
    X = L0 + S0_
    ref = rpca(X, tol=1e-12, maxit=5000)
    assert ref.status == 0
    r = rpca(X, tol=1e-9, maxit=50, S0=ref.S, Y0=ref.Y)
    assert r.iterations == 1
    assert np.linalg.norm(r.L - ref.L) <= 1e-9 * np.linalg.norm(ref.L)
    assert np.linalg.norm(r.S - ref.S) <= 1e-9 * np.linalg.norm(ref.S)


def test_warm_start_from_shifted_window_needs_fewer_iterations():
    """Sliding windows (the real-time use of the method): starting a window
    from the previous window's S and Y, shifted by the step, is a valid start
    of the same iteration and reaches the same tolerance in fewer steps."""
    from synth import make_window
    w = make_window(32, 32, 25, 2, 4, 3, 20.0, 14)
    X = w.X()
    prev = rpca(X[:, :20], tol=1e-6, maxit=2000)
    cur_cold = rpca(X[:, 5:25], tol=1e-6, maxit=2000)
    S0 = np.zeros((X.shape[0], 20))
    Y0 = np.zeros((X.shape[0], 20))
    S0[:, :15] = prev.S[:, 5:]
    Y0[:, :15] = prev.Y[:, 5:]
    cur_warm = rpca(X[:, 5:25], tol=1e-6, maxit=2000, S0=S0, Y0=Y0)
    assert cur_warm.status == 0 and cur_cold.status == 0
    assert cur_warm.iterations < cur_cold.iterations
    # both are tol-accurate solutions of the same problem
    rel = np.linalg.norm(cur_warm.L - cur_cold.L) / np.linalg.norm(cur_cold.L)
    assert rel < 1e-3
