"""Pins of the oracle's Phi, Cholesky and preconditioned-CG functions.

Each test checks the oracle against something other than itself: brute-force
loops, a special case with a closed form, or a theorem of Section 2.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ppcg_ref as R
from oracle import theory_ref as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(n=60, p=25, rho=0.2, tau=0.5, seed=3):
    P = synth.tiny_problem(p, n=n, rho=rho, tau=tau, seed=seed)
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    return P, X


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_phi_three_ways_agree(seed):
    """Dense Phi @ v == matrix-free X^T(omega*(X v)) + d*v == explicit loops."""
    P, X = _small(seed=seed)
    v = np.random.default_rng(seed).standard_normal(P.p)
    dense = R.phi_dense(X, P.omega, P.lam, P.tau) @ v
    free = R.phi_matvec(X, P.omega, P.lam, P.tau, v)
    loops = R.phi_matvec_loops(P.n, P.p, P.row_ptr, P.col_idx, P.omega, P.lam, P.tau, v)
    # Independent dense construction from the 0/1 matrix.
    Xd = P.dense_x()
    by_hand = Xd.T @ np.diag(P.omega) @ Xd @ v + v / (P.tau * P.lam) ** 2
    for other in (free, loops, by_hand):
        assert np.linalg.norm(dense - other) <= 1e-13 * np.linalg.norm(dense)


def test_phi_zero_design_is_prior_precision():
    """X = 0  =>  Phi = tau^-2 Lambda^-2."""
    n, p = 10, 7
    rp = np.zeros(n + 1, dtype=np.int64)
    ci = np.zeros(0, dtype=np.int32)
    X = R.csr_matrix(n, p, rp, ci)
    lam = np.linspace(0.5, 3.0, p)
    Phi = R.phi_dense(X, np.ones(n), lam, 0.3)
    assert np.allclose(Phi, np.diag(1.0 / (0.3 * lam) ** 2), rtol=1e-15, atol=0)


def test_rhs_b_entries_by_hand():
    """b_j = sum_i x_ij omega_i z_i + sum_i x_ij sqrt(omega_i) eta_i + delta_j/(tau lambda_j)."""
    P, X = _small(n=12, p=5)
    rng = np.random.default_rng(4)
    eta, delta = rng.standard_normal(P.n), rng.standard_normal(P.p)
    b = R.rhs_b(X, P.omega, P.z, P.lam, P.tau, eta, delta)
    Xd = P.dense_x()
    for j in range(P.p):
        want = sum(Xd[i, j] * (P.omega[i] * P.z[i] + np.sqrt(P.omega[i]) * eta[i])
                   for i in range(P.n)) + delta[j] / (P.tau * P.lam[j])
        assert abs(b[j] - want) <= 1e-13 * (1 + abs(want))


def test_cholesky_solve_residual(problem_cache):
    P = problem_cache("c0")
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    b = np.random.default_rng(0).standard_normal(P.p)
    beta = R.solve_chol(Phi, b)
    assert np.linalg.norm(Phi @ beta - b) <= 1e-13 * np.linalg.norm(b) * np.linalg.cond(Phi) ** 0.0 + 1e-9 * np.linalg.norm(b)
    # Explicit inverse check on a well conditioned copy: Phi^-1 Phi = I.
    L = R.cholesky(Phi)
    assert np.allclose(L @ L.T, Phi, rtol=1e-12, atol=1e-12 * np.abs(Phi).max())


def test_pcg_equals_cholesky_at_tight_tol(problem_cache):
    """PCG run to 1e-14 agrees with the direct solve (CG is exact in <= p steps)."""
    P = problem_cache("c0")
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    b = R.rhs_b(X, P.omega, P.z, P.lam, P.tau,
                np.random.default_rng(1).standard_normal(P.n),
                np.random.default_rng(2).standard_normal(P.p))
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-14)
    assert res.status == R.STATUS_OK
    exact = R.solve_chol(Phi, b)
    assert np.linalg.norm(res.beta - exact) <= 1e-12 * np.linalg.norm(exact)


def test_pcg_zero_design_one_iteration():
    """X = 0: Phi~ = I so PCG converges in one step to beta = c * delta for
    b = delta / c (c = tau lambda)."""
    n, p = 10, 9
    X = R.csr_matrix(n, p, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32))
    lam = np.exp(np.random.default_rng(0).standard_normal(p))
    tau = 0.2
    delta = np.random.default_rng(1).standard_normal(p)
    b = R.rhs_b(X, np.ones(n), np.zeros(n), lam, tau, np.zeros(n), delta)
    res = R.pcg_solve(X, np.ones(n), lam, tau, b, tol=1e-14)
    assert res.iters == 1
    assert np.allclose(res.beta, tau * lam * delta, rtol=1e-14, atol=0)


def test_thm22_rank_k_terminates_in_k_plus_1():
    """n = k < p: X^T Omega X has rank <= k, Phi~ = I + rank k, so PCG is exact
    within k + 1 iterations (Theorem 2.2)."""
    k, p = 3, 200
    rng = np.random.default_rng(5)
    rp, ci = synth.bernoulli_design(k, p, 0.3, rng)
    X = R.csr_matrix(k, p, rp, ci)
    om = rng.gamma(1.0, 0.25, size=k) + 0.01
    # Moderate scales keep the rounding floor low; the theorem is exact only
    # in exact arithmetic.
    lam = np.exp(0.5 * rng.standard_normal(p))
    tau = 0.5
    b = rng.standard_normal(p)
    res = R.pcg_solve(X, om, lam, tau, b, tol=1e-11)
    assert res.status == R.STATUS_OK
    assert res.iters <= k + 1
    # ... and not trivially: after k iterations the residual is still large.
    assert res.resid_norms[k - 1] > 1e-6 * res.resid_norms[0]
    exact = R.solve_chol(R.phi_dense(X, om, lam, tau), b)
    assert np.linalg.norm(res.beta - exact) <= 1e-9 * np.linalg.norm(exact)


def test_exact_within_p_iterations():
    """CG yields the exact solution after p iterations (Section 2.2)."""
    P, X = _small(n=40, p=6, rho=0.3, tau=1.0)
    # Exactness after p steps holds in exact arithmetic; a small p and moderate
    # local scales keep the loss of orthogonality at the rounding level.
    lam = np.exp(0.3 * np.random.default_rng(10).standard_normal(P.p))
    b = np.random.default_rng(9).standard_normal(P.p)
    res = R.pcg_solve(X, P.omega, lam, P.tau, b, tol=0.0, max_iter=P.p,
                      keep_iterates=True)
    exact = R.solve_chol(R.phi_dense(X, P.omega, lam, P.tau), b)
    # The last iterate (<= p steps; it may stop early on an exact zero) matches.
    assert np.linalg.norm(res.iterates[-1] - exact) <= 1e-8 * np.linalg.norm(exact)


def test_phi_norm_error_monotone_and_theorem_bounds():
    """Optimality (eq. cg_optimality_property) => ||beta_k - beta||_Phi is
    non-increasing; Theorems 2.1 and 2.5 bound it at every k.  In the
    preconditioned variable the relevant norm is the Phi-norm of the error in
    beta, since ||e~||_Phi~ = ||M^1/2 e||_{M^-1/2 Phi M^-1/2} = ||e||_Phi."""
    P, X = _small(n=150, p=30, rho=0.25, tau=1.0, seed=11)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    b = np.random.default_rng(12).standard_normal(P.p)
    exact = R.solve_chol(Phi, b)
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-13, keep_iterates=True)
    errs = [T.phi_norm(it - exact, Phi) for it in res.iterates]
    e0 = errs[0]
    XtOX = Phi - np.diag(R.prior_precision(P.lam, P.tau))
    Phit = T.precond_matrix(XtOX, P.lam, P.tau)
    ev = np.linalg.eigvalsh(Phit)
    kappa = ev[-1] / ev[0]
    for k in range(1, len(errs)):
        assert errs[k] <= errs[k - 1] * (1 + 1e-9) + 1e-12 * e0
        assert errs[k] <= T.thm21_bound(kappa, k) * e0 * (1 + 1e-9) + 1e-12 * e0
    for m in range(0, 6):
        km = T.thm25_kappa(XtOX, P.lam, P.tau, m)
        for mp in range(0, len(errs) - m):
            assert errs[m + mp] <= T.thm25_bound(km, mp) * e0 * (1 + 1e-9) + 1e-12 * e0


def test_thm24_eigenvalue_clustering():
    """1 <= nu_k(Phi~) <= 1 + tau^2 lambda_(k)^2 nu_1(X^T Omega X) (Theorem 2.4)."""
    P, X = _small(n=100, p=40, rho=0.2, tau=0.7, seed=21)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    XtOX = Phi - np.diag(R.prior_precision(P.lam, P.tau))
    ev = np.sort(np.linalg.eigvalsh(T.precond_matrix(XtOX, P.lam, P.tau)))[::-1]
    up = T.thm24_upper(XtOX, P.lam, P.tau)
    assert np.all(ev >= 1 - 1e-10)
    assert np.all(ev <= up * (1 + 1e-10))


def test_termination_identity_and_posterior_bound(problem_cache):
    """||r~_k||^2 = <r_k, m r_k> with r~ = tau lambda r (Supplement S4.2), and
    ||(beta_k - beta)/c|| <= ||c (b - Phi beta_k)|| at every k."""
    P = problem_cache("c0")
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    b = np.random.default_rng(3).standard_normal(P.p)
    exact = R.solve_chol(Phi, b)
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-10, keep_iterates=True)
    c = P.tau * P.lam
    for k in range(0, len(res.iterates), 7):
        rt = R.true_residual(X, P.omega, P.lam, P.tau, b, res.iterates[k])
        assert abs(np.linalg.norm(c * rt) - res.resid_norms[k]) <= 1e-7 * res.resid_norms[0]
        bound = R.posterior_error_bound(X, P.omega, P.lam, P.tau, b, res.iterates[k])
        assert np.linalg.norm((res.iterates[k] - exact) / c) <= bound * (1 + 1e-9) + 1e-14


def test_criteria_thresholds():
    b = np.array([3.0, 4.0])
    m = np.array([4.0, 1.0])
    assert R.stop_threshold(R.REL_PRECOND, 0.1, b, m, 2) == pytest.approx(0.1 * np.sqrt(36 + 16))
    assert R.stop_threshold(R.RMS_PRECOND_ABS, 1e-6, b, m, 2) == pytest.approx(1e-6 * np.sqrt(2))
    assert R.stop_threshold(R.REL_PLAIN, 0.5, b, m, 2) == pytest.approx(2.5)


def test_criterion_value_by_hand():
    """r = (1, 0), b = (0, 4), m = (4, 1):
    REL_PRECOND  sqrt(<r, m r>) / sqrt(<b, m b>) = 2 / 4 = 1/2;
    RMS_PRECOND_ABS  sqrt(<r, m r> / p) = sqrt(4 / 2) = sqrt 2;
    REL_PLAIN  ||r|| / ||b|| = 1/4.
    (A dropped square root gives 1/4, 2 and 1/16; m in the plain rule 1/2.)
    The value is sign-invariant and 1 exactly at the threshold."""
    r, b, m = np.array([1.0, 0.0]), np.array([0.0, 4.0]), np.array([4.0, 1.0])
    assert R.criterion_value(R.REL_PRECOND, r, b, m) == pytest.approx(0.5, rel=1e-15)
    assert R.criterion_value(R.RMS_PRECOND_ABS, r, b, m) == pytest.approx(np.sqrt(2.0), rel=1e-15)
    assert R.criterion_value(R.REL_PLAIN, r, b, m) == pytest.approx(0.25, rel=1e-15)
    for crit in (R.REL_PRECOND, R.RMS_PRECOND_ABS, R.REL_PLAIN):
        assert R.criterion_value(crit, -r, b, m) == R.criterion_value(crit, r, b, m)
    # at the threshold: value == tol  <=>  measure == stop_threshold
    for crit, meas in ((R.REL_PRECOND, 2.0), (R.RMS_PRECOND_ABS, 2.0), (R.REL_PLAIN, 1.0)):
        tol = R.criterion_value(crit, r, b, m)
        assert R.stop_threshold(crit, tol, b, m, 2) == pytest.approx(meas, rel=1e-15)


def test_criterion_value_matches_pcg_history():
    """On a small problem, the value of each rule on the true residual
    b - Phi beta_k of PCG's iterates equals what PCG records for the
    recursive residual (||c r_k|| and ||r_k||, scaled as the rule scales
    them) to rounding, at every k."""
    P, X = _small(n=120, p=30, rho=0.2, tau=0.8, seed=13)
    # moderate local scales keep the gap between the recursive and the true
    # residual (rounding, growing with ||Phi||) far below the values compared
    lam = np.exp(0.4 * np.random.default_rng(18).standard_normal(P.p))
    b = np.random.default_rng(14).standard_normal(P.p)
    res = R.pcg_solve(X, P.omega, lam, P.tau, b, tol=1e-9, keep_iterates=True)
    m = R.precond_inverse(lam, P.tau)
    n0, q0 = res.resid_norms[0], res.plain_norms[0]
    assert res.status == R.STATUS_OK and res.iters > 5
    for k in range(len(res.iterates)):
        rt = R.true_residual(X, P.omega, lam, P.tau, b, res.iterates[k])
        assert R.criterion_value(R.REL_PRECOND, rt, b, m) == pytest.approx(
            res.resid_norms[k] / n0, rel=1e-6, abs=1e-12)
        assert R.criterion_value(R.RMS_PRECOND_ABS, rt, b, m) == pytest.approx(
            res.resid_norms[k] / np.sqrt(P.p), rel=1e-6, abs=1e-12 * n0)
        assert R.criterion_value(R.REL_PLAIN, rt, b, m) == pytest.approx(
            res.plain_norms[k] / q0, rel=1e-6, abs=1e-12)
    # at the stop, the value of the configured rule is at most tol
    rt = R.true_residual(X, P.omega, lam, P.tau, b, res.beta)
    assert R.criterion_value(R.REL_PRECOND, rt, b, m) <= 1e-9 * (1 + 1e-3)


def test_error_metrics_by_hand():
    """Phi = [[4, 2], [2, 3]], mean_rhs = (2, 1): mu = (1/2, 0) and
    diag(Phi^-1) = (3/8, 1/2), so xi^2 = mu^2 + diag(Phi^-1) = (5/8, 1/2).
    For beta - beta_ref = (0.1, -0.2) with beta_ref = (0.5, 0.25), scale
    (0.5, 4): rel_l2 = sqrt(0.05) / sqrt(0.3125), scaled_max = max(0.2,
    0.05), coord_rel = (0.2 + 0.8) / 2 and secmom_rms = sqrt((0.01 / 0.625
    + 0.04 / 0.5) / 2)."""
    Phi = np.array([[4.0, 2.0], [2.0, 3.0]])
    ref = np.array([0.5, 0.25])
    e = R.error_metrics(ref + np.array([0.1, -0.2]), ref, np.array([0.5, 4.0]), Phi,
                        np.array([2.0, 1.0]))
    assert e["rel_l2"] == pytest.approx(np.sqrt(0.05 / 0.3125), rel=1e-14)
    assert e["scaled_max"] == pytest.approx(0.2, rel=1e-14)
    assert e["coord_rel"] == pytest.approx(0.5, rel=1e-14)
    assert e["secmom_rms"] == pytest.approx(np.sqrt((0.01 / 0.625 + 0.04 / 0.5) / 2), rel=1e-14)
    # zero reference coefficients are left out of the coordinate-wise mean
    e = R.error_metrics(np.array([0.1, 1.1]), np.array([0.0, 1.0]), np.ones(2))
    assert e["coord_rel"] == pytest.approx(0.1, rel=1e-14) and "secmom_rms" not in e


def test_secmom_error_under_the_residual_bound():
    """Supplement S4.2, eq. normalized_error_relation_to_precond_resid:
    ||xi^-1 (beta_k - beta)|| <= max_j(xi_j^-1 tau lambda_j) ||Phi~^-1 r~_k||
    <= max_j(xi_j^-1 tau lambda_j) ||r~_k|| at every iterate (the smallest
    eigenvalue of Phi~ is at least one, Theorem 2.4)."""
    P, X = _small(n=150, p=25, rho=0.25, tau=0.5, seed=15)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    mean_b = R.rhs_mean(X, P.omega, P.z)
    b = R.rhs_b(X, P.omega, P.z, P.lam, P.tau, np.random.default_rng(16).standard_normal(P.n),
                np.random.default_rng(17).standard_normal(P.p))
    exact = R.solve_chol(Phi, b)
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-12, keep_iterates=True)
    c = P.tau * P.lam
    mu = R.solve_chol(Phi, mean_b)
    xi = np.sqrt(mu * mu + np.diag(np.linalg.inv(Phi)))
    factor = np.max(c / xi)
    for k in range(len(res.iterates)):
        e = R.error_metrics(res.iterates[k], exact, c, Phi, mean_b)
        rt = R.true_residual(X, P.omega, P.lam, P.tau, b, res.iterates[k])
        norm = e["secmom_rms"] * np.sqrt(P.p)
        assert norm <= factor * np.linalg.norm(c * rt) * (1 + 1e-9) + 1e-13
        # and the prior-scaled error sits under the a-posteriori bound
        assert e["scaled_max"] <= np.linalg.norm(c * rt) * (1 + 1e-9) + 1e-13


def test_paper_rms_rule_stops_where_stated():
    """With the paper's rule p^-1/2 ||r~_k|| <= 1e-6 the oracle stops at the
    first k where the recorded preconditioned residual crosses the threshold."""
    P, X = _small(n=200, p=60, rho=0.1, tau=0.3, seed=8)
    b = np.random.default_rng(1).standard_normal(P.p) * 10
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-6,
                      criterion=R.RMS_PRECOND_ABS)
    h = np.array(res.resid_norms) / np.sqrt(P.p)
    assert h[-1] <= 1e-6 and np.all(h[:-1] > 1e-6)


def test_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "thm25_worked_example.json")))
    rate = np.log10(T.sqrt_kappa_rate(g["kappa"]))
    assert rate <= g["log10_rate_at_most"]
    assert rate == pytest.approx(-0.0867, abs=5e-4)
    assert g["mprime"] * g["log10_rate_at_most"] == pytest.approx(g["log10_factor_after_mprime"])
    assert np.log10(2.0) + g["log10_factor_after_mprime"] == pytest.approx(
        g["log10_factor_with_leading_2"], abs=0.05)
    assert np.log10(T.thm25_bound(g["kappa"], g["mprime"])) <= g["log10_factor_with_leading_2"] + 0.05


def test_notconv_and_breakdown_status():
    P, X = _small(n=100, p=40, tau=5.0)
    b = np.random.default_rng(2).standard_normal(P.p)
    res = R.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=1e-14, max_iter=1)
    assert res.status == R.STATUS_NOTCONV and res.iters == 1
    # An indefinite operator breaks down: <s, A s> <= 0.
    res = R.pcg(lambda v: -v, np.ones(4), np.ones(4), tol=1e-12)
    assert res.status == R.STATUS_BREAKDOWN
