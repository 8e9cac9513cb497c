"""Pin of the oracle's adjoint gradient: central finite differences in FP64.

Loss L(beta) = sum_j w_j beta_j^2, beta = Phi(lambda, tau)^-1 b, so
g = dL/dbeta = 2 w beta.  Every perturbed loss is evaluated by a Cholesky
solve (not by CG), so the finite-difference quotient carries only the
h^2 truncation and eps/h rounding errors.
"""
import numpy as np

from oracle import ppcg_ref as R


_XTOX = {}


def _loss(X, omega, lam, tau, b, w):
    """L at (lambda, tau, b); X^T Omega X is formed once per design (only the
    prior term of Phi depends on lambda and tau)."""
    key = id(X)
    if key not in _XTOX:
        _XTOX[key] = R.phi_dense(X, omega, np.ones(X.shape[1]), 1.0) - np.eye(X.shape[1])
    Phi = _XTOX[key] + np.diag(R.prior_precision(lam, tau))
    beta = R.solve_chol(Phi, b)
    return float(np.sum(w * beta ** 2))


def test_adjoint_gradient_matches_central_differences(problem_cache):
    P = problem_cache("c4small")
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    rng = np.random.default_rng(44)
    w = rng.uniform(0.0, 1.0, P.p)
    b = R.rhs_b(X, P.omega, P.z, P.lam, P.tau, rng.standard_normal(P.n), rng.standard_normal(P.p))
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    beta = R.solve_chol(Phi, b)
    a, g_loglam, g_logtau = R.adjoint_gradient_dense(
        Phi, R.prior_precision(P.lam, P.tau), beta, 2.0 * w * beta)
    h = 1e-6
    loglam = np.log(P.lam)
    fd = np.empty(P.p)
    for j in range(P.p):
        lp = loglam.copy(); lp[j] += h
        lm = loglam.copy(); lm[j] -= h
        fd[j] = (_loss(X, P.omega, np.exp(lp), P.tau, b, w)
                 - _loss(X, P.omega, np.exp(lm), P.tau, b, w)) / (2 * h)
    scale = np.linalg.norm(fd)
    assert np.linalg.norm(fd - g_loglam) <= 1e-6 * scale
    fdt = (_loss(X, P.omega, P.lam, P.tau * np.exp(h), b, w)
           - _loss(X, P.omega, P.lam, P.tau * np.exp(-h), b, w)) / (2 * h)
    assert abs(fdt - g_logtau) <= 1e-6 * max(abs(fdt), 1e-12) + 1e-9 * scale
    for j in rng.choice(P.p, 20, replace=False):
        bp = b.copy(); bp[j] += h
        bm = b.copy(); bm[j] -= h
        fdb = (_loss(X, P.omega, P.lam, P.tau, bp, w) - _loss(X, P.omega, P.lam, P.tau, bm, w)) / (2 * h)
        assert abs(fdb - a[j]) <= 1e-6 * np.linalg.norm(a) + 1e-6 * abs(a[j])


def test_adjoint_planted_sign_error_is_caught(problem_cache):
    """A sign slip in the lambda gradient (a plausible mistake) fails the FD check."""
    P = problem_cache("c4small")
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    rng = np.random.default_rng(45)
    w = rng.uniform(0.0, 1.0, P.p)
    b = rng.standard_normal(P.p) * 50
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    beta = R.solve_chol(Phi, b)
    _, g_loglam, _ = R.adjoint_gradient_dense(Phi, R.prior_precision(P.lam, P.tau), beta, 2 * w * beta)
    h = 1e-6
    j = int(np.argmax(np.abs(g_loglam)))
    lp = np.log(P.lam); lp[j] += h
    lm = np.log(P.lam); lm[j] -= h
    fd = (_loss(X, P.omega, np.exp(lp), P.tau, b, w) - _loss(X, P.omega, np.exp(lm), P.tau, b, w)) / (2 * h)
    assert abs(fd - g_loglam[j]) <= 1e-6 * abs(fd)
    assert abs(fd - (-g_loglam[j])) > 0.5 * abs(fd)
