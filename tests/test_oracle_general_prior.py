"""Pins of the oracle's general diagonal prior and preconditioner (Supplement
S4.3: coefficients without shrinkage get N(0, sigma_j^2) priors, flat when
sigma_j is infinite, and preconditioner scales gamma_j of the caller's
choice).  Checked against closed forms, the Cholesky solution, the
eigenvalue bounds the supplement relies on, and the law of Prop 2.1."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import philox_ref as H
from oracle import ppcg_ref as R
from oracle import stats_ref as S

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _mixed(n=60, p=12, seed=3, q=1):
    """Intercept (flat prior), q more unshrunk coefficients (sigma = 2), the
    rest shrunk (tau lambda); gamma of the unshrunk ones from the marginal
    posterior scale estimate the supplement suggests (c = 2)."""
    rng = np.random.default_rng(seed)
    dense = (rng.random((n, p)) < 0.3).astype(np.float64)
    dense[:, 0] = 1.0
    X = sp.csr_matrix(dense)
    omega = rng.gamma(1.0, 0.25, n) + 0.01
    z = rng.standard_normal(n)
    lam = np.abs(np.tan(np.pi * rng.random(p) / 2)) + 0.05
    tau = 0.3
    d = 1.0 / (tau * lam) ** 2
    d[0] = 0.0
    d[1:q + 1] = 1.0 / 4.0
    Phi = R.phi_dense_general(X, omega, d)
    psi = np.sqrt(np.diag(np.linalg.inv(Phi)))  # posterior scales
    m = (tau * lam) ** 2
    m[:q + 1] = (2.0 * psi[:q + 1]) ** 2
    return X, omega, z, d, m, Phi


def test_intercept_only_flat_prior_closed_form():
    """X = a column of ones, flat prior: Phi = sum(omega), b = sum(omega z) +
    sum(sqrt(omega) eta); one CG step gives b / sum(omega) whatever the
    preconditioner scale."""
    rng = np.random.default_rng(7)
    n = 50
    X = sp.csr_matrix(np.ones((n, 1)))
    omega = rng.gamma(1.0, 0.25, n) + 0.01
    z, eta = rng.standard_normal(n), rng.standard_normal(n)
    d = np.zeros(1)
    b = R.rhs_b_general(X, omega, z, d, eta, rng.standard_normal(1))
    assert abs(b[0] - (np.sum(omega * z) + np.sum(np.sqrt(omega) * eta))) <= 1e-13 * abs(b[0])
    for gamma2 in (1e-3, 2.5, 1e4):
        res = R.pcg_solve_general(X, omega, d, np.array([gamma2]), b, tol=1e-14)
        assert res.iters == 1
        assert abs(res.beta[0] - b[0] / np.sum(omega)) <= 1e-14 * abs(res.beta[0])


def test_phi_diag_is_the_dense_diagonal():
    X, omega, z, d, m, Phi = _mixed()
    assert np.allclose(R.phi_diag(X, omega, d), np.diag(Phi), rtol=1e-14, atol=0)


def test_general_matvec_is_the_dense_product():
    X, omega, z, d, m, Phi = _mixed()
    v = np.random.default_rng(1).standard_normal(Phi.shape[0])
    assert np.allclose(R.phi_matvec_general(X, omega, d, v), Phi @ v, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("q", [1, 3])
def test_general_pcg_matches_cholesky(q):
    X, omega, z, d, m, Phi = _mixed(q=q)
    b = np.random.default_rng(q).standard_normal(Phi.shape[0])
    res = R.pcg_solve_general(X, omega, d, m, b, tol=1e-14, max_iter=10 * Phi.shape[0])
    exact = R.solve_chol(Phi, b)
    assert res.status == R.STATUS_OK
    assert np.linalg.norm(res.beta - exact) <= 1e-11 * np.linalg.norm(exact)


def test_jacobi_preconditioner_solves_too():
    """The Jacobi preconditioner M = diag(Phi) (the paper's comparison) on the
    same system: same solution."""
    X, omega, z, d, m, Phi = _mixed()
    b = np.random.default_rng(9).standard_normal(Phi.shape[0])
    res = R.pcg_solve_general(X, omega, d, 1.0 / R.phi_diag(X, omega, d), b, tol=1e-14,
                              max_iter=10 * Phi.shape[0])
    exact = R.solve_chol(Phi, b)
    assert np.linalg.norm(res.beta - exact) <= 1e-11 * np.linalg.norm(exact)


@pytest.mark.parametrize("q", [1, 3])
def test_modified_preconditioner_eigenvalues(q):
    """Phi~ = M^-1/2 Phi M^-1/2 with M = diag(gamma^-2, tau^-2 lambda^-2): the
    block of the shrunk coefficients has every eigenvalue >= 1 (Theorem 2.4),
    and the eigenvalues of Phi~ interlace those of that block (the Poincare
    separation theorem the supplement invokes), so at most q + 1 of them fall
    below its smallest."""
    X, omega, z, d, m, Phi = _mixed(q=q)
    sq = np.sqrt(m)
    Pt = sq[:, None] * Phi * sq[None, :]
    mu = np.linalg.eigvalsh(Pt)
    nu = np.linalg.eigvalsh(Pt[q + 1:, q + 1:])
    assert nu[0] >= 1.0 - 1e-10
    k = q + 1
    for i in range(nu.size):
        assert mu[i] <= nu[i] + 1e-9 * nu[-1]
        assert nu[i] <= mu[i + k] + 1e-9 * nu[-1]
    assert np.sum(mu < nu[0] - 1e-9 * nu[-1]) <= k


def test_general_b_law():
    """Prop 2.1 with a flat-prior intercept: b ~ N(X^T Omega z, Phi), from the
    counter-based normals (fixed seeds)."""
    X, omega, z, d, m, Phi = _mixed(n=40, p=6, seed=11)
    L = R.cholesky(Phi)
    N = 20_000
    draws = np.arange(N)
    eta = H.normals_many(77, H.STREAM_ETA, 0, draws, X.shape[0])
    delta = H.normals_many(77, H.STREAM_DELTA, 0, draws, X.shape[1])
    omega_ = np.asarray(omega)
    y = omega_ * z + np.sqrt(omega_) * eta
    bs = (X.T @ y.T).T + np.sqrt(d) * delta
    b0 = R.rhs_b_general(X, omega, z, d, eta[5], delta[5])
    assert np.allclose(b0, bs[5], rtol=1e-14, atol=1e-14)
    mean_b = X.T @ (omega_ * z)
    assert S.passes(S.gaussian_tests(S.whiten_b(bs, mean_b, L)))


def test_warm_start_estimator_recovers_the_mean():
    """With draws from a fixed conditional, the rescaled running mean is the
    sample mean of the draws, so beta0 -> the conditional mean mu, the target
    Supplement S4.1 sets for the start: its squared Phi-norm distance to mu has
    expectation p / N against p for the last draw, and CG from it converges."""
    X, omega, z, d, m, Phi = _mixed(q=0)
    p = Phi.shape[0]
    rng = np.random.default_rng(21)
    lam = np.sqrt(1.0 / np.where(d > 0, d, 1.0))  # tau = 1 scales (d = lambda^-2 here)
    tau = 1.0
    L = R.cholesky(Phi)
    mean_b = X.T @ (omega * z)
    mu = R.solve_chol(Phi, mean_b)
    acc = np.zeros(p)
    N = 400
    draws = mu + np.linalg.solve(L.T, rng.standard_normal((p, N))).T
    for k in range(N):
        acc = R.warm_start_accumulate(acc, draws[k], lam, tau)
    beta0 = R.warm_start_vector(acc, N, lam, tau)
    assert np.allclose(beta0, draws.mean(axis=0), rtol=1e-12, atol=1e-14)
    b = R.rhs_b_general(X, omega, z, d, rng.standard_normal(X.shape[0]), rng.standard_normal(p))
    cold = R.pcg_solve_general(X, omega, d, m, b, tol=1e-8)
    warm = R.pcg_solve_general(X, omega, d, m, b, beta0=beta0, tol=1e-8)
    exact = R.solve_chol(Phi, b)
    assert np.linalg.norm(warm.beta - exact) <= 1e-6 * np.linalg.norm(exact)
    assert np.linalg.norm(cold.beta - exact) <= 1e-6 * np.linalg.norm(exact)
    err = lambda v: float((v - mu) @ Phi @ (v - mu))  # noqa: E731
    assert err(beta0) < 0.05 * err(draws[-1])


def test_unshrunk_scales_by_hand_and_by_law():
    """Supplement S4.3's gamma_j = c eta_hat_j: by hand on two draws (sample
    variances 2 and 8 with divisor N - 1), and from many draws of a known
    Gaussian the estimate approaches its variances; the shrunk block keeps
    tau^-2 lambda^-2 and (tau lambda)^2."""
    lam = np.array([7.0, 7.0, 0.5, 2.0])
    tau = 0.1
    d, m = R.unshrunk_prior_precond([0.0, 1.0 / 9.0], [[1.0, 10.0], [3.0, 14.0]], 2.0, lam, tau)
    assert np.array_equal(d, [0.0, 1.0 / 9.0, 1.0 / (0.1 * 0.5) ** 2, 1.0 / (0.1 * 2.0) ** 2])
    assert np.allclose(m, [4.0 * 2.0, 4.0 * 8.0, (0.1 * 0.5) ** 2, (0.1 * 2.0) ** 2], rtol=1e-15)
    d0, m0 = R.unshrunk_prior_precond([], np.zeros((3, 0)), 2.0, lam, tau)
    assert np.allclose(d0 * m0, 1.0, rtol=1e-15)
    rng = np.random.default_rng(8)
    sd = np.array([0.3, 2.0, 11.0])
    draws = np.array([-3.0, 0.0, 40.0]) + sd * rng.standard_normal((20_000, 3))
    _, m = R.unshrunk_prior_precond(np.zeros(3), draws, 1.0, np.ones(5), 1.0)
    assert np.allclose(np.sqrt(m[:3]), sd, rtol=0.02)


def test_jacobi_preconditioned_phi_has_unit_diagonal():
    """M = diag(Phi): M^-1/2 Phi M^-1/2 has ones on its diagonal, with the
    diagonal taken from the dense Phi."""
    X, omega, z, d, m, Phi = _mixed(q=2)
    mj = R.jacobi_precond_inverse(X, omega, d)
    assert np.allclose(mj, 1.0 / np.diag(Phi), rtol=1e-14)
    S_ = np.sqrt(mj)[:, None] * Phi * np.sqrt(mj)[None, :]
    assert np.allclose(np.diag(S_), 1.0, rtol=1e-14)


def test_preconditioner_choice_on_diagonal_systems():
    """A design with one non-zero per row makes X^T Omega X diagonal: the
    Jacobi preconditioner then makes Phi the identity, CG stops after one
    iteration and the choice is Jacobi, while the prior preconditioner needs
    as many iterations as Phi~ has distinct eigenvalues.  With X = 0 both
    preconditioners equal Phi and tie, and a tie keeps the prior one."""
    rng = np.random.default_rng(12)
    n, p = 40, 8
    cols = rng.integers(0, p, n)
    X = sp.csr_matrix((np.ones(n), cols, np.arange(n + 1)), shape=(n, p))
    omega = rng.gamma(1.0, 0.25, n) + 0.01
    lam = np.exp(rng.standard_normal(p))
    d = R.prior_precision(lam, 0.5)
    b = rng.standard_normal(p)
    jac = R.pcg_solve_general(X, omega, d, R.jacobi_precond_inverse(X, omega, d), b, tol=1e-12)
    pri = R.pcg_solve_general(X, omega, d, 1.0 / d, b, tol=1e-12)
    assert jac.iters == 1
    assert pri.iters == np.unique(np.round(1.0 + np.bincount(cols, omega, p) / d, 12)).size
    assert R.choose_preconditioner(pri.iters, jac.iters) == "jacobi"
    Z = sp.csr_matrix((n, p))
    jz = R.pcg_solve_general(Z, omega, d, R.jacobi_precond_inverse(Z, omega, d), b, tol=1e-12)
    pz = R.pcg_solve_general(Z, omega, d, 1.0 / d, b, tol=1e-12)
    assert jz.iters == pz.iters == 1
    assert R.choose_preconditioner(pz.iters, jz.iters) == "prior"
