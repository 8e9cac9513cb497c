"""Pins of the oracle's counter-based normals and of its distribution tests.

* Philox4x64-10 raw words are checked against numpy.random.Philox, an
  independent library implementation of the same published generator.
* The normals are checked by moments and a Kolmogorov-Smirnov test.
* The chi-square harness is checked on exact Cholesky draws (must pass) and
  on a planted mistake (the Omega^1/2 eta term of Prop 2.1 dropped: must
  fail), and the oracle's CG-sampler draws (Prop 2.1 + PCG) must pass.
"""
import numpy as np
import pytest
import scipy.stats as st

import synth
from oracle import philox_ref as H
from oracle import ppcg_ref as R
from oracle import stats_ref as S


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (1, 0, 0, 0)),
    ((12437, 0), (5, 1, 3, 7)),
    ((2**64 - 1, 2**64 - 1), (2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344), (0xA4093822299F31D0, 0x082EFA98EC4E6C89,
                                               0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(key, ctr):
    """numpy's Philox increments its counter (with carry) and then applies
    Philox4x64-10; so its first block for counter c is Philox(c + 1)."""
    c = list(ctr)
    prev = [(c[0] - 1) & H.MASK64] + c[1:]
    if c[0] == 0:  # borrow into word 1 (not used by these cases)
        pytest.skip("borrow case")
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(prev, dtype=np.uint64))
    want = [int(x) for x in bg.random_raw(4)]
    assert list(H.philox4x64_scalar(ctr, key)) == want
    got = H.philox4x64(np.array([ctr], dtype=np.uint64), key)[0]
    assert [int(x) for x in got] == want


def test_philox_vector_equals_scalar():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(64, 4), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    for key in [(1, 2), (2**63 + 5, 17)]:
        v = H.philox4x64(ctr, key)
        for i in range(0, 64, 9):
            assert tuple(int(x) for x in v[i]) == H.philox4x64_scalar(tuple(int(x) for x in ctr[i]), key)


def test_uniform_ranges_exact():
    w = np.array([[0, 0, 2**64 - 1, 2**64 - 1]], dtype=np.uint64)
    ua, ub = H.uniforms_from_words(w)
    assert ua[0, 0] == 0.5 * 2.0 ** -52 and ub[0, 0] == 0.0
    assert ua[0, 1] == (2.0 ** 52 - 0.5) * 2.0 ** -52 and ua[0, 1] < 1.0
    assert ub[0, 1] == (2.0 ** 53 - 1) * 2.0 ** -53 and ub[0, 1] < 1.0


def test_normals_moments_and_ks():
    g = H.normals(12437, H.STREAM_ETA, 0, 0, 1_000_000)
    assert abs(g.mean()) < 5 * 1e-3
    assert abs(g.var() - 1) < 5 * np.sqrt(2 / 1e6)
    assert abs(st.skew(g)) < 5 * np.sqrt(6 / 1e6)
    assert abs(st.kurtosis(g)) < 5 * np.sqrt(24 / 1e6)
    assert st.kstest(g, "norm").pvalue > 1e-3


def test_streams_and_prefix_consistency():
    a = H.normals(1, H.STREAM_ETA, 0, 0, 1003)
    b = H.normals(1, H.STREAM_ETA, 0, 0, 10)
    assert np.array_equal(a[:10], b)  # element k depends only on (block k//4, k%4)
    d = H.normals(1, H.STREAM_DELTA, 0, 0, 1003)
    e = H.normals(1, H.STREAM_ETA, 1, 0, 1003)
    f = H.normals(1, H.STREAM_ETA, 0, 1, 1003)
    for other in (d, e, f):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.15
        assert not np.array_equal(a, other)


def _tiny_setup(p):
    P = synth.tiny_problem(p)
    X = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    Phi = R.phi_dense(X, P.omega, P.lam, P.tau)
    L = R.cholesky(Phi)
    mean_b = R.rhs_mean(X, P.omega, P.z)
    mu = R.solve_chol(Phi, mean_b)
    return P, X, Phi, L, mean_b, mu


N_DRAWS = 20_000


@pytest.mark.parametrize("p", [4, 8])
def test_chi2_cholesky_draws_pass(p):
    P, X, Phi, L, mean_b, mu = _tiny_setup(p)
    rng = np.random.default_rng(100 + p)
    xi = rng.standard_normal((N_DRAWS, p))
    draws = R.draw_chol(Phi, mean_b, xi.T).T  # the oracle's own sampler
    res = S.gaussian_tests(S.whiten_beta(draws, mu, L))
    assert S.passes(res), res
    # one draw at a time is the same sampler
    for s in (0, 7, N_DRAWS - 1):
        assert np.allclose(R.draw_chol(Phi, mean_b, xi[s]), draws[s], rtol=1e-14, atol=1e-14)


def test_draw_chol_by_hand():
    """Phi = [[4, 2], [2, 3]] = L L^T with L = [[2, 0], [1, sqrt 2]];
    mean_rhs = (2, 1) gives mu = Phi^-1 (2, 1) = (1/2, 0); xi = (1, 1) gives
    L^-T xi = ((1 - 2^-1/2) / 2, 2^-1/2).  And L^-T L^-1 = Phi^-1 =
    [[3, -2], [-2, 4]] / 8, the covariance of the draws."""
    Phi = np.array([[4.0, 2.0], [2.0, 3.0]])
    r2 = np.sqrt(2.0)
    beta = R.draw_chol(Phi, np.array([2.0, 1.0]), np.array([1.0, 1.0]))
    assert np.allclose(beta, [0.5 + (1 - 1 / r2) / 2, 1 / r2], rtol=0, atol=1e-15)
    # the deviation part is linear in xi: columns of L^-T from unit vectors
    A = R.draw_chol(Phi, np.zeros(2), np.eye(2))
    assert np.allclose(A @ A.T, np.array([[3.0, -2.0], [-2.0, 4.0]]) / 8, rtol=0, atol=1e-15)
    assert np.allclose(R.draw_chol(Phi, np.array([2.0, 1.0]), np.zeros(2)), [0.5, 0.0],
                       rtol=0, atol=1e-15)


def _cg_sampler_draws(P, X, seed, drop_eta=False):
    draws = np.arange(N_DRAWS)
    eta = H.normals_many(seed, H.STREAM_ETA, 0, draws, P.n)
    delta = H.normals_many(seed, H.STREAM_DELTA, 0, draws, P.p)
    if drop_eta:
        eta = np.zeros_like(eta)
    return R.rhs_b_many(X, P.omega, P.z, P.lam, P.tau, eta, delta)


def test_many_forms_equal_single_forms():
    P, X, Phi, L, mean_b, mu = _tiny_setup(8)
    draws = np.array([0, 5, 17])
    eta = H.normals_many(3, H.STREAM_ETA, 2, draws, P.n)
    delta = H.normals_many(3, H.STREAM_DELTA, 2, draws, P.p)
    B = R.rhs_b_many(X, P.omega, P.z, P.lam, P.tau, eta, delta)
    mv = lambda V: np.column_stack([R.phi_matvec(X, P.omega, P.lam, P.tau, V[:, j])
                                    for j in range(V.shape[1])])
    betas, iters, status = R.pcg_many(mv, B.T, R.precond_inverse(P.lam, P.tau), tol=1e-12)
    for k, t in enumerate(draws):
        e1, d1 = H.eta_delta(3, 2, int(t), P.n, P.p)
        assert np.array_equal(e1, eta[k]) and np.array_equal(d1, delta[k])
        b1 = R.rhs_b(X, P.omega, P.z, P.lam, P.tau, e1, d1)
        assert np.allclose(b1, B[k], rtol=1e-14, atol=1e-14)
        one = R.pcg_solve(X, P.omega, P.lam, P.tau, b1, tol=1e-12)
        assert one.iters == iters[k]
        # Same recurrences; only the summation order of the dot products differs.
        assert np.linalg.norm(one.beta - betas[:, k]) <= 1e-10 * np.linalg.norm(one.beta)


@pytest.mark.parametrize("p", [4, 8])
def test_chi2_prop21_b_and_beta_pass(p):
    """b ~ N(X^T Omega z, Phi) and beta = Phi^-1 b ~ N(mu, Phi^-1) (Prop 2.1),
    with eta, delta from the counter-based normals; beta by PCG to 1e-12."""
    P, X, Phi, L, mean_b, mu = _tiny_setup(p)
    bs = _cg_sampler_draws(P, X, seed=12437 + p)
    assert S.passes(S.gaussian_tests(S.whiten_b(bs, mean_b, L)))
    mv = lambda V: X.T @ (P.omega[:, None] * (X @ V)) + R.prior_precision(P.lam, P.tau)[:, None] * V
    # Rounding can leave a 1e-12 residual short of zero after p steps; allow a
    # few more iterations than the exact-arithmetic bound.
    betas, iters, status = R.pcg_many(mv, bs.T, R.precond_inverse(P.lam, P.tau),
                                      tol=1e-12, max_iter=10 * p)
    assert np.all(status == R.STATUS_OK)
    res = S.gaussian_tests(S.whiten_beta(betas.T, mu, L))
    assert S.passes(res), res


@pytest.mark.parametrize("p", [4, 8])
def test_chi2_negative_control_fails(p):
    """Planted mistake: drop X^T Omega^1/2 eta from b.  Var(b) is then wrong and
    the covariance test must reject it decisively."""
    P, X, Phi, L, mean_b, mu = _tiny_setup(p)
    bs = _cg_sampler_draws(P, X, seed=999 + p, drop_eta=True)
    betas = np.linalg.solve(Phi, bs.T).T
    res = S.gaussian_tests(S.whiten_beta(betas, mu, L))
    assert min(v[1] for v in res.values()) < 1e-6, res
