"""Pins of the oracle's Polya-Gamma sampler (the omega update of the Gibbs
cycle, Supplement S1 step 3): closed-form moments and Laplace transform of
PG(1, c), a two-sample test against the law's defining infinite sum of
weighted exponentials, and the pseudo-response of eq.
pg_augmented_likelihood."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy import stats

from oracle import pg_ref as G
from oracle import philox_ref as H

N = 8000
CS = (0.0, 0.7, -3.0, 12.0, 200.0)


def pg_mean(c):
    """E[PG(1, c)] = tanh(c/2) / (2c), 1/4 at c = 0."""
    return 0.25 if c == 0 else math.tanh(c / 2) / (2 * c)


def pg_var(c):
    """Var[PG(1, c)] = (sinh c - c) sech^2(c/2) / (4 c^3) = (2 tanh(c/2) -
    c sech^2(c/2)) / (4 c^3); 1/24 at c = 0 (series below |c| = 1e-2)."""
    if abs(c) < 1e-2:
        return 1 / 24 - c * c / 240
    e = math.exp(-abs(c))
    sech2 = 4.0 * e / (1.0 + e) ** 2  # sech^2(c/2) without overflow
    return (2 * math.tanh(c / 2) - c * sech2) / (4 * c ** 3)


def pg_laplace(c, s):
    """E[exp(-s omega)] = cosh(c/2) / cosh(sqrt(s/2 + c^2/4))."""
    return math.cosh(c / 2) / math.cosh(math.sqrt(s / 2 + c * c / 4))


def draws(c, n=N, seed=77, draw=0):
    return G.pg_draws(seed, 0, draw, np.full(n, c))


@pytest.fixture(scope="module")
def samples():
    return {c: draws(c) for c in CS}


@pytest.mark.parametrize("c", CS)
def test_moments_match_closed_forms(samples, c):
    w = samples[c]
    m, v = pg_mean(abs(c)), pg_var(abs(c))
    assert np.all(w > 0)
    assert abs(w.mean() - m) <= 5 * math.sqrt(v / N)
    # the sample variance's standard error: sqrt((mu4 - v^2) / N) <= v sqrt(20 / N) here
    assert abs(w.var(ddof=1) - v) <= 5 * v * math.sqrt(20 / N)


@pytest.mark.parametrize("c", (0.0, -3.0, 12.0))
def test_laplace_transform(samples, c):
    w = samples[c]
    for s in (0.5, 2.0, 8.0, 40.0):
        e = np.exp(-s * w)
        assert abs(e.mean() - pg_laplace(c, s)) <= 5 * e.std() / math.sqrt(N) + 1e-12


@pytest.mark.parametrize("c", (0.0, 2.5, 9.0))
def test_matches_the_sum_of_weighted_exponentials(c):
    """PG(1, c) is (1 / (2 pi^2)) sum_k g_k / ((k - 1/2)^2 + c^2 / (4 pi^2)),
    g_k ~ Exp(1) i.i.d.: 400 terms plus the remainder's mean (its spread is
    below 1e-4 of the law's) against the sampler, two-sample KS."""
    rng = np.random.default_rng(5)
    K = 400
    k = np.arange(1, K + 1)
    wts = 1.0 / ((k - 0.5) ** 2 + c * c / (4 * math.pi ** 2))
    kt = np.arange(K + 1, 2_000_001, dtype=np.float64)
    tail = np.sum(1.0 / ((kt - 0.5) ** 2 + c * c / (4 * math.pi ** 2))) + 1.0 / 2_000_000
    ref = (rng.exponential(size=(4000, K)) @ wts + tail) / (2 * math.pi ** 2)
    got = draws(c, n=4000, seed=91)
    assert stats.ks_2samp(got, ref).pvalue > 1e-3


def test_a_wrong_tilt_is_caught():
    """A planted mistake (tilting by |c| instead of |c|/2, i.e. drawing
    PG(1, 2c)) moves the mean by many standard errors."""
    c = 3.0
    bad = G.pg_draws(77, 0, 0, np.full(N, 2 * c))
    assert abs(bad.mean() - pg_mean(c)) > 20 * math.sqrt(pg_var(c) / N)


def test_uniform_stream_layout():
    """Element i's uniforms are the words of blocks (i, 2 | b << 8, chain,
    draw) under key (seed, 0), four per block, in (0, 1)."""
    u = G.Uniforms(11, 3, 5, 42)
    got = [u() for _ in range(9)]
    words = []
    for b in range(3):
        words += H.philox4x64_scalar((42, 2 | (b << 8), 3, 5), (11, 0))
    want = [((w >> 11) + 0.5) * 2.0 ** -53 for w in words[:9]]
    assert got == want and all(0 < x < 1 for x in got)


def test_pg_update_pseudo_response_by_hand():
    """psi = X beta by loops, omega from each element's stream, and
    z = (y - 1/2) / omega on a 4 x 3 design."""
    dense = np.array([[1, 0, 1], [0, 0, 0], [1, 1, 1], [0, 1, 0]], dtype=np.float64)
    X = sp.csr_matrix(dense)
    beta = np.array([0.5, -2.0, 1.25])
    y = np.array([1, 0, 0, 1], dtype=np.uint8)
    omega, z, psi = G.pg_update(X, beta, y, 9, 1, 4)
    assert np.array_equal(psi, [sum(dense[i, j] * beta[j] for j in range(3)) for i in range(4)])
    for i in range(4):
        assert omega[i] == G.pg1_draw(psi[i], G.Uniforms(9, 1, 4, i))
        assert z[i] == (y[i] - 0.5) / omega[i]
    o2, z2, _ = G.pg_update(X, beta, y, 9, 1, 4, idx=[2, 0])
    assert np.array_equal(o2, omega[[2, 0]]) and np.array_equal(z2, z[[2, 0]])


def test_series_ratio_matches_the_terms_and_survives_underflow():
    """a_n / a_0 from its closed form equals the quotient of the terms where
    both are representable, and stays finite where a_0 underflows; extreme
    tilts then draw quickly with the closed-form mean."""
    for x in (0.05, 0.3, 0.64, 0.9, 3.0):
        for n in range(1, 6):
            a0 = G.a_n(0, x)
            assert math.isclose(G.a_ratio(n, x), G.a_n(n, x) / a0, rel_tol=1e-12, abs_tol=1e-300)
    assert G.a_n(0, 2e-4) == 0.0 and G.a_ratio(1, 2e-4) == 0.0
    c = 1e4
    w = draws(c, n=2000, seed=5)
    assert abs(w.mean() - pg_mean(c)) <= 5 * math.sqrt(pg_var(c) / 2000)


def test_right_probability_equals_the_mass_ratio():
    """The log-space weight of the exponential part equals p / (p + q) from
    the masses themselves wherever those are representable, and tends to 0
    (the inverse-Gaussian part) at large tilts."""
    for z in (0.0, 0.3, 1.0, 1.5625, 3.0, 10.0, 40.0):
        p, q = G.mixture_masses(z)
        assert math.isclose(G.right_probability(z), p / (p + q), rel_tol=1e-12)
    assert G.right_probability(5000.0) == 0.0
