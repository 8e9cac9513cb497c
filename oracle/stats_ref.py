"""Chi-square tests of sampler output against its target Gaussian.

Test infrastructure only: see the package docstring.

Prop 2.1 says b ~ N(X^T Omega z, Phi) and beta = Phi^-1 b ~ N(Phi^-1 X^T
Omega z, Phi^-1).  Given N draws and the exact mean and covariance (from a
Cholesky factor Phi = L L^T), the draws are whitened to w_s ~ N(0, I_p) and
three statistics are formed:

* T1 = N ||mean(w)||^2 ~ chi2(p)                         (mean)
* T2 = N [tr S - ln det S - p] ~ chi2(p(p+1)/2),
  S = N^-1 sum_s w_s w_s^T                               (covariance, known-mean
                                                          likelihood ratio)
* T3 = Pearson chi2 of ||w_s||^2 in 20 equiprobable chi2(p) bins ~ chi2(19)
                                                         (shape)
A test passes when every p-value is at least ``alpha``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.stats as st


def whiten_beta(draws, mu, L):
    """w_s = L^T (beta_s - mu): Cov(beta) = Phi^-1 = L^-T L^-1 => Cov(w) = I."""
    return (np.asarray(draws) - mu) @ L


def whiten_b(draws, mean, L):
    """w_s = L^-1 (b_s - mean): Cov(b) = Phi = L L^T => Cov(w) = I."""
    return sla.solve_triangular(L, (np.asarray(draws) - mean).T, lower=True).T


def gaussian_tests(w, nbins=20):
    """p-values (T1, T2, T3) for whitened draws w [N, p]."""
    w = np.asarray(w, dtype=np.float64)
    N, p = w.shape
    wbar = w.mean(axis=0)
    t1 = N * float(wbar @ wbar)
    p1 = float(st.chi2.sf(t1, p))
    S = (w.T @ w) / N
    sign, logdet = np.linalg.slogdet(S)
    t2 = N * (float(np.trace(S)) - logdet - p)
    p2 = float(st.chi2.sf(t2, p * (p + 1) // 2))
    q = np.sum(w * w, axis=1)
    edges = st.chi2.ppf(np.linspace(0.0, 1.0, nbins + 1), p)
    counts, _ = np.histogram(q, bins=edges)
    expected = N / nbins
    t3 = float(np.sum((counts - expected) ** 2 / expected))
    p3 = float(st.chi2.sf(t3, nbins - 1))
    return {"T1": (t1, p1), "T2": (t2, p2), "T3": (t3, p3)}


def passes(res, alpha=1e-3):
    return all(v[1] >= alpha for v in res.values())
