"""Convergence theory of Section 2 restated as functions (test pins).

Test infrastructure only: see the package docstring.
"""
from __future__ import annotations

import numpy as np


def sqrt_kappa_rate(kappa):
    """(sqrt(kappa) - 1) / (sqrt(kappa) + 1), the per-iteration contraction of
    the condition-number bound (Theorem 2.1, eq. cg_bound_by_sqrt_cond_num)."""
    s = np.sqrt(kappa)
    return (s - 1.0) / (s + 1.0)


def thm21_bound(kappa, k):
    """2 ((sqrt kappa - 1)/(sqrt kappa + 1))^k  (Theorem 2.1)."""
    return 2.0 * sqrt_kappa_rate(kappa) ** k


def precond_matrix(XtOX, lam, tau):
    """Phi~ = tau^2 Lambda X^T Omega X Lambda + I (eq. prior_preconditioned_matrix)."""
    c = tau * np.asarray(lam, dtype=np.float64)
    return c[:, None] * XtOX * c[None, :] + np.eye(c.size)


def thm24_upper(XtOX, lam, tau):
    """Upper bounds 1 + tau^2 lambda_(k)^2 nu_1(X^T Omega X), k = 1..p
    (Theorem 2.4), lambda_(k) the k-th largest local scale."""
    nu1 = float(np.linalg.eigvalsh(XtOX)[-1])
    lam_sorted = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    return 1.0 + tau ** 2 * lam_sorted ** 2 * nu1


def thm25_kappa(XtOX, lam, tau, m):
    """kappa~_m = 1 + min_{k+l=m} tau^2 lambda_(k+1)^2 nu_{l+1}((X^T Omega X)_(-k))
    (Theorem 2.5, eq. cg_error_bound_under_prior_preconditioner); (A)_(-k)
    removes the rows/columns of the k largest lambdas."""
    lam = np.asarray(lam, dtype=np.float64)
    order = np.argsort(-lam, kind="stable")
    p = lam.size
    best = np.inf
    for k in range(0, m + 1):
        l = m - k
        if k + 1 > p:
            continue
        keep = order[k:]
        sub = XtOX[np.ix_(keep, keep)]
        ev = np.sort(np.linalg.eigvalsh(sub))[::-1]
        if l >= ev.size:
            val = 0.0
        else:
            val = tau ** 2 * lam[order[k]] ** 2 * max(ev[l], 0.0)
        best = min(best, val)
    return 1.0 + best


def thm25_bound(kappa_m, mprime):
    """2 ((kappa~_m^1/2 - 1)/(kappa~_m^1/2 + 1))^m'  (Theorem 2.5)."""
    return 2.0 * sqrt_kappa_rate(kappa_m) ** mprime


def phi_norm(v, Phi):
    return float(np.sqrt(v @ Phi @ v))
