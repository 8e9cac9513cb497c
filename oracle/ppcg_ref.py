"""Reference (CPU, FP64) of the beta-conditional sampler of Nishimura & Suchard.

Test infrastructure only: see the package docstring.

Notation (Section 1, eq. beta_conditional):
    Phi = X^T Omega X + tau^-2 Lambda^-2,  Omega = diag(omega),
    Lambda = diag(lambda).
We write d_j = tau^-2 lambda_j^-2 for the prior precision and
m_j = (tau lambda_j)^2 = 1/d_j for the inverse of the prior preconditioner
M = tau^-2 Lambda^-2 (Section 2.4).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# Stopping criteria (Supplement S4.2, eq. mean_sq_resid_for_cg_termination and
# the relative readings listed in the design notes).
REL_PRECOND = 0  # ||c*r_k|| <= tol * ||c*b||           (c = tau*lambda)
RMS_PRECOND_ABS = 1  # p^-1/2 ||c*r_k|| <= tol          (the paper's rule)
REL_PLAIN = 2  # ||r_k|| <= tol * ||b||

STATUS_OK, STATUS_NOTCONV, STATUS_BREAKDOWN = 0, 4, 5


def csr_matrix(n, p, row_ptr, col_idx, values=None):
    """X as a SciPy CSR matrix with unit values (binary design)."""
    nnz = int(row_ptr[-1])
    data = np.ones(nnz) if values is None else np.asarray(values, dtype=np.float64)
    return sp.csr_matrix((data, np.asarray(col_idx, dtype=np.int64),
                          np.asarray(row_ptr, dtype=np.int64)), shape=(n, p))


def prior_precision(lam, tau):
    """d_j = tau^-2 lambda_j^-2, the diagonal of the prior term of Phi
    (eq. beta_conditional)."""
    lam = np.asarray(lam, dtype=np.float64)
    return 1.0 / (tau * lam) ** 2


def precond_inverse(lam, tau):
    """m_j = M^-1_jj = (tau lambda_j)^2 for the prior preconditioner
    M = tau^-2 Lambda^-2 (Section 2.4)."""
    lam = np.asarray(lam, dtype=np.float64)
    return (tau * lam) ** 2


def phi_dense(X, omega, lam, tau):
    """Phi = X^T Omega X + tau^-2 Lambda^-2 formed explicitly
    (eq. beta_conditional); the standard method's first step (Section 1)."""
    Xd = X.toarray() if sp.issparse(X) else np.asarray(X, dtype=np.float64)
    xtox = Xd.T @ (np.asarray(omega, dtype=np.float64)[:, None] * Xd)
    return xtox + np.diag(prior_precision(lam, tau))


def phi_matvec(X, omega, lam, tau, v):
    """v -> Phi v through v -> X v and w -> X^T w only (Section 1: Phi v is
    computed without forming Phi)."""
    v = np.asarray(v, dtype=np.float64)
    u = np.asarray(omega, dtype=np.float64) * (X @ v)
    return X.T @ u + prior_precision(lam, tau) * v


def phi_matvec_loops(n, p, row_ptr, col_idx, omega, lam, tau, v):
    """Brute-force Phi v by explicit loops over the non-zeros (tiny inputs)."""
    u = [0.0] * n
    for i in range(n):
        acc = 0.0
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            acc += float(v[int(col_idx[k])])
        u[i] = float(omega[i]) * acc
    out = [0.0] * p
    for i in range(n):
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            out[int(col_idx[k])] += u[i]
    for j in range(p):
        out[j] += float(v[j]) / (tau * float(lam[j])) ** 2
    return np.array(out)


def rhs_mean(X, omega, z):
    """X^T Omega z, the mean of b (Prop 2.1, eq. cg_sampler_target_vector)."""
    return X.T @ (np.asarray(omega, dtype=np.float64) * np.asarray(z, dtype=np.float64))


def rhs_b(X, omega, z, lam, tau, eta, delta):
    """b = X^T Omega z + X^T Omega^1/2 eta + tau^-1 Lambda^-1 delta
    (Prop 2.1, eq. cg_sampler_target_vector)."""
    omega = np.asarray(omega, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    return (X.T @ (omega * np.asarray(z, dtype=np.float64))
            + X.T @ (np.sqrt(omega) * np.asarray(eta, dtype=np.float64))
            + np.asarray(delta, dtype=np.float64) / (tau * lam))


def rhs_b_many(X, omega, z, lam, tau, eta, delta):
    """Prop 2.1's b for many (eta, delta) pairs at once: eta [N, n], delta
    [N, p] -> b [N, p]; row s is ``rhs_b`` of (eta[s], delta[s])."""
    omega = np.asarray(omega, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    mean = X.T @ (omega * np.asarray(z, dtype=np.float64))
    noise = (X.T @ (np.sqrt(omega)[:, None] * np.asarray(eta, dtype=np.float64).T)).T
    return mean[None, :] + noise + np.asarray(delta, dtype=np.float64) / (tau * lam)[None, :]


def cholesky(Phi):
    """Lower Cholesky factor L with Phi = L L^T (the standard method, Section 2.1)."""
    return sla.cholesky(Phi, lower=True)


def solve_chol(Phi, b):
    """beta = Phi^-1 b by Cholesky (the direct method the paper compares to)."""
    c = sla.cho_factor(Phi, lower=True)
    return sla.cho_solve(c, b)


def draw_chol(Phi, mean_rhs, xi):
    """Textbook Cholesky sampler of N(Phi^-1 mean_rhs, Phi^-1):
    beta = mu + L^-T xi with Phi = L L^T, xi ~ N(0, I) (Section 2.1).
    xi is one standard normal vector (p) or one per column (p x N); the
    result has the same shape."""
    L = cholesky(Phi)
    mu = sla.cho_solve((L, True), mean_rhs)
    xi = np.asarray(xi, dtype=np.float64)
    dev = sla.solve_triangular(L.T, xi, lower=False)
    return mu + dev if xi.ndim == 1 else mu[:, None] + dev


@dataclasses.dataclass
class PCGResult:
    beta: np.ndarray
    iters: int
    status: int
    resid_norms: list  # ||c * r_k|| (prior-preconditioned residual) per k
    plain_norms: list  # ||r_k|| per k
    iterates: list | None = None


def stop_threshold(criterion, tol, b, m, p):
    """Right-hand side of the stopping test, in the norm the test uses.

    REL_PRECOND:     ||c*r|| <= tol * ||c*b||   (relative form)
    RMS_PRECOND_ABS: p^-1/2 ||c*r|| <= tol      (eq. mean_sq_resid_for_cg_termination)
    REL_PLAIN:       ||r|| <= tol * ||b||
    """
    if criterion == REL_PRECOND:
        return tol * float(np.sqrt(np.dot(b, m * b)))
    if criterion == RMS_PRECOND_ABS:
        return tol * float(np.sqrt(p))
    if criterion == REL_PLAIN:
        return tol * float(np.linalg.norm(b))
    raise ValueError(criterion)


def pcg(matvec, b, m, beta0=None, tol=1e-10, criterion=REL_PRECOND,
        max_iter=None, keep_iterates=False, threshold=None):
    """Preconditioned conjugate gradient for Phi beta = b.

    Follows the CG algorithm of Supplement S2 (Hestenes-Stiefel form, after
    Golub & Van Loan 11.3.8) with the preconditioner applied through
    v -> M^-1 v only (Section 2.4, eq. preconditioned_system), M^-1 = diag(m).
    The residual is taken as r = b - Phi beta so that the update
    beta <- beta + alpha s descends (the pseudo-code's r = Phi beta - b is a
    sign slip; norms are unaffected).  The prior-preconditioned residual
    r~ = c * r (Supplement S4.2) has ||r~||^2 = <r, m r> = rho.
    """
    b = np.asarray(b, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    p = b.size
    if max_iter is None:
        max_iter = p
    beta = np.zeros(p) if beta0 is None else np.array(beta0, dtype=np.float64)
    r = b - matvec(beta) if beta0 is not None else b.copy()
    z = m * r
    rho = float(np.dot(r, z))
    s = z.copy()
    thr = stop_threshold(criterion, tol, b, m, p) if threshold is None else threshold

    def measure(rho_, r_):
        if criterion == REL_PLAIN:
            return float(np.linalg.norm(r_))
        return float(np.sqrt(max(rho_, 0.0)))

    hist = [float(np.sqrt(max(rho, 0.0)))]
    plain = [float(np.linalg.norm(r))]
    its = [beta.copy()] if keep_iterates else None
    k = 0
    status = STATUS_OK
    while measure(rho, r) > thr:
        if k >= max_iter:
            status = STATUS_NOTCONV
            break
        v = matvec(s)
        sv = float(np.dot(s, v))
        if not np.isfinite(sv) or sv <= 0.0:
            status = STATUS_BREAKDOWN
            break
        alpha = rho / sv
        beta = beta + alpha * s
        r = r - alpha * v
        z = m * r
        rho_new = float(np.dot(r, z))
        s = z + (rho_new / rho) * s
        rho = rho_new
        k += 1
        hist.append(float(np.sqrt(max(rho, 0.0))))
        plain.append(float(np.linalg.norm(r)))
        if keep_iterates:
            its.append(beta.copy())
    return PCGResult(beta, k, status, hist, plain, its)


def pcg_many(matvec_cols, B, m, tol=1e-10, criterion=REL_PRECOND, max_iter=None):
    """Independent preconditioned CG runs, one per column of B [p, N].

    Each column follows exactly the recurrences of ``pcg`` (same scalars, same
    stopping rule, beta0 = 0); columns that have stopped are frozen.  Returns
    (beta [p, N], iters [N], status [N]).  ``matvec_cols`` maps a [p, k] block
    to Phi times it.
    """
    B = np.asarray(B, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    p, N = B.shape
    if max_iter is None:
        max_iter = p
    thr = np.array([stop_threshold(criterion, tol, B[:, j], m, p) for j in range(N)])
    beta = np.zeros((p, N))
    r = B.copy()
    z = m[:, None] * r
    rho = np.sum(r * z, axis=0)
    s = z.copy()
    iters = np.zeros(N, dtype=np.int64)
    status = np.full(N, STATUS_OK)

    def measure():
        if criterion == REL_PLAIN:
            return np.linalg.norm(r, axis=0)
        return np.sqrt(np.maximum(rho, 0.0))

    active = measure() > thr
    while np.any(active):
        over = active & (iters >= max_iter)
        status[over] = STATUS_NOTCONV
        active &= ~over
        if not np.any(active):
            break
        idx = np.nonzero(active)[0]
        v = matvec_cols(s[:, idx])
        sv = np.sum(s[:, idx] * v, axis=0)
        bad = ~np.isfinite(sv) | (sv <= 0.0)
        status[idx[bad]] = STATUS_BREAKDOWN
        ok = ~bad
        idx, v, sv = idx[ok], v[:, ok], sv[ok]
        alpha = rho[idx] / sv
        beta[:, idx] += alpha * s[:, idx]
        r[:, idx] -= alpha * v
        z_new = m[:, None] * r[:, idx]
        rho_new = np.sum(r[:, idx] * z_new, axis=0)
        s[:, idx] = z_new + (rho_new / rho[idx]) * s[:, idx]
        rho[idx] = rho_new
        iters[idx] += 1
        active[:] = False
        active[idx] = measure()[idx] > thr[idx]
    return beta, iters, status


def pcg_solve(X, omega, lam, tau, b, beta0=None, tol=1e-10,
              criterion=REL_PRECOND, max_iter=None, keep_iterates=False):
    """Prior-preconditioned CG on Phi beta = b using sparse matvecs only
    (Sections 2.2-2.4; start beta0 = 0 by default, Section 2.7)."""
    mv = lambda v: phi_matvec(X, omega, lam, tau, v)  # noqa: E731
    return pcg(mv, b, precond_inverse(lam, tau), beta0, tol, criterion,
               max_iter, keep_iterates)


def true_residual(X, omega, lam, tau, b, beta):
    """r = b - Phi beta recomputed from scratch in FP64."""
    return np.asarray(b, dtype=np.float64) - phi_matvec(X, omega, lam, tau, beta)


def criterion_value(criterion, r, b, m):
    """Left-hand side / right-hand side of the stopping rule for a residual r
    (1.0 means exactly at tolerance; see ``stop_threshold``)."""
    p = b.size
    if criterion == REL_PRECOND:
        return float(np.sqrt(np.dot(r, m * r)) / np.sqrt(np.dot(b, m * b)))
    if criterion == RMS_PRECOND_ABS:
        return float(np.sqrt(np.dot(r, m * r) / p))
    if criterion == REL_PLAIN:
        return float(np.linalg.norm(r) / np.linalg.norm(b))
    raise ValueError(criterion)


def error_metrics(beta, beta_ref, scale, Phi=None, mean_rhs=None):
    """Distances of an iterate from a reference solution (FP64).

    rel_l2:     ||beta - beta_ref||_2 / ||beta_ref||_2
    scaled_max: max_j |beta_j - beta_ref_j| / scale_j, scale = tau lambda
                (the prior scale of beta_j, Supplement S4.2; any positive
                scale, e.g. sqrt(M^-1) of a general preconditioner)
    coord_rel:  mean_j |(beta - beta_ref)_j / (beta_ref)_j|, the coordinate-
                wise relative error averaged over the coefficients that
                Section 3.2 plots (coefficients with beta_ref_j = 0 left out)
    secmom_rms: {p^-1 sum_j xi_j^-2 (beta - beta_ref)_j^2}^1/2 with xi_j^2 =
                E[beta_j^2] = mu_j^2 + (Phi^-1)_jj under N(Phi^-1 mean_rhs,
                Phi^-1): eq. cg_sampler_error_metric divided by p^1/2, the
                form plotted beside the RMS residual in Supplement S8.2; only
                when Phi and mean_rhs are given (small p).
    """
    beta = np.asarray(beta, dtype=np.float64)
    ref = np.asarray(beta_ref, dtype=np.float64)
    d = beta - ref
    nr = float(np.linalg.norm(ref))
    out = {
        "rel_l2": float(np.linalg.norm(d) / nr) if nr > 0 else float(np.linalg.norm(d)),
        "scaled_max": float(np.max(np.abs(d) / np.asarray(scale, dtype=np.float64))),
    }
    nz = ref != 0.0
    out["coord_rel"] = float(np.mean(np.abs(d[nz] / ref[nz]))) if np.any(nz) else 0.0
    if Phi is not None and mean_rhs is not None:
        L = cholesky(Phi)
        mu = sla.cho_solve((L, True), mean_rhs)
        Linv = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)
        var = np.sum(Linv * Linv, axis=0)  # diag(Phi^-1) = diag(L^-T L^-1)
        xi2 = mu * mu + var
        out["secmom_rms"] = float(np.sqrt(np.mean(d * d / xi2)))
    return out


def posterior_error_bound(X, omega, lam, tau, b, beta):
    """Rigorous bound ||(beta_k - beta)/c||_2 <= ||c * (b - Phi beta_k)||_2.

    From beta_k - beta = M^-1/2 Phi~^-1 r~_k (Supplement S4.2) and the smallest
    eigenvalue of Phi~ being at least one (Theorem 2.4), c = tau*lambda."""
    c = tau * np.asarray(lam, dtype=np.float64)
    return float(np.linalg.norm(c * true_residual(X, omega, lam, tau, b, beta)))


def adjoint_gradient_dense(Phi, d, beta, g):
    """Gradient of a loss L(beta), beta = Phi^-1 b, with respect to b,
    log lambda and log tau, given g = dL/dbeta.

    Differentiating Phi beta = b (eq. linear_system_for_cg_sampler) gives
    dL = a^T (db - dPhi beta) with a = Phi^-1 g (Phi symmetric).  Only the prior
    term d_j = exp(-2 log tau - 2 log lambda_j) of Phi depends on lambda, tau,
    so dL/dlog lambda_j = 2 d_j a_j beta_j and dL/dlog tau = sum_j of the same.
    Here a is computed by Cholesky.
    """
    a = solve_chol(Phi, g)
    gl = 2.0 * d * a * beta
    return a, gl, float(np.sum(gl))


def sampler_draw(X, omega, z, lam, tau, eta, delta, tol=1e-10,
                 criterion=REL_PRECOND, max_iter=None):
    """One CG-sampler draw (Prop 2.1): form b from (eta, delta), then solve
    Phi beta = b by prior-preconditioned CG from beta0 = 0."""
    b = rhs_b(X, omega, z, lam, tau, eta, delta)
    return b, pcg_solve(X, omega, lam, tau, b, None, tol, criterion, max_iter)


# ---- general diagonal prior and preconditioner (Supplement S4.3) ----
# Coefficients estimated without shrinkage (an intercept, effects of
# interest) get independent N(0, sigma_j^2) priors, sigma_j = infinity for a
# flat prior: Phi = X^T Omega X + diag(d) with d_j = sigma_j^-2 (0 when flat)
# for them and tau^-2 lambda_j^-2 for the rest, and the preconditioner
# becomes M = diag(gamma^-2, tau^-2 lambda^-2) for scales gamma_j chosen by
# the caller (the supplement suggests c times a posterior scale estimate).
# Here d is any non-negative prior precision and m = M^-1's diagonal.


def phi_dense_general(X, omega, d):
    """Phi = X^T Omega X + diag(d) formed explicitly (small problems only)."""
    XO = X.multiply(np.asarray(omega, dtype=np.float64)[:, None]).tocsr()
    Phi = (X.T @ XO).toarray()
    Phi[np.diag_indices_from(Phi)] += np.asarray(d, dtype=np.float64)
    return Phi


def phi_matvec_general(X, omega, d, v):
    """v -> Phi v = X^T (omega * (X v)) + d * v through the two products only."""
    v = np.asarray(v, dtype=np.float64)
    return X.T @ (np.asarray(omega, dtype=np.float64) * (X @ v)) + np.asarray(d) * v


def phi_diag(X, omega, d):
    """diag(Phi) = sum over the non-zeros of column j of omega_i (X binary)
    plus d_j: the inverse of the Jacobi preconditioner's diagonal."""
    return np.asarray(X.T @ np.asarray(omega, dtype=np.float64)).ravel() + np.asarray(d)


def rhs_b_general(X, omega, z, d, eta, delta):
    """Prop 2.1 with the prior precision diag(d):
    b = X^T Omega z + X^T Omega^1/2 eta + diag(d)^1/2 delta, so that
    b ~ N(X^T Omega z, X^T Omega X + diag(d)) = N(X^T Omega z, Phi)."""
    omega = np.asarray(omega, dtype=np.float64)
    y = omega * np.asarray(z, dtype=np.float64) + np.sqrt(omega) * np.asarray(eta)
    return X.T @ y + np.sqrt(np.asarray(d, dtype=np.float64)) * np.asarray(delta)


def pcg_solve_general(X, omega, d, m, b, beta0=None, tol=1e-10,
                      criterion=REL_PRECOND, max_iter=None):
    """Preconditioned CG (the recurrences of ``pcg``) on
    (X^T Omega X + diag(d)) beta = b with M^-1 = diag(m)."""
    mv = lambda v: phi_matvec_general(X, omega, d, v)  # noqa: E731
    return pcg(mv, b, m, beta0, tol, criterion, max_iter)


# ---- initial vector (Supplement S4.1: choice of initial vector) ----
def warm_start_accumulate(acc, beta, lam_prev, tau_prev):
    """Running sum of the draws rescaled by the shrinkage scales they were
    drawn under: acc + beta^(i) / (tau^(i-1) lambda^(i-1))."""
    return np.asarray(acc, dtype=np.float64) + np.asarray(beta, dtype=np.float64) / (
        tau_prev * np.asarray(lam_prev, dtype=np.float64))


def warm_start_vector(acc, count, lam, tau):
    """beta0 = tau lambda * (acc / count): the estimate of E[beta / (tau lambda)]
    rescaled by the scales the next draw is conditioned on."""
    return tau * np.asarray(lam, dtype=np.float64) * (np.asarray(acc, dtype=np.float64) / count)


def unshrunk_prior_precond(sigma_inv2, draws_q, c, lam, tau):
    """Prior precision d and preconditioner inverse m of Supplement S4.3 when
    the leading q + 1 coefficients are unshrunk: d_j = sigma_j^-2 (0 for a
    flat prior) and m_j = gamma_j^2 = (c eta_hat_j)^2 with eta_hat_j^2 the
    sample variance (divisor N - 1) of that coefficient over the N earlier
    draws in `draws_q` (N x (q + 1)); the rest d_j = tau^-2 lambda_j^-2 and
    m_j = (tau lambda_j)^2.  `lam` has all p entries (its leading q + 1 are
    not used)."""
    sigma_inv2 = np.asarray(sigma_inv2, dtype=np.float64)
    q1 = sigma_inv2.size
    d = prior_precision(lam, tau)
    m = precond_inverse(lam, tau)
    if q1:
        d[:q1] = sigma_inv2
        m[:q1] = c * c * np.var(np.asarray(draws_q, dtype=np.float64), axis=0, ddof=1)
    return d, m


def jacobi_precond_inverse(X, omega, d):
    """M^-1 of the Jacobi preconditioner M = diag(Phi_11, ..., Phi_pp)
    (Section 3.3, the alternative the paper compares against)."""
    return 1.0 / phi_diag(X, omega, d)


def choose_preconditioner(iters_prior, iters_jacobi):
    """The adaptive choice of Supplement S5: the preconditioner that reached
    the stopping rule in fewer iterations on the same draw (one pass-pair
    each, so iterations measure cost; the Jacobi diagonal's extra column pass
    is why a tie keeps the prior preconditioner, the paper's first choice)."""
    return "jacobi" if iters_jacobi < iters_prior else "prior"
