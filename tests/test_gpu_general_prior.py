"""GPU parity of the general diagonal prior and preconditioner (Supplement
S4.3): a flat-prior intercept column and N(0, sigma^2) coefficients beside
shrunk ones, the Jacobi preconditioner from diag(Phi), and warm starts —
against the oracle's Cholesky solution of the same b (1e-10 relative in FP64
at tight tolerance, 1e-5 in the FP32 form)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
import paper_1810_12437_amd as pk  # noqa: E402
import synth  # noqa: E402
from oracle import philox_ref as H  # noqa: E402
from oracle import ppcg_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def with_intercept(P):
    """P's design with a column of ones prepended (column 0: the intercept)."""
    rows = []
    for i in range(P.n):
        cols = P.col_idx[P.row_ptr[i]:P.row_ptr[i + 1]].astype(np.int64) + 1
        rows.append(np.concatenate([[0], cols]))
    row_ptr = np.zeros(P.n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col_idx = np.concatenate(rows).astype(np.int32)
    return P.n, P.p + 1, row_ptr, col_idx


def setup(n=3000, p=400, q=2, seed=5):
    P = synth.scaled_problem(n, p, seed=seed, tau=2e-2)
    n, p1, row_ptr, col_idx = with_intercept(P)
    X = pk.Matrix(n, p1, row_ptr, col_idx)
    Xs = R.csr_matrix(n, p1, row_ptr, col_idx)
    lam = np.concatenate([[1.0], P.lam])
    d = 1.0 / (P.tau * lam) ** 2
    d[0] = 0.0                  # flat prior on the intercept
    d[1:q + 1] = 1.0 / 9.0      # sigma = 3 for q effects of interest
    Phi = R.phi_dense_general(Xs, P.omega, d)
    psi = np.sqrt(np.diag(np.linalg.inv(Phi)))
    m = (P.tau * lam) ** 2
    m[:q + 1] = (2.0 * psi[:q + 1]) ** 2   # gamma = c psi, c = 2
    return P, X, Xs, d, m, Phi


def t64(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_phi_diag_matches_oracle():
    P, X, Xs, d, m, Phi = setup()
    got = pk.phi_diag(X, t64(P.omega), t64(d)).cpu().numpy()
    ref = R.phi_diag(Xs, P.omega, d)
    say("[phi_diag] rel err", rel(got, ref))
    assert rel(got, ref) <= 1e-13
    got32 = pk.phi_diag(X, t64(P.omega).float(), t64(d)).cpu().numpy()
    ref32 = R.phi_diag(Xs, np.float32(P.omega).astype(np.float64), d)
    assert rel(got32, ref32) <= 1e-13


def test_draw_general_matches_oracle():
    P, X, Xs, d, m, Phi = setup()
    for draw_index in (0, 3):
        eta, delta = H.eta_delta(41, 0, draw_index, P.n, Phi.shape[0])
        b = R.rhs_b_general(Xs, P.omega, P.z, d, eta, delta)
        exact = R.solve_chol(Phi, b)
        beta, info = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 41, 0, draw_index,
                                     precond_inv=t64(m), tol=1e-13)
        e = rel(beta.cpu().numpy(), exact)
        say(f"[draw_general] draw {draw_index} iters {info['iters']} rel err {e:.2e}")
        assert info["status"] == pk.OK and e <= 1e-10


def test_solve_general_jacobi_and_prior_preconditioners():
    """Both preconditioners reach the Cholesky solution; the iteration counts
    are reported (the paper compares the two, Section 2.4)."""
    P, X, Xs, d, m, Phi = setup(seed=6)
    b = np.random.default_rng(2).standard_normal(Phi.shape[0])
    exact = R.solve_chol(Phi, b)
    diag = pk.phi_diag(X, t64(P.omega), t64(d))
    its = {}
    for name, mi in (("prior", t64(m)), ("jacobi", 1.0 / diag)):
        beta, info = pk.solve_general(X, t64(P.omega), t64(d), t64(b), precond_inv=mi, tol=1e-13)
        e = rel(beta.cpu().numpy(), exact)
        its[name] = info["iters"]
        say(f"[solve_general] {name}: iters {info['iters']} rel err {e:.2e}")
        assert info["status"] == pk.OK and e <= 1e-10
        ref = R.pcg_solve_general(Xs, P.omega, d, mi.cpu().numpy(), b, tol=1e-13)
        assert abs(info["iters"] - ref.iters) <= max(3, 0.05 * ref.iters)


def test_warm_start_from_the_solution_stops_at_once():
    P, X, Xs, d, m, Phi = setup(seed=7)
    b = np.random.default_rng(4).standard_normal(Phi.shape[0])
    exact = R.solve_chol(Phi, b)
    _, cold = pk.solve_general(X, t64(P.omega), t64(d), t64(b), precond_inv=t64(m), tol=1e-8)
    beta, warm = pk.solve_general(X, t64(P.omega), t64(d), t64(b), precond_inv=t64(m),
                                  beta0=t64(exact), tol=1e-8)
    say(f"[warm start] cold {cold['iters']} warm {warm['iters']}")
    assert warm["iters"] <= 1 and cold["iters"] > 10
    assert rel(beta.cpu().numpy(), exact) <= 1e-8


def test_general_prior_reduces_to_the_shrinkage_prior():
    """prior_prec = tau^-2 lambda^-2 with the default preconditioner gives the
    ppcg_draw draw (same b up to the rounding of sqrt(d) against 1/(tau
    lambda))."""
    P = synth.scaled_problem(3000, 400, seed=8, tau=2e-2)
    X = pk.Matrix.from_problem(P)
    d = R.prior_precision(P.lam, P.tau)
    a, ia = pk.draw(X, t64(P.omega), t64(P.z), t64(P.lam), P.tau, 5, 1, 2, tol=1e-12)
    b_, ib = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 5, 1, 2, tol=1e-12)
    say(f"[reduces] iters {ia['iters']} {ib['iters']} rel diff {rel(b_.cpu().numpy(), a.cpu().numpy()):.2e}")
    assert rel(b_.cpu().numpy(), a.cpu().numpy()) <= 1e-10


def test_draw_general_f32_matches_f64_oracle():
    P, X, Xs, d, m, Phi = setup(seed=9)
    c32 = lambda a: np.float32(a).astype(np.float64)  # noqa: E731
    eta, delta = H.eta_delta(13, 0, 0, P.n, Phi.shape[0])
    Phi32 = R.phi_dense_general(Xs, c32(P.omega), d)
    b = R.rhs_b_general(Xs, c32(P.omega), c32(P.z), d, eta, delta)
    exact = R.solve_chol(Phi32, b)
    beta, info = pk.draw_general(X, t64(P.omega).float(), t64(P.z).float(), t64(d), 13, 0, 0,
                                 precond_inv=t64(m), tol=1e-8)
    e = rel(beta.double().cpu().numpy(), exact)
    say(f"[draw_general f32] iters {info['iters']}+{info['refine_iters']} rel err {e:.2e}")
    assert info["status"] == pk.OK and e <= 1e-5


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_warm_start_vector_matches_oracle(dt):
    """The running sum and the start vector against the oracle's, with the
    shrinkage scales changing between draws as they do in the Gibbs sampler."""
    p = 1537
    rng = np.random.default_rng(17)
    ws = pk.WarmStart(p)
    acc = np.zeros(p)
    for k in range(4):
        beta = rng.standard_normal(p)
        lam = np.exp(rng.standard_normal(p))
        tau = float(np.exp(rng.standard_normal()))
        if dt == torch.float32:
            beta, lam = np.float32(beta).astype(np.float64), np.float32(lam).astype(np.float64)
        ws.add(t64(beta).to(dt), t64(lam).to(dt), tau)
        acc = R.warm_start_accumulate(acc, beta, lam, tau)
    got_acc = ws.acc.cpu().numpy()
    say(f"[warm start {dt}] acc rel err {rel(got_acc, acc):.2e}")
    assert np.allclose(got_acc, acc, rtol=1e-15, atol=0)
    lam = np.exp(rng.standard_normal(p))
    if dt == torch.float32:
        lam = np.float32(lam).astype(np.float64)
    got = ws.vector(t64(lam).to(dt), 0.3).double().cpu().numpy()
    ref = R.warm_start_vector(acc, 4, lam, 0.3)
    if dt == torch.float32:
        ref = np.float32(ref).astype(np.float64)
        assert np.array_equal(got, ref)
    else:
        assert np.allclose(got, ref, rtol=1e-15, atol=0)


def test_warm_start_from_past_draws():
    """Draws from one conditional: the start vector is the sample mean of 16
    draws, whose squared Phi-norm distance to the conditional mean mu (the
    target Supplement S4.1 sets for the start) has expectation p / 16 against p
    for the previous draw; CG from it reaches the Cholesky solution.  The
    iteration counts are reported: the paper finds the initial vector changes
    them by about 10% at most."""
    P = synth.scaled_problem(3000, 400, seed=10, tau=2e-2)
    X = pk.Matrix.from_problem(P)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    d = R.prior_precision(P.lam, P.tau)
    lam = t64(P.lam)
    ws = pk.WarmStart(P.p)
    assert ws.vector(lam, P.tau) is None
    for k in range(16):
        beta, _ = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 3, 0, k, tol=1e-10)
        ws.add(beta, lam, P.tau)
    prev = beta.cpu().numpy()
    beta0 = ws.vector(lam, P.tau)
    Phi = R.phi_dense_general(Xs, P.omega, d)
    eta, delta = H.eta_delta(3, 0, 16, P.n, P.p)
    exact = R.solve_chol(Phi, R.rhs_b_general(Xs, P.omega, P.z, d, eta, delta))
    mu = R.solve_chol(Phi, Xs.T @ (P.omega * P.z))
    phi_err = lambda v: float((v - mu) @ Phi @ (v - mu))  # noqa: E731
    e_mean, e_prev = phi_err(beta0.cpu().numpy()), phi_err(prev)
    _, cold = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 3, 0, 16, tol=1e-8)
    beta, warm = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 3, 0, 16, beta0=beta0,
                                 tol=1e-8)
    say(f"[warm start from draws] Phi-norm^2 to mu: mean {e_mean:.1f} previous draw "
        f"{e_prev:.1f} (p = {P.p}); iters cold {cold['iters']} warm {warm['iters']}")
    assert e_mean < 0.25 * e_prev
    assert rel(beta.cpu().numpy(), exact) <= 1e-6


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_unshrunk_scales_match_oracle(dt):
    """Running moments of the leading q + 1 coefficients over 6 draws, then
    d and M^-1 of Supplement S4.3, against the oracle's sample variance; a
    coefficient that never moved gets NaN (a solve with it breaks down)."""
    rng = np.random.default_rng(31)
    p, q1, N = 700, 5, 6
    draws = rng.standard_normal((N, p)) * np.array([0.2, 1.0, 3.0, 10.0, 0.0] + [1.0] * (p - 5))
    draws[:, :q1] += np.array([5.0, -1.0, 0.0, 30.0, 2.0])
    lam = np.exp(rng.standard_normal(p))
    if dt == torch.float32:
        draws, lam = np.float32(draws).astype(np.float64), np.float32(lam).astype(np.float64)
    mean = torch.zeros(q1, dtype=torch.float64, device=DEV)
    m2 = torch.zeros_like(mean)
    for k in range(N):
        pk.moments_update(mean, m2, t64(draws[k]).to(dt), k + 1)
    sig = np.array([0.0, 0.25, 1e-2, 0.0, 1.0])
    d, m = pk.unshrunk_setup(t64(lam).to(dt), 0.03, sigma_inv2=t64(sig), m2=m2, count=N, c=2.0)
    d_ref, m_ref = R.unshrunk_prior_precond(sig, draws[:, :q1], 2.0, lam, 0.03)
    got_d, got_m = d.cpu().numpy(), m.cpu().numpy()
    assert np.allclose(mean.cpu().numpy(), draws[:, :q1].mean(axis=0), rtol=1e-13, atol=1e-13)
    assert np.allclose(got_d, d_ref, rtol=1e-15, atol=0)
    assert np.isnan(got_m[4]) and m_ref[4] == 0.0
    assert np.allclose(got_m[:4], m_ref[:4], rtol=1e-12, atol=0)
    assert np.allclose(got_m[q1:], m_ref[q1:], rtol=1e-15, atol=0)
    d0, m0 = pk.unshrunk_setup(t64(lam).to(dt), 0.03)
    assert np.allclose(d0.cpu().numpy(), R.prior_precision(lam, 0.03), rtol=1e-15, atol=0)
    assert np.allclose(m0.cpu().numpy(), R.precond_inverse(lam, 0.03), rtol=1e-15, atol=0)


def test_jacobi_precond_matches_oracle():
    P, X, Xs, d, m, Phi = setup(seed=12)
    got = pk.jacobi_precond(X, t64(P.omega), t64(d)).cpu().numpy()
    ref = R.jacobi_precond_inverse(Xs, P.omega, d)
    assert rel(got, ref) <= 1e-13


def duplicated_pairs(n=3000, p=400, pairs=100, seed=5):
    """Binary design whose first 2 * pairs columns come in identical pairs,
    weakly shrunk (tau = 1, lambda log-uniform in [1, 10]); the rest strongly
    shrunk.  Jacobi scaling leaves eigenvalues near d / (2 a) for each pair,
    the prior preconditioner none below 1."""
    rng = np.random.default_rng(seed)
    dense = rng.random((n, p)) < 0.02
    for k in range(pairs):
        col = rng.random(n) < rng.uniform(0.05, 0.3)
        dense[:, 2 * k] = col
        dense[:, 2 * k + 1] = col
    Xs = sp.csr_matrix(dense.astype(np.float64))
    omega = rng.gamma(1.0, 0.25, n) + 0.01
    z = rng.standard_normal(n)
    lam = np.full(p, 1e-3)
    lam[:2 * pairs] = np.exp(rng.uniform(0.0, np.log(10.0), 2 * pairs))
    d = R.prior_precision(lam, 1.0)
    X = pk.Matrix(n, p, Xs.indptr.astype(np.int64), Xs.indices.astype(np.int32))
    return X, Xs, omega, z, d


@pytest.mark.parametrize("case", ["jacobi_wins", "prior_wins"])
def test_switch_choice_and_draws(case):
    """The switch's trial picks the preconditioner the oracle's CG needs fewer
    iterations with (cases chosen with a wide margin), returns that draw (it
    matches Cholesky), and the next draws use the kept choice until the next
    trial."""
    if case == "jacobi_wins":
        P = synth.scaled_problem(3000, 400, seed=5, tau=2e-2)
        X = pk.Matrix.from_problem(P)
        Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
        d = R.prior_precision(P.lam, P.tau)
        omega, z = P.omega, P.z
        Phi = R.phi_dense_general(Xs, omega, d)
    else:
        X, Xs, omega, z, d = duplicated_pairs()
        Phi = R.phi_dense_general(Xs, omega, d)
    n, p = Xs.shape
    bref = np.random.default_rng(3).standard_normal(p)
    ip = R.pcg_solve_general(Xs, omega, d, 1.0 / d, bref, tol=1e-8).iters
    ij = R.pcg_solve_general(Xs, omega, d, R.jacobi_precond_inverse(Xs, omega, d), bref,
                             tol=1e-8).iters
    want = R.choose_preconditioner(ip, ij)
    S = pk.Switch(p, period=3)
    for k in range(4):
        beta, info = S.draw(X, t64(omega), t64(z), t64(d), 7, 0, k, tol=1e-12)
        st = S.state()
        eta, delta = H.eta_delta(7, 0, k, n, p)
        exact = R.solve_chol(Phi, R.rhs_b_general(Xs, omega, z, d, eta, delta))
        e = rel(beta.cpu().numpy(), exact)
        say(f"[switch {case}] draw {k}: {st} iters {info['iters']} rel err {e:.2e} "
            f"(oracle at 1e-8: prior {ip}, jacobi {ij})")
        assert st["choice"] == want and st["draws"] == k + 1
        assert info["status"] == pk.OK and e <= (1e-10 if case == "jacobi_wins" else 1e-7)
        if k in (0, 3):   # trials
            chosen = st["iters_jacobi"] if want == "jacobi" else st["iters_prior"]
            assert info["iters"] + info["refine_iters"] == chosen
    S.close()
