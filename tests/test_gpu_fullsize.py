"""Parity at the full n = 1e5, p = 2e4 workload, in the launch configuration
bench.py times, against the oracle's stored solution (written by
tests/golden/make_c1_reference.py, oracle only) and the oracle's FP64 matvec."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1810_12437_amd as pk  # noqa: E402
import synth  # noqa: E402
from oracle import ppcg_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "c1_draw0_reference.npz")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def c1():
    say("[fullsize] generating n=1e5 p=2e4")
    P = synth.make_problem("c1")
    return P, pk.Matrix.from_problem(P), np.load(GOLD)


def _vecs(P, dt):
    return (torch.as_tensor(P.omega, device="cuda").to(dt), torch.as_tensor(P.z, device="cuda").to(dt),
            torch.as_tensor(P.lam, device="cuda").to(dt))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_f32_draw_matches_oracle_at_1e_5(c1):
    P, X, g = c1
    assert int(g["nnz"]) == P.nnz
    om, z, lam = _vecs(P, torch.float32)
    beta, info = pk.draw(X, om, z, lam, P.tau, int(g["seed"]), int(g["chain"]), int(g["draw"]),
                         tol=1e-6)
    err = _rel(beta.cpu().numpy(), g["beta_f32"])
    say(f"   f32 tol 1e-6: iters {info['iters']}+{info['refine_iters']} err {err:.2e} "
        f"true/tol {info['resid_true']:.3f}")
    assert info["status"] == 0
    assert info["resid_true"] <= 1.0
    assert err <= 1e-5
    _check_prior_scaled(P, g, beta.double().cpu().numpy(), g["beta_f32"], f32=True)


def test_f64_draw_matches_oracle_at_1e_10(c1):
    P, X, g = c1
    om, z, lam = _vecs(P, torch.float64)
    beta, info = pk.draw(X, om, z, lam, P.tau, int(g["seed"]), int(g["chain"]), int(g["draw"]),
                         tol=1e-12)
    err = _rel(beta.cpu().numpy(), g["beta_f64"])
    say(f"   f64 tol 1e-12: iters {info['iters']} (oracle {int(g['iters_f64'])}) err {err:.2e}")
    assert info["status"] == 0 and info["resid_true"] <= 1.0
    assert abs(info["iters"] - int(g["iters_f64"])) <= 10
    assert err <= 1e-10
    _check_prior_scaled(P, g, beta.cpu().numpy(), g["beta_f64"], f32=False)


def _check_prior_scaled(P, g, got, ref, f32):
    """Per coordinate, on the prior scale tau lambda_j: both the draw and the
    stored oracle solution are within ||tau lambda (b - Phi beta)|| of the
    exact solution (the smallest eigenvalue of the preconditioned Phi is at
    least one, Theorem 2.4), so they differ by at most the sum of the two
    bounds (residuals recomputed by the oracle in FP64)."""
    from oracle import philox_ref as H
    c = (lambda a: np.float32(a).astype(np.float64)) if f32 else (lambda a: a)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    eta, delta = H.eta_delta(int(g["seed"]), int(g["chain"]), int(g["draw"]), P.n, P.p)
    b = R.rhs_b(Xs, c(P.omega), c(P.z), c(P.lam), P.tau, eta, delta)
    ref = np.asarray(ref, np.float64)
    bound = (R.posterior_error_bound(Xs, c(P.omega), c(P.lam), P.tau, b, got)
             + R.posterior_error_bound(Xs, c(P.omega), c(P.lam), P.tau, b, ref))
    e = R.error_metrics(got, ref, P.tau * c(P.lam))
    say(f"   prior-scaled max error {e['scaled_max']:.2e} (bound {bound:.2e}), "
        f"mean coordinate-wise relative {e['coord_rel']:.2e}")
    assert e["scaled_max"] <= bound


def test_phi_matvec_full_size(c1):
    P, X, _ = c1
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    v = np.random.default_rng(1).standard_normal(P.p)
    ref = R.phi_matvec(Xs, P.omega, P.lam, P.tau, v)
    om, _, lam = _vecs(P, torch.float64)
    got = pk.phi_matvec(X, om, lam, P.tau, torch.as_tensor(v, device="cuda")).cpu().numpy()
    assert _rel(got, ref) <= 1e-13
    om32, _, lam32 = _vecs(P, torch.float32)
    got32 = pk.phi_matvec(X, om32, lam32, P.tau,
                          torch.as_tensor(v, device="cuda").float()).cpu().numpy()
    c = lambda a: np.float32(a).astype(np.float64)  # noqa: E731
    ref32 = R.phi_matvec(Xs, c(P.omega), c(P.lam), P.tau, c(v))
    assert _rel(got32, ref32) <= 1e-5


def test_adjoint_eight_chains_full_size(c1):
    """The adjoint form at full size: 8 chains on the n = 1e5, p = 2e4 design
    (per-chain omega, z, lambda, tau), loss sum_j w_j beta_j^2 with w ~ U(0, 1).
    Dense Cholesky is out of reach here, so the checks are those that hold at
    any size: the adjoint solve's FP64 true residual Phi a - g, recomputed by
    the oracle, meets the rule (tol 1e-10); grad log lambda_j = 2 d_j a_j beta_j and grad
    log tau = its sum, recomputed by the oracle from the returned a and beta
    (1e-12); and for one chain a central difference of the loss in log tau
    (losses from solves at 1e-13, step 1e-4) agrees with grad log tau to 1e-5."""
    P, X, _ = c1
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    chains = synth.shared_x_chains(P, 8, seed=1815)
    rng = np.random.default_rng(1814)
    t = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    for c, (om, z, lam, tau) in enumerate(chains):
        w = rng.uniform(0.0, 1.0, P.p)
        b = rng.standard_normal(P.p)
        beta, info = pk.solve(X, t(om), t(lam), tau, t(b), tol=1e-12)
        g = 2.0 * t(w) * beta
        gb, gl, gt, ia = pk.solve_backward(X, t(om), t(lam), tau, beta, g, tol=1e-10)
        a, bt, gn = gb.cpu().numpy(), beta.cpu().numpy(), g.cpu().numpy()
        cm = tau * np.asarray(lam)
        r = gn - R.phi_matvec(Xs, om, lam, tau, a)
        rule = float(np.linalg.norm(cm * r) / (1e-10 * np.linalg.norm(cm * gn)))
        d = R.prior_precision(lam, tau)
        gl_ref = 2.0 * d * a * bt
        egl = float(np.max(np.abs(gl.cpu().numpy() - gl_ref) / np.maximum(np.abs(gl_ref), 1e-300)))
        say(f"   adjoint chain {c}: iters {info['iters']}/{ia['iters']} rule {rule:.3f} "
            f"grad log lambda rel {egl:.1e}")
        assert info["status"] == pk.OK and ia["status"] == pk.OK
        assert rule <= 1.0 + 1e-6
        assert egl <= 1e-12
        assert abs(float(gt.item()) - gl_ref.sum()) <= 1e-12 * np.abs(gl_ref).sum()
        if c == 0:
            h = 1e-4
            loss = []
            for sgn in (1.0, -1.0):
                bs, _ = pk.solve(X, t(om), t(lam), tau * np.exp(sgn * h), t(b), tol=1e-13)
                loss.append(float((w * bs.cpu().numpy() ** 2).sum()))
            fd = (loss[0] - loss[1]) / (2 * h)
            say(f"   chain 0 d loss / d log tau: adjoint {float(gt.item()):.8e} FD {fd:.8e}")
            assert abs(fd - float(gt.item())) <= 1e-5 * abs(fd)


def _golden_rhs(P, g):
    from oracle import philox_ref as H
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    eta, delta = H.eta_delta(int(g["seed"]), int(g["chain"]), int(g["draw"]), P.n, P.p)
    return R.rhs_b(Xs, P.omega, P.z, P.lam, P.tau, eta, delta)


@pytest.mark.parametrize("dt", [pk.F64, pk.F32], ids=["f64", "f32"])
def test_restart_steps_full_size(c1, dt):
    """One and two CG iterations at n = 1e5, p = 2e4, in the launch
    configuration the benchmark times, from zero, from the oracle's iterate
    20 and from the stored converged solution, against the oracle: FP64 to
    1e-10 and FP32 to 1e-5 (norm-wise and prior-scaled maximum), wherever two
    summation orders of the oracle agree (the reasoning is in
    tests/test_gpu_iterates.py)."""
    from tests.test_gpu_iterates import Oracle, check_restart_steps, gpu_steps, shrinkage
    P, X, g = c1
    b = _golden_rhs(P, g)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    starts = [("zero", None),
              ("K0=20", R.pcg_solve(Xs, P.omega, P.lam, P.tau, b, tol=0.0, max_iter=20).beta),
              ("converged", np.asarray(g["beta_f64"], np.float64))]
    d, m = shrinkage(P, dt)
    check_restart_steps("c1", Oracle(P, d, m, dt), gpu_steps(X, P, dt), b, starts, dt)


def test_flat_prior_intercept_full_size(c1):
    """The use case of Supplement S4.3 at n = 1e5, p = 2e4: column 0 of the
    design set to ones (an intercept with 1e5 entries: five FP64 panels of
    20,471 rows and three FP32 panels of 40,943, every part longer than one
    wavefront sums whole, so cut into pieces), a flat prior on it (prior
    precision 0) with gamma_0^2 = 4 / sum(omega) (c = 2 times the scale of
    the intercept given the rest), the shrinkage prior on the others.
    * One and two iterations from zero and from the oracle's iterate 20
      against the oracle: FP64 1e-10, FP32 1e-5.
    * A draw at tol 1e-10: the rule holds on the FP64 true residual
      recomputed by the oracle.
    * A solve at tol 1e-12 against the oracle's CG at the same tolerance:
      1e-10."""
    from tests.test_gpu_iterates import Oracle, add_dense, check_restart_steps, tdev
    from oracle import philox_ref as H
    P0, _, _ = c1
    P = add_dense(P0, col=0)
    X = pk.Matrix.from_problem(P)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    d = R.prior_precision(P.lam, P.tau)
    m = R.precond_inverse(P.lam, P.tau)
    d[0] = 0.0
    m[0] = 4.0 / float(np.sum(P.omega))
    t64 = lambda a: torch.as_tensor(np.asarray(a, np.float64), device="cuda")  # noqa: E731
    rng = np.random.default_rng(1817)
    b = R.rhs_b_general(Xs, P.omega, P.z, d, rng.standard_normal(P.n), rng.standard_normal(P.p))
    for dt in (pk.F64, pk.F32):
        cast = (lambda a: a) if dt == pk.F64 else (lambda a: np.float32(a).astype(np.float64))

        def gpu(bv, beta0, K, dt=dt):
            beta, info = pk.solve_general(X, tdev(P.omega, dt), t64(d), tdev(bv, dt),
                                          precond_inv=t64(m),
                                          beta0=None if beta0 is None else tdev(beta0, dt),
                                          tol=0.0, max_iter=K, refine=0)
            return beta.double().cpu().numpy(), info

        start = R.pcg_solve_general(Xs, cast(P.omega), d, m, cast(b), tol=0.0, max_iter=20).beta
        check_restart_steps("c1 intercept", Oracle(P, d, m, dt), gpu, b,
                            [("zero", None), ("K0=20", start)], dt)
    # a draw at the configured tolerance: the rule on the FP64 true residual
    beta, info = pk.draw_general(X, t64(P.omega), t64(P.z), t64(d), 12437, 0, 3,
                                 precond_inv=t64(m), tol=1e-10)
    eta, delta = H.eta_delta(12437, 0, 3, P.n, P.p)
    bd = R.rhs_b_general(Xs, P.omega, P.z, d, eta, delta)
    got = beta.cpu().numpy()
    rule = R.criterion_value(R.REL_PRECOND, bd - R.phi_matvec_general(Xs, P.omega, d, got), bd, m)
    say(f"[intercept c1] draw iters {info['iters']} rule {rule / 1e-10:.3f} x tol")
    assert info["status"] == pk.OK and rule <= 1e-10 * (1 + 1e-6)
    # converged solve against the oracle's CG
    sol, info = pk.solve_general(X, t64(P.omega), t64(d), t64(b), precond_inv=t64(m), tol=1e-12)
    ref = R.pcg_solve_general(Xs, P.omega, d, m, b, tol=1e-12)
    e = R.error_metrics(sol.cpu().numpy(), ref.beta, np.sqrt(m))
    say(f"[intercept c1] tol 1e-12: iters {info['iters']} (oracle {ref.iters}) {e}")
    assert info["status"] == pk.OK and e["rel_l2"] <= 1e-10
