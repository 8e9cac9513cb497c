"""Writes c1_draw0_reference.npz: the oracle's beta for one full-size draw.

Workload: synth.make_problem("c1") (n = 1e5, p = 2e4, column-law binary X,
tau = 1e-3), eta and delta from the counter-based generator with seed 12437,
chain 0, draw 0 (Prop 2.1), solved by the oracle's prior-preconditioned CG to
relative preconditioned residual 1e-12.  Also stored: the rigorous bound
||(beta_ref - beta)/c|| <= ||c (b - Phi beta_ref)|| (Supplement S4.2 with
Theorem 2.4), so users of the file know how exact it is.  Calls only synth
and oracle/.  Run: python tests/golden/make_c1_reference.py  (about a minute).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import philox_ref, ppcg_ref  # noqa: E402

SEED, CHAIN, DRAW, TOL = 12437, 0, 0, 1e-12


def main():
    P = synth.make_problem("c1")
    X = ppcg_ref.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    out = {}
    for name, cast in (("f64", lambda a: a), ("f32", lambda a: np.float32(a).astype(np.float64))):
        om, z, lam = cast(P.omega), cast(P.z), cast(P.lam)
        eta, delta = philox_ref.eta_delta(SEED, CHAIN, DRAW, P.n, P.p)
        b = ppcg_ref.rhs_b(X, om, z, lam, P.tau, eta, delta)
        res = ppcg_ref.pcg_solve(X, om, lam, P.tau, b, tol=TOL)
        bound = ppcg_ref.posterior_error_bound(X, om, lam, P.tau, b, res.beta)
        out[f"beta_{name}"] = res.beta
        out[f"iters_{name}"] = res.iters
        out[f"scaled_err_bound_{name}"] = bound
        out[f"scaled_norm_{name}"] = float(np.linalg.norm(res.beta / (P.tau * lam)))
        print(name, "iters", res.iters, "bound", bound, flush=True)
    np.savez(os.path.join(HERE, "c1_draw0_reference.npz"), seed=SEED, chain=CHAIN, draw=DRAW,
             tol=TOL, nnz=P.nnz, **out)


if __name__ == "__main__":
    main()
