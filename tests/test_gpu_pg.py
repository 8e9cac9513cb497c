"""GPU parity of the Polya-Gamma omega update (Supplement S1, step 3):
element-by-element against the oracle's sampler on the same counter-based
uniforms.  Both sides take every accept/reject decision in FP64, so equal
inputs give equal decisions except where a decision value lands within a
rounding error of its threshold (probability ~1e-15 per decision); omega
then agrees to the rounding of the arithmetic after the decisions."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1810_12437_amd as pk  # noqa: E402
import synth  # noqa: E402
from oracle import pg_ref as G  # noqa: E402
from oracle import ppcg_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_pg_sample_matches_oracle():
    """3000 tilts spanning 0, both signs, the two inverse-Gaussian branches
    (|c|/2 below and above 1/0.64), |c| up to 300 and two beyond the range
    where the series' leading term underflows (1e4, -3e3), over a ragged
    tail."""
    rng = np.random.default_rng(4)
    c = np.concatenate([[0.0, -0.0, 3.125, -3.125, 300.0, -300.0, 1e-300, 1e4, -3e3],
                        rng.standard_normal(1000) * 0.5, rng.standard_normal(1000) * 6.0,
                        rng.uniform(-300, 300, 991)])
    got = pk.pg_sample(torch.as_tensor(c, device=DEV), 123, 4, 9).cpu().numpy()
    ref = G.pg_draws(123, 4, 9, c)
    err = np.abs(got - ref) / ref
    say(f"[pg_sample] n {c.size} max rel err {err.max():.2e}")
    assert np.all(got > 0)
    assert np.all(err <= 1e-12)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_pg_update_matches_oracle(dt):
    """psi = X beta by the row pass, omega and z against the oracle's
    (FP64 1e-12; FP32 outputs are the FP64 values rounded, so 1e-7), on a
    design that spans several panels with a ragged tail."""
    P = synth.scaled_problem(5003, 700, seed=13, tau=5e-2)
    X = pk.Matrix.from_problem(P)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    rng = np.random.default_rng(2)
    beta = rng.standard_normal(P.p) * 0.3
    if dt == torch.float32:
        beta = np.float32(beta).astype(np.float64)
    y = (rng.random(P.n) < 0.3).astype(np.uint8)
    om, z = pk.pg_update(X, torch.as_tensor(beta, device=DEV).to(dt),
                         torch.as_tensor(y, device=DEV), 55, 1, 7)
    o_ref, z_ref, psi = G.pg_update(Xs, beta, y, 55, 1, 7)
    tol = 1e-12 if dt == torch.float64 else 1e-7
    eo = np.abs(om.double().cpu().numpy() - o_ref) / o_ref
    ez = np.abs(z.double().cpu().numpy() - z_ref) / np.abs(z_ref)
    say(f"[pg_update {dt}] psi range [{psi.min():.2f}, {psi.max():.2f}] "
        f"max rel err omega {eo.max():.2e} z {ez.max():.2e}")
    assert np.all(eo <= tol) and np.all(ez <= tol)


def test_pg_update_full_size_sampled():
    """n = 1e5, p = 2e4 (52.6 M non-zeros): omega and z on 400 sampled rows
    (the oracle draws them one by one from their own streams), and the mean
    of all omega against E[PG(1, psi)] = tanh(psi/2) / (2 psi) within 5
    standard errors."""
    P = synth.make_problem("c1")
    X = pk.Matrix.from_problem(P)
    Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
    rng = np.random.default_rng(8)
    beta = rng.standard_normal(P.p) * 0.01
    beta[:50] = rng.standard_normal(50)
    y = (rng.random(P.n) < 0.5).astype(np.uint8)
    om, z = pk.pg_update(X, torch.as_tensor(beta, device=DEV), torch.as_tensor(y, device=DEV),
                         12437, 0, 3)
    om, z = om.cpu().numpy(), z.cpu().numpy()
    idx = np.sort(rng.choice(P.n, 400, replace=False))
    o_ref, z_ref, psi = G.pg_update(Xs, beta, y, 12437, 0, 3, idx=idx)
    eo = np.abs(om[idx] - o_ref) / o_ref
    assert np.all(eo <= 1e-12) and np.allclose(z[idx], z_ref, rtol=1e-12, atol=0)
    a = np.abs(psi)
    small = a < 1e-3
    mean = np.where(small, 0.25 - a * a / 48, np.tanh(a / 2) / (2 * np.where(small, 1, a)))
    var = np.where(small, 1 / 24, (2 * np.tanh(a / 2) - a / np.cosh(a / 2) ** 2) /
                   (4 * np.where(small, 1, a) ** 3))
    zstat = (om.sum() - mean.sum()) / np.sqrt(var.sum())
    say(f"[pg_update full] max rel err {eo.max():.2e}; mean z-score {zstat:.2f}")
    assert abs(zstat) < 5
