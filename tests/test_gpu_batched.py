"""GPU parity of the batched form: many chains of uneven size (each with its
own design, or several on one design) solved with one launch per CG phase.

Each chain's batched result must equal the single-chain call's bitwise (the
same kernels, blocks and summation order), and the single-chain path is held
to the oracle by test_gpu_parity.py; the FP64 batch is also checked against
the oracle directly at a tight tolerance (1e-10 relative in beta).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1810_12437_amd as pk  # noqa: E402
import synth  # noqa: E402
from oracle import philox_ref as H  # noqa: E402
from oracle import ppcg_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def chains_for_test(scale=0.1, count=6):
    """Uneven chains of the batched workload's laws at reduced size, plus two
    extra chains on the first chain's design with their own vectors."""
    probs = synth.batched_problems(count=count, seed=77, scale=scale)
    base = probs[0]
    extra = synth.shared_x_chains(base, 2, seed=78)
    return probs, [(base, om, z, lam, tau) for om, z, lam, tau in extra]


def build(dtype):
    probs, extra = chains_for_test()
    mats = [pk.Matrix.from_problem(P) for P in probs]
    dt = torch.float64 if dtype == pk.F64 else torch.float32
    rows = []  # (matrix, omega, z, lambda, tau)
    for X, P in zip(mats, probs):
        rows.append((X, torch.as_tensor(P.omega, device=DEV).to(dt),
                     torch.as_tensor(P.z, device=DEV).to(dt),
                     torch.as_tensor(P.lam, device=DEV).to(dt), P.tau))
    for P, om, z, lam, tau in extra:
        rows.append((mats[0], torch.as_tensor(om, device=DEV).to(dt),
                     torch.as_tensor(z, device=DEV).to(dt),
                     torch.as_tensor(lam, device=DEV).to(dt), tau))
    return probs, extra, rows


@pytest.mark.parametrize("dtype", [pk.F64, pk.F32])
def test_batched_draw_equals_single_draws(dtype):
    probs, extra, rows = build(dtype)
    say("batched draw dtype", dtype, "chains", [(r[0].n, r[0].p) for r in rows])
    B = pk.Batch([r[0] for r in rows], dtype=dtype)
    seeds = [12437 + c for c in range(len(rows))]
    chains = list(range(len(rows)))
    draws = [3 + c for c in range(len(rows))]
    betas, infos = B.draw([r[1] for r in rows], [r[2] for r in rows], [r[3] for r in rows],
                          [r[4] for r in rows], seeds, chains, draws, tol=1e-8)
    iters = [i["iters"] for i in infos]
    say("iterations per chain", iters)
    assert len(set(iters)) > 1  # chains stop at different iterations
    for c, (X, om, z, lam, tau) in enumerate(rows):
        ref, info = pk.draw(X, om, z, lam, tau, seeds[c], chains[c], draws[c], tol=1e-8)
        same = bool(torch.equal(betas[c], ref))
        say("chain", c, "bitwise equal", same, "iters", infos[c]["iters"], info["iters"])
        assert same
        assert infos[c]["iters"] == info["iters"]
        assert infos[c]["refine_iters"] == info["refine_iters"]
        assert infos[c]["status"] == pk.OK
        assert infos[c]["resid_true"] <= 1.0


def test_batched_solve_matches_oracle():
    """FP64 batched solves at a tight tolerance against the oracle's Cholesky
    solution of each chain (1e-10 relative)."""
    probs, extra, rows = build(pk.F64)
    B = pk.Batch([r[0] for r in rows], dtype=pk.F64)
    rng = np.random.default_rng(5)
    bs_np = [rng.standard_normal(r[0].p) for r in rows]
    betas, infos = B.solve([r[1] for r in rows], [r[3] for r in rows], [r[4] for r in rows],
                           [torch.as_tensor(b, device=DEV) for b in bs_np], tol=1e-13)
    allp = probs + [e[0] for e in extra]
    for c, (X, om, z, lam, tau) in enumerate(rows):
        P = allp[c]
        Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
        Phi = R.phi_dense(Xs, om.cpu().numpy(), lam.cpu().numpy(), tau)
        exact = R.solve_chol(Phi, bs_np[c])
        got = betas[c].cpu().numpy()
        e = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
        say("chain", c, "p", X.p, "iters", infos[c]["iters"], "rel err", e)
        assert e <= 1e-10
        assert infos[c]["resid_true"] <= 1.0


def test_batched_draw_matches_oracle_draw():
    """One FP64 chain of the batch against the oracle's own draw (same eta,
    delta stream, Prop 2.1's b, CG at a tight tolerance)."""
    probs, extra, rows = build(pk.F64)
    B = pk.Batch([r[0] for r in rows], dtype=pk.F64)
    n = len(rows)
    betas, infos = B.draw([r[1] for r in rows], [r[2] for r in rows], [r[3] for r in rows],
                          [r[4] for r in rows], [9] * n, list(range(n)), [0] * n, tol=1e-13)
    for c in (0, n - 1):
        P = (probs + [e[0] for e in extra])[c]
        X, om, z, lam, tau = rows[c]
        Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
        eta, delta = H.eta_delta(9, c, 0, P.n, P.p)
        b = R.rhs_b(Xs, om.cpu().numpy(), z.cpu().numpy(), lam.cpu().numpy(), tau, eta, delta)
        Phi = R.phi_dense(Xs, om.cpu().numpy(), lam.cpu().numpy(), tau)
        exact = R.solve_chol(Phi, b)
        e = float(np.linalg.norm(betas[c].cpu().numpy() - exact) / np.linalg.norm(exact))
        say("chain", c, "rel err vs oracle draw", e)
        assert e <= 1e-10


def test_batched_per_chain_status_and_repeat():
    """A chain capped below its needs reports ENOTCONV without disturbing the
    others; a second call on the same batch with other draw indices is again
    equal to the single-chain draws."""
    probs, extra, rows = build(pk.F64)
    B = pk.Batch([r[0] for r in rows], dtype=pk.F64)
    n = len(rows)
    args = ([r[1] for r in rows], [r[2] for r in rows], [r[3] for r in rows],
            [r[4] for r in rows], [1] * n, list(range(n)))
    betas, infos = B.draw(*args, [5] * n, tol=1e-8, max_iter=3)
    assert all(i["status"] == pk.ENOTCONV for i in infos if i["iters"] >= 3)
    betas2, infos2 = B.draw(*args, [6] * n, tol=1e-8)
    for c, (X, om, z, lam, tau) in enumerate(rows):
        ref, info = pk.draw(X, om, z, lam, tau, 1, c, 6, tol=1e-8)
        assert torch.equal(betas2[c], ref)
        assert infos2[c]["status"] == pk.OK


# ---- shared design: K interleaved vectors per X pass ----

def shared_setup(nchains, dtype, n=6000, p=3000, seed=31):
    base = synth.scaled_problem(n, p, seed=seed, tau=2e-3, name="shared")
    chains = synth.shared_x_chains(base, nchains, seed=seed + 1)
    dt = torch.float64 if dtype == pk.F64 else torch.float32
    B = pk.Batch.shared(base.n, base.p, base.row_ptr, base.col_idx, nchains, dtype=dtype)
    vecs = [(torch.as_tensor(om, device=DEV).to(dt), torch.as_tensor(z, device=DEV).to(dt),
             torch.as_tensor(lam, device=DEV).to(dt), tau) for om, z, lam, tau in chains]
    return base, chains, B, vecs


@pytest.mark.parametrize("nchains", [1, 2, 3, 8])
def test_shared_solve_matches_cholesky(nchains):
    """Shared-design solves against Cholesky at a tight tolerance: one and
    two chains run the K = 2 passes (one of them with an empty slot), three
    and eight the groups of four."""
    base, chains, B, vecs = shared_setup(nchains, pk.F64)
    say("shared solve", nchains, "chains, n", base.n, "p", base.p)
    rng = np.random.default_rng(nchains)
    bs = [rng.standard_normal(base.p) for _ in range(nchains)]
    betas, infos = B.solve([v[0] for v in vecs], [v[2] for v in vecs], [v[3] for v in vecs],
                           [torch.as_tensor(b, device=DEV) for b in bs], tol=1e-13)
    Xs = R.csr_matrix(base.n, base.p, base.row_ptr, base.col_idx)
    for c, (om, z, lam, tau) in enumerate(chains):
        exact = R.solve_chol(R.phi_dense(Xs, om, lam, tau), bs[c])
        e = float(np.linalg.norm(betas[c].cpu().numpy() - exact) / np.linalg.norm(exact))
        say("chain", c, "iters", infos[c]["iters"], "rel err", e)
        assert e <= 1e-10
        assert infos[c]["status"] == pk.OK and infos[c]["resid_true"] <= 1.0


def test_shared_draw_matches_single_chain_draws():
    """Shared-design draws against the single-chain path on the same
    arguments: both converge to the same beta (1e-10 at a tight tolerance),
    with iteration counts within a plateau's reach."""
    base, chains, B, vecs = shared_setup(5, pk.F64)
    X = pk.Matrix.from_problem(base)
    n = len(vecs)
    betas, infos = B.draw([v[0] for v in vecs], [v[1] for v in vecs], [v[2] for v in vecs],
                          [v[3] for v in vecs], [44] * n, list(range(n)), [2] * n, tol=1e-13)
    for c, (om, z, lam, tau) in enumerate(vecs):
        ref, info = pk.draw(X, om, z, lam, tau, 44, c, 2, tol=1e-13)
        e = float(torch.linalg.norm(betas[c] - ref) / torch.linalg.norm(ref))
        say("chain", c, "iters", infos[c]["iters"], info["iters"], "rel diff", e)
        assert e <= 1e-10
        assert abs(infos[c]["iters"] - info["iters"]) <= max(3, 0.05 * info["iters"])


def test_shared_slot_reassignment_keeps_draws():
    """FP64 batches of five to eight chains on one design run as two groups
    of four; after a call the chains are dealt to the groups by falling
    iteration count.  The slot does not change a chain's arithmetic: a draw
    after the reassignment equals, bit for bit and iteration for iteration,
    the same draw from a fresh batch with the chains in their first slots."""
    base, chains, B0, vecs = shared_setup(8, pk.F64)
    n = len(vecs)
    args = lambda d: ([44] * n, list(range(n)), [d] * n)  # noqa: E731
    cols = lambda v: [[x[i] for x in v] for i in range(4)]  # noqa: E731
    _, inf0 = B0.draw(*cols(vecs), *args(0), tol=1e-8)
    its = [i["iters"] + i["refine_iters"] for i in inf0]
    say("[slots] iterations by chain", its)
    # chains handed over by rising count: the reassignment reverses them
    order = sorted(range(n), key=lambda c: (its[c], c))
    v2 = [vecs[c] for c in order]
    assert sorted(its) != sorted(its, reverse=True)
    B1 = pk.Batch.shared(base.n, base.p, base.row_ptr, base.col_idx, n, dtype=pk.F64)
    B1.draw(*cols(v2), *args(0), tol=1e-8)
    b1, i1 = B1.draw(*cols(v2), *args(1), tol=1e-8)
    B2 = pk.Batch.shared(base.n, base.p, base.row_ptr, base.col_idx, n, dtype=pk.F64)
    b2, i2 = B2.draw(*cols(v2), *args(1), tol=1e-8)
    for c in range(n):
        assert torch.equal(b1[c], b2[c]), c
        assert (i1[c]["iters"], i1[c]["refine_iters"]) == (i2[c]["iters"], i2[c]["refine_iters"])
        assert i1[c]["status"] == pk.OK


@pytest.mark.parametrize("nchains", [2, 4])
def test_shared_f32_matches_f64_oracle(nchains):
    """FP32 shared-design draws (with the refinement restart) against the FP64
    oracle's Cholesky solution to 1e-5: two chains run the K = 2 passes, four
    one group of four."""
    base, chains, B, vecs = shared_setup(nchains, pk.F32)
    n = len(vecs)
    betas, infos = B.draw([v[0] for v in vecs], [v[1] for v in vecs], [v[2] for v in vecs],
                          [v[3] for v in vecs], [5] * n, list(range(n)), [0] * n, tol=1e-12)
    Xs = R.csr_matrix(base.n, base.p, base.row_ptr, base.col_idx)
    for c in range(n):
        om = vecs[c][0].double().cpu().numpy()
        z = vecs[c][1].double().cpu().numpy()
        lam = vecs[c][2].double().cpu().numpy()
        tau = vecs[c][3]
        eta, delta = H.eta_delta(5, c, 0, base.n, base.p)
        b = R.rhs_b(Xs, om, z, lam, tau, eta, delta)
        exact = R.solve_chol(R.phi_dense(Xs, om, lam, tau), b)
        e = float(np.linalg.norm(betas[c].double().cpu().numpy() - exact) / np.linalg.norm(exact))
        say("chain", c, "iters", infos[c]["iters"], "+", infos[c]["refine_iters"], "rel err", e)
        assert e <= 1e-5


@pytest.mark.parametrize("form", ["uneven", "shared"])
@pytest.mark.parametrize("dtype", [pk.F64, pk.F32])
def test_graph_replays_equal_direct_launches(form, dtype):
    """Each check batch of the batched loop is a replayed HIP graph (recaptured
    when chains finish).  Draws alternate between graph replay and direct
    launches, with the host synchronising between calls, over several draws
    (so each graph is replayed many times, also after other work): every
    replayed result equals the direct one bitwise, with the same iteration
    counts."""
    if form == "uneven":
        probs, extra, rows = build(dtype)
        B = pk.Batch([r[0] for r in rows], dtype=dtype)
        vec = lambda i: [r[i] for r in rows]  # noqa: E731
        om, z, lam, tau = vec(1), vec(2), vec(3), vec(4)
    else:
        base, chains, B, vecs = shared_setup(5, dtype)
        om, z, lam, tau = ([v[i] for v in vecs] for i in range(4))
    n = len(om)
    for d in range(3):
        args = ([SEED_G + c for c in range(n)], list(range(n)), [d] * n)
        bg, ig = B.draw(om, z, lam, tau, *args, tol=1e-8)
        torch.cuda.synchronize()
        be, ie = B.draw(om, z, lam, tau, *args, tol=1e-8, no_graph=1)
        torch.cuda.synchronize()
        its = [i["iters"] + i["refine_iters"] for i in ig]
        say(f"[graph {form} {dtype}] draw {d} iterations {its}")
        for c in range(n):
            assert torch.equal(bg[c], be[c])
            assert (ig[c]["iters"], ig[c]["refine_iters"]) == (ie[c]["iters"], ie[c]["refine_iters"])
            assert ig[c]["status"] == pk.OK


SEED_G = 9090
