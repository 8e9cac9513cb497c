#!/usr/bin/env python3
"""Throughput of the prior-preconditioned CG sampler on one MI355X.

A step is one Gibbs beta-draw (Prop 2.1): counter-based eta and delta, the
right-hand side b, prior-preconditioned CG to the stopping rule and the FP64
true residual of the result.  The workload is n = 1e5 observations, p = 2e4
binary features with log-uniform column densities in [1e-4, 0.2], tau = 1e-3
and 50 signal columns, relative preconditioned residual 1e-6.

Prints one JSON line: draws/s of the headline form (FP64 vectors and
scalars, the faster form at the 1e-5 accuracy bar), the FP32-vector form with
its FP64 refinement beside it, the HBM roofline of the dominant kernel (the X
pass, timed with HIP events on the solver's stream during the timed draws),
the general-prior forms on the same draws (prior preconditioner cold and
warm-started, Jacobi, the adaptive switch), the adjoint form against plain
solves of the same systems, Gibbs steps with the device
Polya-Gamma omega update, summaries of the other workloads (8 chains on the
same design, 32 uneven chains, the 200-step sequence at n = 5e5, p = 5e4;
``--no-forms`` skips them), and the CPU baselines timed on this host: the
oracle's CG draw (one thread) at n = 1e5, p = 2e4 and at n = 2000, p = 500,
and the direct Cholesky draw the paper compares with (all BLAS threads; at
n = 1e5 from a bounded sample), with the host's CPU model and core count.

``--copy-calibration`` instead times a plain 512 MiB device copy: its
FETCH_SIZE / WRITE_SIZE counters calibrate the pass kernel's counters.
``--form shared`` measures 8 chains on the n = 1e5, p = 2e4 design (each
with its own omega, z, lambda, tau and stream), every X pass serving all 8.
``--form batched`` instead measures the batched form: 32 independent chains
with n log-uniform in [2e4, 2e5], p in [5e3, 4e4], tau in [1e-4, 1e-2] (the
same column law), one batched draw of all chains per step, against the same
chains drawn one at a time.  ``--form large`` runs the 200-step Gibbs-style
sequence on the n = 5e5, p = 5e4 design (FP32 with refinement, omega and
lambda redrawn per step, adaptive preconditioner) and times its passes where
the index streams exceed the MALL.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "Gibbs beta-draws/sec + SpMV-CG HBM GB/s (% peak), n=1e5 p=2e4, rel err<=1e-5"
SEED = 12437
COPY_BYTES = 512 << 20
FORM_STEPS = 5  # timed steps of the shared-design and batched summaries in the default line

# HBM traffic of one X-pass launch (k_panel<double, 1> row pass and
# k_panel<double, 2> column pass, averaged) on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, mean
# over the launches of the profiled draws) scaled by the same counters of a
# plain 512 MiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for
# the kernel sources it was measured on (SHA-256 over the files below); any
# change to them reports null until the counters are taken again.
PASS_SOURCES = ("paper_1810_12437_amd/csrc/ppcg_kernels.hip",
                "paper_1810_12437_amd/csrc/ppcg_layout.h",
                "paper_1810_12437_amd/csrc/ppcg_panels.h")
TRAFFIC = {
    "sources_sha256": "ea67f121b8d91bc57e260fe28354456bb61157b265666b9f720fc41bd0aea102",
    # mean of the row and column variants: (FETCH_SIZE KiB x 2.0 + WRITE_SIZE KiB x 1.0) x 1024
    "bytes_per_launch": 75581235,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 200 for --form large, the sequence length)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32-vector form")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the accuracy check of the timed configuration")
    ap.add_argument("--cpu-draws", type=int, default=2,
                    help="complete oracle draws in the bounded CPU sample")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the prior / warm-start / Jacobi / switch comparison")
    ap.add_argument("--no-gibbs", action="store_true",
                    help="skip the Gibbs steps with the device Polya-Gamma update")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the shared-design, batched and large workloads in the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--form", choices=("single", "batched", "shared", "large"), default="single",
                    help="single: the n=1e5 p=2e4 draw (default); batched: 32 uneven chains; "
                         "shared: 8 chains on the n=1e5 p=2e4 design; large: the 200-step "
                         "sequence on the n=5e5 p=5e4 design")
    return ap.parse_args()


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in PASS_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def int32_pass_bytes(P, sv):
    """Bytes one launch of each X pass would move in a plain int32 CSR / CSC
    format (index stream, offsets, gathered vector once, scale, output); the
    int32-equivalent rate of the compact panel format is reported beside its
    own."""
    nnz, n, p = P.nnz, P.n, P.p
    rows = int(np.count_nonzero(np.diff(P.row_ptr)))
    cols = int(np.count_nonzero(np.bincount(P.col_idx, minlength=p)))
    csr = 4 * nnz + 8 * (rows + 1) + sv * p + sv * n + sv * rows
    csc = 4 * nnz + 8 * (cols + 1) + sv * n + sv * cols
    return csr, csc


def vec_bytes(p, sv):
    """Bytes of the three p-vector phases of one CG iteration: <s, q + d s>;
    beta += alpha s, r -= alpha q, rho; s = M^-1 r + ratio s."""
    dot = p * (sv + sv + 8)
    upd = p * (sv + sv + 8 + 8 + 8 + 8 + 8 + 8)
    direc = p * (8 + 8 + sv + sv)
    return dot + upd + direc


def run_form(pk, torch, X, P, dtype, steps, warmup, tol):
    dt = torch.float32 if dtype == pk.F32 else torch.float64
    om = torch.as_tensor(P.omega, device="cuda").to(dt)
    z = torch.as_tensor(P.z, device="cuda").to(dt)
    lam = torch.as_tensor(P.lam, device="cuda").to(dt)
    for w in range(warmup):
        pk.draw(X, om, z, lam, P.tau, SEED, 0, 1000 + w, tol=tol)
    torch.cuda.synchronize()
    X.profile(True)
    infos = []
    t0 = time.perf_counter()
    for k in range(steps):
        _, info = pk.draw(X, om, z, lam, P.tau, SEED, 0, k, tol=tol)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = X.stats()
    X.profile(False)
    iters = np.array([i["iters"] + i["refine_iters"] for i in infos], dtype=np.float64)
    return {"elapsed": t1 - t0, "infos": infos, "stats": stats, "iters": iters}


def pass_time_ms(st):
    return (st["csr_ms"] + st["csc_ms"]) / max(st["csr_launches"] + st["csc_launches"], 1)


def check_accuracy(pk, torch, X, P, tol):
    """Relative error of draw (SEED, 0, 0) of each form against the oracle's
    solution of the same draw (stored by the oracle-only script
    tests/golden/make_c1_reference.py)."""
    gold = os.path.join(ROOT, "tests", "golden", "c1_draw0_reference.npz")
    if not os.path.exists(gold):
        return {}
    g = np.load(gold)
    out = {}
    for name, dt, key in (("f64", torch.float64, "beta_f64"), ("f32", torch.float32, "beta_f32")):
        om = torch.as_tensor(P.omega, device="cuda").to(dt)
        zz = torch.as_tensor(P.z, device="cuda").to(dt)
        la = torch.as_tensor(P.lam, device="cuda").to(dt)
        b0, _ = pk.draw(X, om, zz, la, P.tau, int(g["seed"]), int(g["chain"]), int(g["draw"]),
                        tol=tol)
        ref = g[key]
        out[name] = float(np.linalg.norm(b0.double().cpu().numpy() - ref) / np.linalg.norm(ref))
    return out


def host_info():
    """The host the CPU baselines ran on: CPU model, logical CPUs, the CPUs
    this process may use, and the BLAS threads."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")}
                for i in threadpool_info()]
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable, "blas": blas}


def cpu_baseline(P, tol, draws):
    """The oracle as it stands, on this host, one thread: `draws` complete
    draws of the same workload (Prop 2.1's b, then PCG to the same stopping
    rule), timed end to end."""
    from threadpoolctl import threadpool_limits

    from oracle import philox_ref, ppcg_ref

    iters = []
    with threadpool_limits(1):
        X = ppcg_ref.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
        t0 = time.perf_counter()
        for k in range(draws):
            eta, delta = philox_ref.eta_delta(SEED, 0, k, P.n, P.p)
            b = ppcg_ref.rhs_b(X, P.omega, P.z, P.lam, P.tau, eta, delta)
            iters.append(ppcg_ref.pcg_solve(X, P.omega, P.lam, P.tau, b, tol=tol).iters)
        el = time.perf_counter() - t0
    return {
        "value": draws / el, "unit": "draws/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle (NumPy/SciPy FP64, 1 thread) at n=1e5 p=2e4: {draws} complete "
                   f"draws (Prop 2.1 b, PCG to relative preconditioned residual {tol:g}; "
                   f"{', '.join(map(str, iters))} iterations) in {el:.1f} s"),
    }


def cpu_small_and_direct(P1, tol):
    """The CPU baselines beside the oracle's CG draw at n = 1e5, p = 2e4:

    * the oracle's CG draw at n = 2000, p = 500 (one thread): median of 5
      after one warm-up;
    * the direct Cholesky draw (the standard method the paper compares
      with, Section 2.1 and Supplement S7.3: Phi = X^T Omega X by SciPy's
      sparse product, one thread, then LAPACK's Cholesky, the solve for the
      mean and the triangular solve for the noise with every BLAS thread of
      this process): at n = 2000, p = 500 in full (median of 5 after one
      warm-up); at n = 1e5, p = 2e4 from a bounded sample: the sparse
      product over the first 5,000 rows, scaled by n / 5,000 (its work is a
      sum over rows), plus the full-size dense factorisation and solves of
      that sample's Phi with the prior added (the same size and cost as the
      full one)."""
    import synth
    from oracle import philox_ref, ppcg_ref

    from threadpoolctl import threadpool_limits

    out = {}
    P0 = synth.make_problem("c0")
    X0 = ppcg_ref.csr_matrix(P0.n, P0.p, P0.row_ptr, P0.col_idx)
    d0 = ppcg_ref.prior_precision(P0.lam, P0.tau)

    def direct(X, P, d, k):
        Phi = ppcg_ref.phi_dense_general(X, P.omega, d)
        xi = np.random.default_rng(k).standard_normal(P.p)
        return ppcg_ref.draw_chol(Phi, ppcg_ref.rhs_mean(X, P.omega, P.z), xi)

    def oracle_cg(k):
        eta, delta = philox_ref.eta_delta(SEED, 0, k, P0.n, P0.p)
        b = ppcg_ref.rhs_b(X0, P0.omega, P0.z, P0.lam, P0.tau, eta, delta)
        return ppcg_ref.pcg_solve(X0, P0.omega, P0.lam, P0.tau, b, tol=1e-10).iters

    def median_of_5(fn):
        fn(99)
        ts = []
        for k in range(5):
            t0 = time.perf_counter()
            fn(k)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    with threadpool_limits(1):
        t = median_of_5(oracle_cg)
    out["oracle_cg_c0"] = {"draws_per_s": 1.0 / t, "threads": 1,
                           "sample": "n=2000 p=500, tol 1e-10, median of 5 after 1 warm-up"}
    t = median_of_5(lambda k: direct(X0, P0, d0, k))
    out["direct_cholesky_c0"] = {"draws_per_s": 1.0 / t,
                                 "sample": "n=2000 p=500, median of 5 after 1 warm-up"}
    X1 = ppcg_ref.csr_matrix(P1.n, P1.p, P1.row_ptr, P1.col_idx)
    rows = 5000
    Xs = X1[:rows]
    t0 = time.perf_counter()
    XO = Xs.multiply(P1.omega[:rows, None]).tocsr()
    G = (Xs.T @ XO).toarray()
    t_prod = time.perf_counter() - t0
    del XO
    G[np.diag_indices_from(G)] += ppcg_ref.prior_precision(P1.lam, P1.tau)
    xi = np.random.default_rng(5).standard_normal(P1.p)
    t0 = time.perf_counter()
    ppcg_ref.draw_chol(G, ppcg_ref.rhs_mean(X1, P1.omega, P1.z), xi)
    t_chol = time.perf_counter() - t0
    del G
    t_draw = t_prod * (P1.n / rows) + t_chol
    out["direct_cholesky_c1"] = {
        "draws_per_s": 1.0 / t_draw, "s_per_draw": t_draw,
        "sparse_product_s": t_prod * (P1.n / rows), "factor_and_solves_s": t_chol,
        "sample": (f"n=1e5 p=2e4: X^T Omega X over the first {rows} rows in {t_prod:.1f} s "
                   f"(one thread), scaled by n/{rows}; Cholesky, mean and noise solves of a "
                   f"{P1.p} x {P1.p} Phi in {t_chol:.1f} s on the BLAS threads"),
    }
    return out


def precond_forms(pk, torch, P, X, steps, warmup, tol):
    """The general-prior entry points on the same workload and draws (FP64):
    the prior preconditioner through ppcg_draw_general (cold, and warm-started
    from the rescaled running mean of the draws before it), the Jacobi
    preconditioner (its M^-1 recomputed every draw), and the adaptive switch
    (a trial of both on its first draw).  Each with the relative error of
    draw (SEED, 0, 0) against the oracle's stored solution."""
    gold = os.path.join(ROOT, "tests", "golden", "c1_draw0_reference.npz")
    ref = np.load(gold)["beta_f64"] if os.path.exists(gold) else None
    om = torch.as_tensor(P.omega, device="cuda")
    zz = torch.as_tensor(P.z, device="cuda")
    la = torch.as_tensor(P.lam, device="cuda")
    d, m = pk.unshrunk_setup(la, P.tau)
    out = {}

    def err(beta):
        if ref is None:
            return None
        return float(np.linalg.norm(beta.cpu().numpy() - ref) / np.linalg.norm(ref))

    def timed(name, one):
        for w in range(warmup):
            one(1000 + w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = [one(k) for k in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"draws_per_s": steps / el, "cg_iters_mean": float(np.mean(its))}

    def prior(k):
        _, i = pk.draw_general(X, om, zz, d, SEED, 0, k, precond_inv=m, tol=tol)
        return i["iters"] + i["refine_iters"]

    timed("prior", prior)
    out["prior"]["rel_err_vs_oracle"] = err(pk.draw_general(X, om, zz, d, SEED, 0, 0,
                                                            precond_inv=m, tol=tol)[0])
    ws = pk.WarmStart(P.p)

    def warm(k):
        b0 = ws.vector(la, P.tau)
        beta, i = pk.draw_general(X, om, zz, d, SEED, 0, k, precond_inv=m, beta0=b0, tol=tol)
        ws.add(beta, la, P.tau)
        return i["iters"] + i["refine_iters"]

    timed("prior_warm_start", warm)

    def jacobi(k):
        mj = pk.jacobi_precond(X, om, d)
        _, i = pk.draw_general(X, om, zz, d, SEED, 0, k, precond_inv=mj, tol=tol)
        return i["iters"] + i["refine_iters"]

    timed("jacobi", jacobi)
    out["jacobi"]["rel_err_vs_oracle"] = err(pk.draw_general(
        X, om, zz, d, SEED, 0, 0, precond_inv=pk.jacobi_precond(X, om, d), tol=tol)[0])
    sw = pk.Switch(P.p, period=100)

    def switch(k):
        _, i = sw.draw(X, om, zz, d, SEED, 0, k, precond_inv=m, tol=tol)
        return i["iters"] + i["refine_iters"]

    timed("switch_period_100", switch)
    out["switch_period_100"].update(sw.state())
    sw.close()
    return out


def gibbs_forms(pk, torch, P, X, steps, warmup, tol):
    """Gibbs steps on the same design: y ~ Bernoulli(logistic(X beta_true))
    with the 50 signal columns at 1 (seeded), then per step omega ~ PG(1,
    X beta) and z = (y - 1/2)/omega on the device (Supplement S1, step 3)
    followed by the beta draw (step 4) with lambda and tau held at the
    workload's values (their updates depend on the shrinkage prior).  Timed
    from beta = 0 after `warmup` steps; reported per form: steps/s, mean CG
    iterations, and the PG update alone (its share of a step)."""
    rng = np.random.default_rng(SEED + 1)
    beta_true = np.zeros(P.p)
    beta_true[:50] = 1.0
    import scipy.sparse as sp
    Xs = sp.csr_matrix((np.ones(P.nnz), P.col_idx, P.row_ptr), shape=(P.n, P.p))
    psi = Xs @ beta_true
    y = torch.as_tensor((rng.random(P.n) < 1.0 / (1.0 + np.exp(-psi))).astype(np.uint8),
                        device="cuda")
    la = torch.as_tensor(P.lam, device="cuda")
    d, m = pk.unshrunk_setup(la, P.tau)
    out = {"y_mean": float(y.float().mean().item())}

    def run(name, draw):
        beta = torch.zeros(P.p, dtype=torch.float64, device="cuda")
        for w in range(warmup):
            om, z = pk.pg_update(X, beta, y, SEED, 0, 10_000 + w)
            beta, _ = draw(om, z, 10_000 + w)
        torch.cuda.synchronize()
        its = []
        t0 = time.perf_counter()
        for k in range(steps):
            om, z = pk.pg_update(X, beta, y, SEED, 0, k)
            beta, info = draw(om, z, k)
            its.append(info["iters"] + info["refine_iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"steps_per_s": steps / el, "cg_iters_mean": float(np.mean(its))}
        return beta

    beta = run("prior", lambda om, z, k: pk.draw(X, om, z, la, P.tau, SEED, 0, k, tol=tol))
    sw = pk.Switch(P.p, period=100)
    run("switch_period_100",
        lambda om, z, k: sw.draw(X, om, z, d, SEED, 0, k, precond_inv=m, tol=tol))
    out["switch_period_100"].update(sw.state())
    sw.close()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for k in range(steps):
        pk.pg_update(X, beta, y, SEED, 0, k)
    ev[1].record()
    ev[1].synchronize()
    out["pg_update_ms"] = ev[0].elapsed_time(ev[1]) / steps
    return out


def adjoint_forms(pk, torch, P, X, steps, warmup, tol):
    """The adjoint form on the same workload (FP64): a = Phi^-1 g for the loss
    sum_j w_j beta_j^2 (g = 2 w beta, w ~ U(0, 1)) and the gradients with
    respect to b, log lambda and log tau, against plain solves of the same
    systems; each timed over `steps` right-hand sides after `warmup`."""
    rng = np.random.default_rng(SEED + 2)
    om = torch.as_tensor(P.omega, device="cuda")
    la = torch.as_tensor(P.lam, device="cuda")
    w = torch.as_tensor(rng.uniform(0.0, 1.0, P.p), device="cuda")
    bs = [torch.as_tensor(rng.standard_normal(P.p), device="cuda") for _ in range(warmup + steps)]

    def timed(one):
        for k in range(warmup):
            one(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = [one(k) for k in range(warmup, warmup + steps)]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, its

    betas = {}

    def forward(k):
        betas[k], info = pk.solve(X, om, la, P.tau, bs[k], tol=tol)
        return info["iters"]

    def backward(k):
        _, _, _, info = pk.solve_backward(X, om, la, P.tau, betas[k], 2.0 * w * betas[k], tol=tol)
        return info["iters"]

    el_f, its_f = timed(forward)
    el_b, its_b = timed(backward)
    return {"backward_per_s": steps / el_b, "backward_cg_iters_mean": float(np.mean(its_b)),
            "solve_per_s": steps / el_f, "solve_cg_iters_mean": float(np.mean(its_f)),
            "backward_vs_solve": el_f / el_b}


def copy_rate():
    """Best of 5 timed 512 MiB device-to-device copies: (ms, GB/s read + written)."""
    import torch

    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ms = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    best = min(ms)
    del src, dst
    return best, 2 * COPY_BYTES / (best * 1e-3) / 1e9


def copy_calibration():
    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    best, gbps = copy_rate()
    print(json.dumps({"copy_calibration": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES,
                                           "best_ms": best, "gbps": gbps}}), flush=True)


def batched_summary(pk, torch, steps, warmup, tol, no_f32=False):
    """32 independent chains of uneven size (n log-uniform [2e4, 2e5], p in
    [5e3, 4e4], tau in [1e-4, 1e-2], the column law), one batched draw of all
    chains per step, against the same chains drawn one at a time."""
    import gc
    from concurrent.futures import ThreadPoolExecutor

    import synth

    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"[bench] generating 32 chains ({workers} processes) ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    probs = synth.batched_problems(count=32, workers=workers)
    t_gen = time.perf_counter() - t0
    nnz = sum(P.nnz for P in probs)
    print(f"[bench] total nnz {nnz} in {t_gen:.1f} s; building handles",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=4) as ex:
        mats = list(ex.map(pk.Matrix.from_problem, probs))
    t_build = time.perf_counter() - t0
    C = len(probs)
    forms = {}
    for name, dtype, dt in (("f64", pk.F64, torch.float64), ("f32", pk.F32, torch.float32)):
        if name == "f32" and no_f32:
            continue
        B = pk.Batch(mats, dtype=dtype)
        om = [torch.as_tensor(P.omega, device="cuda").to(dt) for P in probs]
        zz = [torch.as_tensor(P.z, device="cuda").to(dt) for P in probs]
        la = [torch.as_tensor(P.lam, device="cuda").to(dt) for P in probs]
        ta = [P.tau for P in probs]
        seeds = [SEED] * C
        chains = list(range(C))
        for w in range(warmup):
            B.draw(om, zz, la, ta, seeds, chains, [1000 + w] * C, tol=tol)
        torch.cuda.synchronize()
        print(f"[bench] timing batched {name} ({steps} steps)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        iters = []
        for k in range(steps):
            _, infos = B.draw(om, zz, la, ta, seeds, chains, [k] * C, tol=tol)
            iters.append([i["iters"] + i["refine_iters"] for i in infos])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        it = np.array(iters, dtype=np.float64)
        f = {"chain_draws_per_s": C * steps / el, "ms_per_step": 1e3 * el / steps,
             "cg_iters_mean": float(it.mean()), "cg_iters_max": float(it.max()),
             "cg_iters_min": float(it.min())}
        # the same chains one at a time (single-chain path)
        t0 = time.perf_counter()
        for c in range(C):
            pk.draw(mats[c], om[c], zz[c], la[c], ta[c], SEED, c, 0, tol=tol)
        torch.cuda.synchronize()
        f["single_chain_path_chain_draws_per_s"] = C / (time.perf_counter() - t0)
        f["speedup_vs_single_chain_path"] = (f["chain_draws_per_s"] /
                                             f["single_chain_path_chain_draws_per_s"])
        forms[name] = f
        B.close()
    for m in mats:
        m.close()
    del mats, probs
    gc.collect()
    return {"chains": C, "nnz_total": int(nnz), "steps": steps, "generate_s": t_gen,
            "handle_build_s": t_build, "forms": forms,
            "workload": ("32 chains, n log-uniform [2e4, 2e5], p log-uniform [5e3, 4e4], "
                         "column densities log-uniform [1e-4, 0.2], tau log-uniform "
                         f"[1e-4, 1e-2]; relative preconditioned residual {tol:g}")}


def run_batched(args):
    import torch

    import paper_1810_12437_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    s = batched_summary(pk, torch, args.steps, args.warmup, args.tol, args.no_f32)
    forms = s["forms"]
    out = {
        "metric": "batched chain-draws/sec, 32 uneven chains",
        "value": forms["f64"]["chain_draws_per_s"],
        "unit": "chain-draws/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": forms["f64"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s["workload"], "chains": s["chains"],
                   "nnz_total": s["nnz_total"], "tol": args.tol, "seed": SEED},
        "generate_s": s["generate_s"], "handle_build_s": s["handle_build_s"],
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


def shared_summary(pk, torch, P, X, steps, warmup, tol, no_f32=False):
    """8 chains on the design of P (handle X for the single-chain path), each
    with its own omega, z, lambda, tau and stream; every X pass serves one
    group of four (K = 4 interleaved vectors).  Per form: chain-draws/s over `steps`
    batched draws against the same chains drawn one at a time."""
    import synth

    C = 8
    chains = synth.shared_x_chains(P, C, seed=1815)
    forms = {}
    for name, dtype, dt in (("f64", pk.F64, torch.float64), ("f32", pk.F32, torch.float32)):
        if name == "f32" and no_f32:
            continue
        t0 = time.perf_counter()
        B = pk.Batch.shared(P.n, P.p, P.row_ptr, P.col_idx, C, dtype=dtype)
        t_build = time.perf_counter() - t0
        om = [torch.as_tensor(c[0], device="cuda").to(dt) for c in chains]
        zz = [torch.as_tensor(c[1], device="cuda").to(dt) for c in chains]
        la = [torch.as_tensor(c[2], device="cuda").to(dt) for c in chains]
        ta = [c[3] for c in chains]
        for w in range(warmup):
            B.draw(om, zz, la, ta, [SEED] * C, list(range(C)), [1000 + w] * C, tol=tol)
        torch.cuda.synchronize()
        print(f"[bench] timing shared {name} ({steps} steps)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        iters = []
        for k in range(steps):
            _, infos = B.draw(om, zz, la, ta, [SEED] * C, list(range(C)), [k] * C, tol=tol)
            iters.append([i["iters"] + i["refine_iters"] for i in infos])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        it = np.array(iters, dtype=np.float64)
        f = {"chain_draws_per_s": C * steps / el, "ms_per_step": 1e3 * el / steps,
             "cg_iters_mean": float(it.mean()), "cg_iters_max": float(it.max()),
             "handle_build_s": t_build}
        t0 = time.perf_counter()
        for c in range(C):
            pk.draw(X, om[c], zz[c], la[c], ta[c], SEED, c, 0, tol=tol)
        torch.cuda.synchronize()
        f["single_chain_path_chain_draws_per_s"] = C / (time.perf_counter() - t0)
        f["speedup_vs_single_chain_path"] = (f["chain_draws_per_s"] /
                                             f["single_chain_path_chain_draws_per_s"])
        forms[name] = f
        B.close()
    return {"chains": C, "steps": steps, "forms": forms,
            "workload": ("8 chains on one n=1e5 p=2e4 binary X (column densities log-uniform "
                         "[1e-4, 0.2]); per-chain omega, z, lambda, tau = 1e-3 x exp(U[-1/2, 1/2]); "
                         f"relative preconditioned residual {tol:g}")}


def run_shared(args):
    import torch

    import paper_1810_12437_amd as pk
    import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    print("[bench] generating the n=1e5 p=2e4 design and 8 chains ...", file=sys.stderr,
          flush=True)
    P = synth.make_problem("c1")
    X = pk.Matrix.from_problem(P)
    s = shared_summary(pk, torch, P, X, args.steps, args.warmup, args.tol, args.no_f32)
    forms = s["forms"]
    out = {
        "metric": "shared-design chain-draws/sec, 8 chains, n=1e5 p=2e4",
        "value": forms["f64"]["chain_draws_per_s"],
        "unit": "chain-draws/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": forms["f64"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s["workload"], "chains": s["chains"], "nnz": P.nnz,
                   "tol": args.tol, "seed": SEED},
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


def large_summary(pk, torch, steps, warmup, tol):
    """The Gibbs-style sequence on the large design (n = 5e5, p = 5e4, 6.6e8
    non-zeros; tau = 0.05): 200 steps (``--steps``), each with omega and
    lambda redrawn from the config-0 laws (all steps' vectors resident in HBM
    before the timed region), FP32 vectors with the FP64 refinement restart,
    relative preconditioned residual ``--tol``, through the adaptive switch
    (period 100).  The pass kernels are timed with HIP events over the whole
    sequence; at this size the index streams (1.3 GB per orientation) cannot
    sit in the 256 MB MALL, so the pass rate is an HBM figure.  A 100-
    iteration prior-preconditioned FP64 solve is timed beside it (the prior
    preconditioner does not converge within p iterations on this law)."""
    import gc

    import synth

    t0 = time.perf_counter()
    P = synth.large_problem()
    t_gen = time.perf_counter() - t0
    print(f"[bench] large design nnz={P.nnz} in {t_gen:.1f} s; building the handle",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    X = pk.Matrix.from_csc(P.n, P.p, P.col_ptr, P.row_idx)
    t_build = time.perf_counter() - t0
    om_all = torch.empty((steps, P.n), dtype=torch.float32, device="cuda")
    la_all = torch.empty((steps, P.p), dtype=torch.float32, device="cuda")
    for k in range(steps):
        om, la = synth.sequence_vectors(P.n, P.p, k)
        om_all[k].copy_(torch.as_tensor(om))
        la_all[k].copy_(torch.as_tensor(la))
    z = torch.as_tensor(P.z, device="cuda").float()
    sw = pk.Switch(P.p, period=100)
    for w in range(warmup):
        d, m = pk.unshrunk_setup(la_all[w % steps], P.tau)
        sw.draw(X, om_all[w % steps], z, d, SEED, 1, w, precond_inv=m, tol=tol)
    sw.close()
    sw = pk.Switch(P.p, period=100)
    torch.cuda.synchronize()
    print(f"[bench] timing the {steps}-step sequence", file=sys.stderr, flush=True)
    X.profile(True)
    infos, choices = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        d, m = pk.unshrunk_setup(la_all[k], P.tau)
        _, info = sw.draw(X, om_all[k], z, d, SEED, 0, k, precond_inv=m, tol=tol)
        infos.append(info)
        if k % 100 == 0:
            choices.append(sw.state())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = X.stats()
    X.profile(False)
    sw.close()
    its = np.array([i["iters"] + i["refine_iters"] for i in infos], dtype=np.float64)
    c32, s32 = X.pass_bytes(pk.F32)
    t_pass = pass_time_ms(st)
    seq = {
        "steps": steps, "draws_per_s": steps / el, "ms_per_step": 1e3 * el / steps,
        "cg_iters_mean": float(its.mean()), "cg_iters_min": float(its.min()),
        "cg_iters_max": float(its.max()), "refined_draws": int(sum(i["refined"] for i in infos)),
        "not_converged": int(sum(i["status"] != pk.OK for i in infos)),
        "max_true_resid_over_tol": float(max(i["resid_true"] for i in infos)),
        "trials": choices,
        "pass_us": 1e3 * t_pass, "pass_launches": st["csr_launches"] + st["csc_launches"],
        "pass_gbps": 0.5 * (c32 + s32) / (t_pass * 1e-3) / 1e9,
    }
    seq["pass_frac"] = seq["pass_gbps"] / HBM_PEAK_GBPS
    _, copy_gbps = copy_rate()
    seq["copy_gbps"] = copy_gbps
    seq["pass_frac_of_copy"] = seq["pass_gbps"] / copy_gbps
    # the prior preconditioner's passes in FP64, 100 iterations of draw 0
    t = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    X.profile(True)
    _, info = pk.draw(X, t(P.omega), t(P.z), t(P.lam), P.tau, SEED, 0, 0, tol=tol,
                      max_iter=100)
    torch.cuda.synchronize()
    st = X.stats()
    X.profile(False)
    c64, s64 = X.pass_bytes(pk.F64)
    t64 = pass_time_ms(st)
    prior = {"status": info["status"], "iters": info["iters"],
             "resid_true_over_tol": info["resid_true"], "pass_us": 1e3 * t64,
             "pass_gbps": 0.5 * (c64 + s64) / (t64 * 1e-3) / 1e9,
             "row_pass_us": 1e3 * st["csr_ms"] / max(st["csr_launches"], 1),
             "col_pass_us": 1e3 * st["csc_ms"] / max(st["csc_launches"], 1),
             "bytes_per_launch": 0.5 * (c64 + s64)}
    prior["pass_frac"] = prior["pass_gbps"] / HBM_PEAK_GBPS
    prior["pass_frac_of_copy"] = prior["pass_gbps"] / copy_gbps
    del X, om_all, la_all, z
    gc.collect()
    return {"generate_s": t_gen, "handle_build_s": t_build, "sequence": seq,
            "prior_fp64_100_iterations": prior, "nnz": P.nnz, "n": P.n, "p": P.p,
            "tau": P.tau,
            "workload": ("n=5e5 p=5e4 binary X, column densities log-uniform "
                         "[1e-4, 0.2], tau=0.05, omega ~ Gamma(1, 0.25) + 0.01 and "
                         "lambda ~ half-Cauchy redrawn per step; FP32 vectors with the FP64 "
                         "refinement restart; adaptive prior/Jacobi preconditioner; "
                         f"relative residual {tol:g}")}


def run_large(args):
    import torch

    import paper_1810_12437_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    s = large_summary(pk, torch, args.steps, args.warmup, args.tol)
    seq = s["sequence"]
    out = {
        "metric": "Gibbs-style sequence draws/sec, n=5e5 p=5e4, FP32 + FP64 refinement",
        "value": seq["draws_per_s"], "unit": "draws/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": seq["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": s["workload"], "nnz": s["nnz"], "n": s["n"], "p": s["p"],
                   "tau": s["tau"]},
        "generate_s": s["generate_s"], "handle_build_s": s["handle_build_s"],
        "sequence": seq, "prior_fp64_100_iterations": s["prior_fp64_100_iterations"],
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.steps is None:
        args.steps = 200 if args.form == "large" else 20
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the sampler's "
              "data-parallel path is measured on a single MI355X (a multi-GPU run would "
              "row-partition X and all-reduce one p-vector per CG iteration).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.form == "batched":
        run_batched(args)
        return
    if args.form == "shared":
        run_shared(args)
        return
    if args.form == "large":
        run_large(args)
        return
    import torch

    import paper_1810_12437_amd as pk
    import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    print("[bench] generating workload n=1e5 p=2e4 ...", file=sys.stderr, flush=True)
    P = synth.make_problem("c1")
    X = pk.Matrix.from_problem(P)
    rel = {} if args.no_check else check_accuracy(pk, torch, X, P, args.tol)
    print(f"[bench] nnz={P.nnz}; rel err vs oracle {rel}; timing FP64 form "
          f"({args.warmup}+{args.steps} draws)", file=sys.stderr, flush=True)
    r64 = run_form(pk, torch, X, P, pk.F64, args.steps, args.warmup, args.tol)
    el, st, iters = r64["elapsed"], r64["stats"], r64["iters"]
    K = float(iters.mean())
    csr_b, csc_b = X.pass_bytes(pk.F64)
    csr_i32, csc_i32 = int32_pass_bytes(P, 8)
    t_pass = pass_time_ms(st)
    bytes_per_launch = 0.5 * (csr_b + csc_b)
    achieved = bytes_per_launch / (t_pass * 1e-3) / 1e9
    _, copy_gbps = copy_rate()  # achievable bandwidth on this device, after the timed draws
    iter_bytes = csr_b + csc_b + vec_bytes(P.p, 8)
    cg_gbps = iter_bytes * iters.sum() / el / 1e9
    traffic = None
    if TRAFFIC["bytes_per_launch"] is not None and TRAFFIC["sources_sha256"] == sources_sha256():
        traffic = TRAFFIC["bytes_per_launch"]
    out = {
        "metric": METRIC,
        "value": args.steps / el,
        "unit": "draws/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("n=1e5 p=2e4 binary X, column densities log-uniform [1e-4, 0.2], "
                         "tau=1e-3, 50 signal columns; FP64 vectors and scalars; "
                         f"relative preconditioned residual {args.tol:g}"),
            "nnz": P.nnz, "n": P.n, "p": P.p, "tol": args.tol, "seed": SEED,
        },
        "rel_err_vs_oracle": rel.get("f64"),
        "cg_iters_mean": K,
        "cg_iters_per_s": float(iters.sum() / el),
        "cg_hbm_gbps": cg_gbps,
        "cg_hbm_frac": cg_gbps / HBM_PEAK_GBPS,
        "max_true_resid_over_tol": float(max(i["resid_true"] for i in r64["infos"])),
        "roofline": {
            "kernel": "k_panel<double, 1> row pass (X s) and k_panel<double, 2> column pass (X^T u)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
            "avg_launch_us": 1e3 * t_pass,
            "row_pass_us": 1e3 * st["csr_ms"] / max(st["csr_launches"], 1),
            "col_pass_us": 1e3 * st["csc_ms"] / max(st["csc_launches"], 1),
            "launches": st["csr_launches"] + st["csc_launches"],
            "bytes_per_launch": bytes_per_launch,
            "int32_csr_csc_equiv_gbps": 0.5 * (csr_i32 + csc_i32) / (t_pass * 1e-3) / 1e9,
            "copy_gbps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
        },
    }
    if not args.no_f32:
        steps32 = max(3, args.steps // 2)
        print(f"[bench] timing FP32-vector form (1+{steps32} draws)", file=sys.stderr, flush=True)
        r32 = run_form(pk, torch, X, P, pk.F32, steps32, 1, args.tol)
        c32, s32 = X.pass_bytes(pk.F32)
        it32 = r32["iters"]
        out["f32_form"] = {
            "draws_per_s": steps32 / r32["elapsed"], "cg_iters_mean": float(it32.mean()),
            "cg_iters_per_s": float(it32.sum() / r32["elapsed"]),
            "cg_hbm_gbps": (c32 + s32 + vec_bytes(P.p, 4)) * it32.sum() / r32["elapsed"] / 1e9,
            "pass_gbps": 0.5 * (c32 + s32) / (pass_time_ms(r32["stats"]) * 1e-3) / 1e9,
            "refined_draws": int(sum(i["refined"] for i in r32["infos"])),
            "rel_err_vs_oracle": rel.get("f32"),
        }
    if not args.no_precond:
        print(f"[bench] preconditioner forms ({args.warmup}+{args.steps} draws each)",
              file=sys.stderr, flush=True)
        out["preconditioner_forms"] = precond_forms(pk, torch, P, X, args.steps, args.warmup,
                                                    args.tol)
    if not args.no_precond:
        print(f"[bench] adjoint form ({args.warmup}+{args.steps} solves)", file=sys.stderr,
              flush=True)
        out["adjoint_form"] = adjoint_forms(pk, torch, P, X, args.steps, args.warmup, args.tol)
    if not args.no_gibbs:
        print(f"[bench] Gibbs steps with the Polya-Gamma update ({args.warmup}+{args.steps} "
              "per form)", file=sys.stderr, flush=True)
        out["gibbs_step"] = gibbs_forms(pk, torch, P, X, args.steps, args.warmup, args.tol)
    if not args.no_forms:
        # the other workloads, summarised in the same line (fewer timed steps
        # than their own --form runs, except the large sequence, whose 200
        # steps are the workload)
        print("[bench] shared-design form (8 chains)", file=sys.stderr, flush=True)
        out["shared_form"] = shared_summary(pk, torch, P, X, FORM_STEPS, 1, args.tol,
                                            args.no_f32)
        print("[bench] batched form (32 uneven chains)", file=sys.stderr, flush=True)
        out["batched_form"] = batched_summary(pk, torch, FORM_STEPS, 1, args.tol, args.no_f32)
        print("[bench] large form (n=5e5 p=5e4, 200-step sequence)", file=sys.stderr,
              flush=True)
        out["large_form"] = large_summary(pk, torch, 200, 2, args.tol)
    if not args.no_cpu:
        print(f"[bench] CPU oracle sample ({args.cpu_draws} draws)", file=sys.stderr,
              flush=True)
        cb = cpu_baseline(P, args.tol, args.cpu_draws)
        cb["host"] = host_info()
        print("[bench] CPU oracle at n=2000 p=500 and the direct Cholesky draw",
              file=sys.stderr, flush=True)
        cb.update(cpu_small_and_direct(P, args.tol))
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
