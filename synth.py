"""Seeded synthetic inputs for the prior-preconditioned CG sampler.

This module only draws random inputs: a binary design X (as CSR index
arrays), the Polya-Gamma stand-in weights omega, the pseudo-response z, the
local scales lambda and the global scale tau.  It holds none of the sampler's
arithmetic, and both the CPU oracle tests and the GPU path consume exactly the
arrays it returns.

Shapes and laws follow the workloads of the paper's setting (Section 1,
eq. beta_conditional; the application design of Section 4 is a sparse binary
matrix of infrequent features, 4 % dense), restated as these recipes:

* ``bernoulli_design``: i.i.d. Bernoulli(rho) entries.
* ``column_law_design``: per column j a density d_j = exp(U[ln dmin, ln dmax]),
  a count k_j ~ Binomial(n, d_j) and k_j distinct rows drawn uniformly.
* omega_i ~ Gamma(shape 1, scale 0.25) + 0.01 stands in for Polya-Gamma
  PG(1, psi) draws (mean 1/4 at psi = 0); z_i ~ N(0, 1); lambda_j is
  half-Cauchy(0, 1), optionally with a block of columns forced into
  log-uniform [10, 100] (the "signal" coefficients, cf. the simulation design
  of Section 3.2 where the first s coefficients are the signals).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "bernoulli_design",
    "column_law_design",
    "make_problem",
    "tiny_problem",
    "scaled_problem",
    "batched_problems",
    "shared_x_chains",
    "CONFIG_NAMES",
]


@dataclasses.dataclass
class Problem:
    """One beta-conditional: X (CSR, binary), omega, z, lambda, tau."""

    name: str
    n: int
    p: int
    row_ptr: np.ndarray  # int64 [n+1]
    col_idx: np.ndarray  # int32 [nnz], sorted within each row, unique
    omega: np.ndarray  # float64 [n], > 0
    z: np.ndarray  # float64 [n]
    lam: np.ndarray  # float64 [p], > 0
    tau: float

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense_x(self) -> np.ndarray:
        """Dense 0/1 copy of X (tiny problems only)."""
        x = np.zeros((self.n, self.p))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        x[rows, self.col_idx] = 1.0
        return x


def _csr_from_pairs(n: int, p: int, rows: np.ndarray, cols: np.ndarray):
    """Sorted, duplicate-free CSR index arrays from (row, col) pairs."""
    key = rows.astype(np.int64) * p + cols.astype(np.int64)
    key = np.unique(key)
    r = key // p
    c = (key - r * p).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return row_ptr, c


def bernoulli_design(n: int, p: int, rho: float, rng: np.random.Generator):
    """CSR index arrays of an n x p matrix with i.i.d. Bernoulli(rho) entries."""
    rows_out, cols_out = [], []
    block = max(1, int(4_000_000 // max(p, 1)))
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        m = rng.random((r1 - r0, p)) < rho
        rr, cc = np.nonzero(m)
        rows_out.append(rr + r0)
        cols_out.append(cc)
    rows = np.concatenate(rows_out) if rows_out else np.zeros(0, np.int64)
    cols = np.concatenate(cols_out) if cols_out else np.zeros(0, np.int64)
    return _csr_from_pairs(n, p, rows, cols)


def column_law_design(n: int, p: int, rng: np.random.Generator,
                      dmin: float = 1e-4, dmax: float = 0.2):
    """CSR index arrays under the log-uniform column-density law.

    Column j gets density d_j = exp(U[ln dmin, ln dmax]) and k_j ~ Binomial(n,
    d_j) distinct rows chosen uniformly.  Distinct rows are obtained by drawing
    with replacement and topping up until every column holds k_j distinct
    rows, which yields a uniformly random k_j-subset.
    """
    dens = np.exp(rng.uniform(math.log(dmin), math.log(dmax), size=p))
    k = rng.binomial(n, dens).astype(np.int64)
    k = np.minimum(k, n)
    have = np.zeros(p, dtype=np.int64)
    keys = np.zeros(0, dtype=np.int64)  # col * n + row, unique
    need = k.copy()
    while need.sum() > 0:
        cols = np.repeat(np.arange(p, dtype=np.int64), need)
        rows = rng.integers(0, n, size=cols.size, dtype=np.int64)
        keys = np.unique(np.concatenate([keys, cols * n + rows]))
        have = np.bincount(keys // n, minlength=p).astype(np.int64)
        need = k - have  # never negative: each round draws only the deficit
    cols = keys // n
    rows = keys - cols * n
    return _csr_from_pairs(n, p, rows, cols)


def column_law_csc(n: int, p: int, rng: np.random.Generator,
                   dmin: float = 1e-4, dmax: float = 0.2):
    """CSC index arrays (col_ptr, row_idx) under the same log-uniform
    column-density law, for large designs.

    A Binomial(n, d_j) count of distinct, uniformly chosen rows is the same
    law as i.i.d. Bernoulli(d_j) entries down the column, so each column's
    rows are drawn as running sums of Geometric(d_j) gaps: sorted and
    distinct by construction, O(nnz) work.  Each column draws
    ceil(n d_j + 8 sqrt(n d_j) + 16) gaps, which reach row n except with
    probability below 1e-14 per column (an error if one does not).
    """
    dens = np.exp(rng.uniform(math.log(dmin), math.log(dmax), size=p))
    mu = n * dens
    m = np.ceil(mu + 8.0 * np.sqrt(mu) + 16.0).astype(np.int64)
    starts = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(m, out=starts[1:])
    pos = np.cumsum(rng.geometric(np.repeat(dens, m)))
    ends = pos[starts[1:] - 1]
    base = np.concatenate([[0], ends[:-1]])
    rows = pos - np.repeat(base, m) - 1
    del pos
    if np.any(rows[starts[1:] - 1] < n):
        raise RuntimeError("a column's gaps ended before row n; draw with another seed")
    keep = rows < n
    cnt = np.add.reduceat(keep, starts[:-1]).astype(np.int64)
    rows = rows[keep].astype(np.int32)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(cnt, out=col_ptr[1:])
    return col_ptr, rows


@dataclasses.dataclass
class CscProblem:
    """A large workload held column-major (X = CSC index arrays)."""
    name: str
    n: int
    p: int
    col_ptr: np.ndarray  # int64 [p+1]
    row_idx: np.ndarray  # int32 [nnz], increasing within each column
    omega: np.ndarray
    z: np.ndarray
    lam: np.ndarray
    tau: float

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])


def large_problem(seed: int = 1812) -> CscProblem:
    """n = 5e5, p = 5e4 under the column-density law, config-0 vector laws
    (omega ~ Gamma(1, 0.25) + 0.01, z ~ N(0, 1), lambda ~ half-Cauchy),
    tau = 0.05; the sequence's later steps redraw omega and lambda with
    ``sequence_vectors``."""
    rng = np.random.default_rng(seed)
    n, p = 500_000, 50_000
    cp, ri = column_law_csc(n, p, rng)
    om, z, lam = _vectors(n, p, rng)
    return CscProblem("large", n, p, cp, ri, om, z, lam, 0.05)


def sequence_vectors(n: int, p: int, step: int, seed: int = 1816):
    """omega, lambda of step `step` of the Gibbs-style sequence (config-0
    laws, redrawn per step); z is held."""
    rng = np.random.default_rng([seed, step])
    omega = rng.gamma(1.0, 0.25, size=n) + 0.01
    lam = np.maximum(np.abs(rng.standard_cauchy(size=p)), 1e-300)
    return omega, lam


def _vectors(n: int, p: int, rng: np.random.Generator, n_forced: int = 0):
    omega = rng.gamma(1.0, 0.25, size=n) + 0.01
    z = rng.standard_normal(n)
    lam = np.abs(rng.standard_cauchy(size=p))
    lam = np.maximum(lam, 1e-300)
    if n_forced:
        m = min(n_forced, p)
        lam[:m] = np.exp(rng.uniform(math.log(10.0), math.log(100.0), size=m))
    return omega, z, lam


CONFIG_NAMES = ("c0", "c1", "c2", "c4small")


def make_problem(name: str, seed: int | None = None) -> Problem:
    """The fixed workloads.

    c0: n=2000, p=500, Bernoulli(0.05) design, tau=0.05.
    c1: n=1e5, p=2e4, column-density law, 50 forced lambdas, tau=1e-3.
    c2: n=5e5, p=5e4, column-density law, tau=0.05, through the CSR path
        (slow at this size: ``large_problem`` builds the same law column-major
        in O(nnz)).
    c4small: n=2000, p=400, the c1 laws at 1/50 scale (adjoint checks).
    """
    base = {"c0": 1810, "c1": 1811, "c2": 1812, "c4small": 1814}[name]
    rng = np.random.default_rng(base if seed is None else seed)
    if name == "c0":
        n, p = 2000, 500
        rp, ci = bernoulli_design(n, p, 0.05, rng)
        om, z, lam = _vectors(n, p, rng)
        tau = 0.05
    elif name == "c1":
        n, p = 100_000, 20_000
        rp, ci = column_law_design(n, p, rng)
        om, z, lam = _vectors(n, p, rng, n_forced=50)
        tau = 1e-3
    elif name == "c2":
        n, p = 500_000, 50_000
        rp, ci = column_law_design(n, p, rng)
        om, z, lam = _vectors(n, p, rng)
        tau = 0.05
    elif name == "c4small":
        n, p = 2000, 400
        rp, ci = column_law_design(n, p, rng)
        om, z, lam = _vectors(n, p, rng, n_forced=50)
        tau = 1e-3
    else:
        raise KeyError(name)
    return Problem(name, n, p, rp, ci, om, z, lam, float(tau))


def scaled_problem(n: int, p: int, seed: int, tau: float = 1e-3,
                   n_forced: int = 50, dmin: float = 1e-4, dmax: float = 0.2,
                   name: str = "scaled") -> Problem:
    """A column-law problem of arbitrary size (parity sweeps, ragged tails)."""
    rng = np.random.default_rng(seed)
    rp, ci = column_law_design(n, p, rng, dmin, dmax)
    om, z, lam = _vectors(n, p, rng, n_forced=n_forced)
    return Problem(name, n, p, rp, ci, om, z, lam, float(tau))


def gapped_problem(n: int, p: int, seed: int, tau: float = 0.3) -> Problem:
    """Columns whose consecutive rows lie a drawn gap apart: a third with gaps
    uniform in [200, 600) (runs cut at gaps above 255), a third with gaps in
    [256, 4000) (isolated entries), the rest Bernoulli(0.3); stresses the
    index groups of sparse segments (structure tests)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for j in range(p):
        kind = j % 3
        if kind == 2:
            r = np.flatnonzero(rng.random(n) < 0.3)
        else:
            lo, hi = (200, 600) if kind == 0 else (256, 4000)
            gaps = rng.integers(lo, hi, size=n // lo + 1)
            r = np.cumsum(gaps) - gaps[0] + int(rng.integers(0, lo))
            r = r[r < n]
        rows.append(r)
        cols.append(np.full(len(r), j))
    rp, ci = _csr_from_pairs(n, p, np.concatenate(rows), np.concatenate(cols))
    om, z, lam = _vectors(n, p, rng)
    return Problem("gapped", n, p, rp, ci, om, z, lam, float(tau))


def tiny_problem(p: int, n: int = 40, rho: float = 0.3, tau: float = 1.0,
                 seed: int = 7) -> Problem:
    """Tiny Bernoulli problems for distribution tests (dense Cholesky is exact)."""
    rng = np.random.default_rng(seed)
    rp, ci = bernoulli_design(n, p, rho, rng)
    om, z, lam = _vectors(n, p, rng)
    return Problem(f"tiny_p{p}", n, p, rp, ci, om, z, lam, float(tau))


def _batched_chain(args):
    c, n, p, tau, subseed = args
    sub = np.random.default_rng(subseed)
    rp, ci = column_law_design(n, p, sub)
    om, z, lam = _vectors(n, p, sub, n_forced=min(50, p // 8))
    return Problem(f"chain{c}", n, p, rp, ci, om, z, lam, float(tau))


def batched_problems(count: int = 32, seed: int = 1813, nmin: float = 2e4,
                     nmax: float = 2e5, pmin: float = 5e3, pmax: float = 4e4,
                     scale: float = 1.0, workers: int = 1) -> list[Problem]:
    """Independent chains of uneven size: n, p log-uniform, tau log-uniform
    in [1e-4, 1e-2], column-density law.  ``scale`` shrinks n and p for tests.
    Each chain draws from its own generator, so ``workers`` > 1 (processes)
    gives the same chains."""
    rng = np.random.default_rng(seed)
    specs = []
    for c in range(count):
        n = max(8, int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax))) * scale)))
        p = max(4, int(round(math.exp(rng.uniform(math.log(pmin), math.log(pmax))) * scale)))
        tau = math.exp(rng.uniform(math.log(1e-4), math.log(1e-2)))
        specs.append((c, n, p, tau, int(rng.integers(0, 2**63 - 1))))
    if workers <= 1:
        return [_batched_chain(s) for s in specs]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_batched_chain, specs))


def shared_x_chains(base: Problem, count: int, seed: int):
    """Per-chain (omega, z, lambda, tau) on one shared design ``base``."""
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(count):
        om, z, lam = _vectors(base.n, base.p, rng, n_forced=min(50, base.p // 8))
        tau = base.tau * math.exp(rng.uniform(-0.5, 0.5))
        chains.append((om, z, lam, float(tau)))
    return chains
