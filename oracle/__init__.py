"""CPU FP64 oracle for the prior-preconditioned CG sampler.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this package; only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path: it is a plain, slow,
obviously-correct restatement of the paper's definitions in NumPy/SciPy at
double precision.

Modules
-------
ppcg_ref   Phi (dense and matrix-free), Prop 2.1 right-hand side, Cholesky
           solve and draw, preconditioned CG, adjoint gradient.
philox_ref Philox4x64-10 counter-based generator and the Box-Muller normals
           the sampler draws eta and delta from.
pg_ref     Polya-Gamma PG(1, c) draws (Devroye's exact sampler) and the
           pseudo-response of the Gibbs cycle's omega update.
stats_ref  Chi-square tests of draws against N(mu, Phi^-1) and N(m, Phi).
theory_ref The convergence bounds of Section 2 (used as test pins).

Every function names the passage of the paper it follows.  Parity status of
each function (what pins it to something other than itself) is listed in the
test modules ``tests/test_oracle_*.py``.
"""
from . import pg_ref, philox_ref, ppcg_ref, stats_ref, theory_ref  # noqa: F401
