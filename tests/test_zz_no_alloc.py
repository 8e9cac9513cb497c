"""The entry point that allocates nothing (ppcg_phi_matvec_noalloc) against
ppcg_phi_matvec, through the C ABI.

Two calls in a row on one device, the second on a smaller design, so the
second finds the first's values in the shared scratch array: both must equal
ppcg_phi_matvec bitwise (the same kernels in the same order; the oracle's
product is checked too, FP64 1e-12 and FP32 1e-5), in FP64 and FP32.  A
design whose partial sums exceed the fixed scratch is refused with
PPCG_ETOOBIG and its output left untouched."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1810_12437_amd as pk  # noqa: E402
import synth  # noqa: E402
from oracle import ppcg_ref as R  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def with_ones_column(P):
    """P with column 0 set to ones: at 40,000 rows its segments are cut into
    pieces, so the piece buffers of the scratch are used too."""
    rows = np.repeat(np.arange(P.n, dtype=np.int64), np.diff(P.row_ptr))
    key = np.unique(np.concatenate([rows * P.p + P.col_idx, np.arange(P.n) * P.p]))
    r = key // P.p
    rp = np.zeros(P.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=P.n), out=rp[1:])
    return synth.Problem(P.name, P.n, P.p, rp, (key - r * P.p).astype(np.int32), P.omega, P.z,
                         P.lam, P.tau)


@pytest.mark.parametrize("dt", [pk.F64, pk.F32], ids=["f64", "f32"])
def test_noalloc_matches_phi_matvec_on_two_calls(dt):
    big = with_ones_column(synth.scaled_problem(40000, 3000, seed=61, tau=0.02))
    small = synth.make_problem("c0")
    cast = (lambda a: np.asarray(a, np.float64)) if dt == pk.F64 else (
        lambda a: np.float32(a).astype(np.float64))
    tdt = torch.float64 if dt == pk.F64 else torch.float32
    for P in (big, small):
        X = pk.Matrix.from_problem(P)
        v = np.random.default_rng(P.n).standard_normal(P.p)
        om = torch.as_tensor(P.omega, device="cuda").to(tdt)
        lam = torch.as_tensor(P.lam, device="cuda").to(tdt)
        vt = torch.as_tensor(v, device="cuda").to(tdt)
        out = torch.full((P.p,), float("nan"), dtype=tdt, device="cuda")
        say(f"[noalloc] dtype={dt} n={P.n} p={P.p} nnz={P.nnz}")
        assert pk.phi_matvec_noalloc(X, om, lam, P.tau, vt, out) == pk.OK
        want = pk.phi_matvec(X, om, lam, P.tau, vt)
        torch.cuda.synchronize()
        assert torch.equal(out, want)
        Xs = R.csr_matrix(P.n, P.p, P.row_ptr, P.col_idx)
        ref = R.phi_matvec(Xs, cast(P.omega), cast(P.lam), P.tau, cast(v))
        e = float(np.linalg.norm(out.double().cpu().numpy() - ref) / np.linalg.norm(ref))
        say(f"   equal to ppcg_phi_matvec; rel err vs oracle {e:.1e}")
        assert e <= (1e-12 if dt == pk.F64 else 1e-5)


def test_noalloc_refuses_designs_beyond_its_scratch():
    """n = 2e5, p = 5e5, one entry per column: the column pass's FP64 partial
    sums alone are 10 panels x 5e5 x 8 B = 40 MB, over the 32 MiB array."""
    n, p = 200_000, 500_000
    rng = np.random.default_rng(62)
    rows = rng.integers(0, n, size=p)
    key = np.unique(rows * p + np.arange(p))
    r = key // p
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    X = pk.Matrix(n, p, rp, (key - r * p).astype(np.int32))
    om = torch.full((n,), 0.25, dtype=torch.float64, device="cuda")
    lam = torch.ones(p, dtype=torch.float64, device="cuda")
    v = torch.ones(p, dtype=torch.float64, device="cuda")
    out = torch.full((p,), 7.0, dtype=torch.float64, device="cuda")
    assert pk.phi_matvec_noalloc(X, om, lam, 0.5, v, out) == pk.ETOOBIG
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
