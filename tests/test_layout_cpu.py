"""The panel-blocked layout of the X passes, checked on the host.

``tests/layout_check.cpp`` builds the library's tables (``ppcg_panels.h``)
for both orientations of X at both value sizes and runs a lane-by-lane model
of the pass kernel's reads over them (every window's loads, the stand-in
loads of idle lanes and of steps past a wavefront's end, the segmented lane
sums of packed chunks, the whole-wavefront sums of long chunks and of the
pieces of segments longer than one wavefront sums whole, the decode of the
one-vector tables' compact groups (a first index, a pad count and byte
differences, or 16-bit differences in the wide groups of sparse segments;
every index inside the panel) and the consumer's total over panels and
pieces).  Integer values make every sum exact, so the
model's X v and X^T u must equal the direct products element by element.
The program is built with AddressSanitizer and UndefinedBehaviorSanitizer,
so a read outside a table is reported by the sanitizer as well as by the
model's own bounds checks.

The cases reach every chunk kind: segments cut into pieces (a flat-prior
intercept column over n = 1e5 rows, Supplement S4.3; a dense column of
40,000 rows; a dense row of 16,400 columns), segment lengths on both sides
of the packed, long and piece thresholds, and the oracle-size design.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1810_12437_amd", "csrc")

# Thresholds of the layout (ppcg_layout.h): 16 entries per group, packed
# segments up to 64 x 4 groups, one wavefront sums at most 16 windows of
# 1024 entries whole.
GROUP, PACKED_MAX, LONG_MAX = 16, 64 * 4 * 16, 16 * 1024


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("layout") / "layout_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", CSRC, os.path.join(HERE, "layout_check.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _csr_from_columns(n, p, cols):
    """CSR arrays from a list of per-column row arrays."""
    rows = np.concatenate([np.asarray(c, dtype=np.int64) for c in cols]) if cols else np.zeros(0)
    cj = np.concatenate([np.full(len(c), j, dtype=np.int64) for j, c in enumerate(cols)])
    key = np.unique(rows * p + cj)
    r, c = key // p, (key % p).astype(np.int32)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    return rp, c


def _run(checker, tmp_path, n, p, rp, ci):
    f = tmp_path / "x.bin"
    with open(f, "wb") as fh:
        np.array([n, p, int(rp[-1])], dtype=np.int64).tofile(fh)
        np.asarray(rp, dtype=np.int64).tofile(fh)
        np.asarray(ci, dtype=np.int32).tofile(fh)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([checker, str(f)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"layout check failed:\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_intercept_column_over_1e5_rows(checker, tmp_path):
    """A flat-prior intercept (an all-ones column, Supplement S4.3) beside a
    column-law design at n = 1e5: in every panel of the row index the
    intercept's segment exceeds what one wavefront sums whole, so it is cut
    into pieces (FP64 panels of ~20,000 rows, FP32 of ~33,334)."""
    n, p = 100_000, 400
    rng = np.random.default_rng(31)
    rp0, ci0 = synth.column_law_design(n, p - 1, rng)
    # column 0: the intercept; the design's columns shift by one
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp0))
    cols = [np.arange(n)] + [rows[ci0 == j] for j in range(p - 1)]
    rp, ci = _csr_from_columns(n, p, cols)
    st = _run(checker, tmp_path, n, p, rp, ci)
    assert st["piece_chunks"] > 0 and st["pieces"] > 0 and st["long"] > 0
    assert st["mismatches"] == 0


def test_dense_column_and_dense_row(checker, tmp_path):
    """A dense column of 40,000 rows (two FP64 panels of 20,000: pieces in
    both; one FP32 panel of 40,000: three pieces) and a dense row of 16,400
    columns (one panel: pieces in the row orientation)."""
    n, p = 40_000, 16_400
    rng = np.random.default_rng(32)
    cols = [np.arange(n)]
    for j in range(1, p):
        k = int(rng.integers(0, 3))
        cols.append(np.concatenate([[7], rng.choice(n, size=k, replace=False)]))
    rp, ci = _csr_from_columns(n, p, cols)
    assert rp[8] - rp[7] == p  # row 7 is dense
    st = _run(checker, tmp_path, n, p, rp, ci)
    assert st["piece_chunks"] >= 2 * 2 + 3 and st["mismatches"] == 0


def test_segment_lengths_at_the_thresholds(checker, tmp_path):
    """Column lengths one group, one packed chunk, one long chunk and one
    wavefront's whole sum on either side of each threshold, and exact
    multiples of the piece length; rows of the same lengths."""
    lens = [1, GROUP - 1, GROUP, GROUP + 1, PACKED_MAX - GROUP, PACKED_MAX, PACKED_MAX + 1,
            LONG_MAX - 1, LONG_MAX, LONG_MAX + 1, 2 * LONG_MAX, 2 * LONG_MAX + 1, 3 * LONG_MAX - 7]
    n = max(lens) + 3
    rng = np.random.default_rng(33)
    cols = [np.sort(rng.choice(n, size=k, replace=False)) for k in lens]
    # rows of the same lengths: a block of columns shared by a few rows
    p_rows = LONG_MAX + 100
    p = len(lens) + p_rows
    for i, k in enumerate([GROUP + 1, PACKED_MAX + 1, LONG_MAX, LONG_MAX + 1]):
        for j in rng.choice(p_rows, size=k, replace=False):
            while len(cols) <= len(lens) + j:
                cols.append(np.zeros(0, dtype=np.int64))
            cols[len(lens) + j] = np.append(cols[len(lens) + j], i)
    while len(cols) < p:
        cols.append(np.zeros(0, dtype=np.int64))
    rp, ci = _csr_from_columns(n, p, cols)
    st = _run(checker, tmp_path, n, p, rp, ci)
    assert st["packed"] > 0 and st["long"] > 0 and st["piece_chunks"] > 0
    assert st["mismatches"] == 0


def test_oracle_size_and_ragged_designs(checker, tmp_path, problem_cache):
    """The n = 2000, p = 500 Bernoulli design, a column-law design with a
    ragged tail and a design with empty rows and columns."""
    P = problem_cache("c0")
    st = _run(checker, tmp_path, P.n, P.p, P.row_ptr, P.col_idx)
    assert st["mismatches"] == 0 and st["packed"] > 0
    P = synth.scaled_problem(4001, 903, seed=6)
    st = _run(checker, tmp_path, P.n, P.p, P.row_ptr, P.col_idx)
    assert st["mismatches"] == 0 and st["compact_groups"] > 0
    rng = np.random.default_rng(34)
    M = rng.random((900, 300)) < 0.1
    M[:, ::7] = False
    M[::5, :] = False
    rows, cols = np.nonzero(M)
    rp = np.zeros(901, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=900), out=rp[1:])
    st = _run(checker, tmp_path, 900, 300, rp, cols.astype(np.int32))
    assert st["mismatches"] == 0


def test_compact_groups_of_the_column_law(checker, tmp_path):
    """A column-law design at n = 30,000, p = 6,000 (densities down to 1e-4,
    so runs with differences beyond 255 cut groups short, and the sparsest
    columns take wide groups) and a design of very short columns beside a
    dense one: the compact groups reproduce X v and X^T u exactly."""
    P = synth.scaled_problem(30000, 6000, seed=35)
    st = _run(checker, tmp_path, P.n, P.p, P.row_ptr, P.col_idx)
    assert st["mismatches"] == 0 and st["compact_groups"] > st["wide_groups"] > 0
    n, p = 300, 21000
    rng = np.random.default_rng(36)
    cols = [np.sort(rng.choice(n, size=int(rng.integers(1, 5)), replace=False))
            for _ in range(p)]
    cols[0] = np.arange(n)
    rp, ci = _csr_from_columns(n, p, cols)
    st = _run(checker, tmp_path, n, p, rp, ci)
    assert st["mismatches"] == 0


def test_wide_groups_of_gapped_columns(checker, tmp_path):
    """Columns whose rows lie 200 to 600 apart (runs the 255 limit cuts) or
    256 to 4000 apart (isolated entries) beside Bernoulli(0.3) columns: the
    sparse ones take wide groups (16-bit differences), chunks of both kinds
    interleave, and the model reproduces X v and X^T u exactly."""
    P = synth.gapped_problem(12000, 400, seed=8)
    st = _run(checker, tmp_path, P.n, P.p, P.row_ptr, P.col_idx)
    assert st["mismatches"] == 0 and st["wide_groups"] > 1000
