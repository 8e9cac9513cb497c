"""bench.py's host side, without a GPU: the one-GPU refusal, the int32
CSR/CSC byte count reported beside the panel format's own bytes, and the
source hash that keeps the recorded HBM traffic tied to the kernels it was
counted on."""
import os
import string
import subprocess
import sys

import numpy as np

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_int32_pass_bytes_on_a_small_design():
    """A 3 x 4 binary X with rows {0, 2}, {}, {1, 2, 3}: 5 non-zeros, two
    non-empty rows, four non-empty columns, FP64 vectors."""
    rp = np.array([0, 2, 2, 5], np.int64)
    ci = np.array([0, 2, 1, 2, 3], np.int32)
    P = synth.Problem("t", 3, 4, rp, ci, np.ones(3), np.zeros(3), np.ones(4), 1.0)
    csr, csc = bench.int32_pass_bytes(P, 8)
    # row pass: 5 int32 indices, 3 int64 row offsets (two rows and the end),
    # the gathered p-vector, omega over n, two row outputs
    assert csr == 5 * 4 + 3 * 8 + 4 * 8 + 3 * 8 + 2 * 8
    # column pass: 5 int32 indices, 5 int64 column offsets, u over n, four
    # column outputs
    assert csc == 5 * 4 + 5 * 8 + 3 * 8 + 4 * 8


def test_traffic_record_names_its_sources():
    h = bench.sources_sha256()
    assert len(h) == 64 and set(h) <= set(string.hexdigits.lower())
    rec = bench.TRAFFIC
    assert set(rec) == {"sources_sha256", "bytes_per_launch"}
    assert len(rec["sources_sha256"]) == 64
    assert rec["bytes_per_launch"] is None or rec["bytes_per_launch"] > 0
    for rel in bench.PASS_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, rel)), rel
