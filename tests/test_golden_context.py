"""The paper's cost figures for its application design (Supplement S7.3 and
S7.4), used as context by the benchmark: check that they read as FP64 values
with int32 indices (12 B per non-zero, sizes in GiB) and one operation (a
multiply-add) per non-zero per product, the readings the benchmark's
comparison rests on."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def fig():
    with open(os.path.join(HERE, "golden", "supp_s7_cost_figures.json")) as f:
        return json.load(f)


def test_csr_size_is_fp64_values_with_int32_indices(fig):
    gib = 12 * fig["nnz"] / 2**30
    assert gib == pytest.approx(fig["csr_gb"], rel=5e-3)
    # 8-byte indices or 4-byte values would be far off.
    assert 16 * fig["nnz"] / 2**30 > 1.3 * fig["csr_gb"]
    assert 8 * fig["nnz"] / 2**30 < 0.7 * fig["csr_gb"]


def test_dense_phi_sizes_are_fp64_gib(fig):
    assert 8 * fig["p"] ** 2 / 2**30 == pytest.approx(fig["dense_phi_gb"], rel=5e-3)
    assert 8 * 1e5**2 / 2**30 == pytest.approx(fig["dense_phi_gb_at_p_1e5"], rel=5e-3)


def test_operation_counts_are_one_multiply_add_per_nonzero(fig):
    # X v and X^T w: one multiply-add per non-zero each.
    assert 2 * fig["nnz"] == pytest.approx(fig["flops_matvec_pair"], rel=1e-2)
    # A CG iteration is counted as twice the product pair.
    assert 2 * fig["flops_matvec_pair"] == pytest.approx(fig["flops_cg_iteration"], rel=1e-9)
    # Cholesky of Phi: p^3 / 3 multiply-adds, counted once each.
    assert fig["p"] ** 3 / 3 == pytest.approx(fig["flops_cholesky"], rel=0.01)
