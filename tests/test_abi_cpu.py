"""Host-only checks of the C ABI: the library loads, exports every function
include/ppcg.h declares, its structs have the header's layout, and argument
validation rejects bad inputs before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1810_12437_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppcg.h")

needs_lib = pytest.mark.skipif(not os.path.exists(pk.LIB_PATH), reason="libppcg.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ppcg_[a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(pk.EXPORTED_SYMBOLS)


@needs_lib
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ppcg_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ppcg.h"\n'
        "int main(void){\n"
        ' printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ppcg_options), offsetof(ppcg_options, tol),'
        " offsetof(ppcg_options, true_resid), offsetof(ppcg_options, check_every),"
        " offsetof(ppcg_options, loop_factor), offsetof(ppcg_options, reserved));\n"
        ' printf("%zu %zu %zu %zu\\n", sizeof(ppcg_info), offsetof(ppcg_info, resid_rec),'
        " offsetof(ppcg_info, bnorm_precond), offsetof(ppcg_info, resid_true_first));\n"
        ' printf("%zu %zu %zu %zu %zu\\n", sizeof(ppcg_chain), offsetof(ppcg_chain, lambda),'
        " offsetof(ppcg_chain, tau), offsetof(ppcg_chain, seed),"
        " offsetof(ppcg_chain, draw_index));\n"
        " return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    o = [int(x) for x in lines[0].split()]
    i = [int(x) for x in lines[1].split()]
    assert o == [ctypes.sizeof(pk.Options), pk.Options.tol.offset, pk.Options.true_resid.offset,
                 pk.Options.check_every.offset, pk.Options.loop_factor.offset,
                 pk.Options.reserved.offset]
    assert i == [ctypes.sizeof(pk.Info), pk.Info.resid_rec.offset, pk.Info.bnorm_precond.offset,
                 pk.Info.resid_true_first.offset]
    ch = [int(x) for x in lines[2].split()]
    assert ch == [ctypes.sizeof(pk.Chain), pk.Chain.lambda_.offset, pk.Chain.tau.offset,
                  pk.Chain.seed.offset, pk.Chain.draw_index.offset]


@needs_lib
def test_host_only_entry_points():
    L = pk.lib()
    assert L.ppcg_version().startswith(b"ppcg")
    assert L.ppcg_status_string(pk.ENOTCONV) == b"not converged within max_iter"
    o = pk.Options()
    L.ppcg_options_default(ctypes.byref(o), pk.F32)
    assert (o.dtype, o.criterion, o.tol, o.refine, o.true_resid) == (pk.F32, pk.REL_PRECOND, 1e-6, -1, 1)


def _create(n, p, rp, ci, values=None, mem=pk.MEM_HOST):
    L = pk.lib()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    rc = L.ppcg_matrix_create(ctypes.byref(h), n, p, int(ci.size),
                              rp.ctypes.data_as(ctypes.c_void_p),
                              ci.ctypes.data_as(ctypes.c_void_p) if ci.size else None,
                              values, mem, None)
    return rc


@needs_lib
@pytest.mark.parametrize("case", ["offset0", "tail", "decreasing", "range", "unsorted", "dup",
                                  "negative", "values", "sizes", "mem"])
def test_create_rejects_bad_csr(case):
    rp, ci, n, p, values, mem = [0, 2, 3], [0, 2, 1], 2, 3, None, pk.MEM_HOST
    if case == "offset0":
        rp = [1, 2, 3]
    elif case == "tail":
        rp = [0, 2, 2]
    elif case == "decreasing":
        n, rp = 3, [0, 2, 1, 3]
    elif case == "range":
        ci = [0, 3, 1]
    elif case == "unsorted":
        ci = [2, 0, 1]
    elif case == "dup":
        ci = [1, 1, 1]
    elif case == "negative":
        ci = [-1, 2, 1]
    elif case == "values":
        values = ctypes.c_void_p(1)
    elif case == "sizes":
        p = 0
    elif case == "mem":
        mem = 7
    assert _create(n, p, rp, ci, values, mem) == pk.EINVAL


@needs_lib
def test_create_valid_input_reaches_device_check():
    """Valid input passes validation; without a GPU the call stops at the
    device check (on a GPU machine it succeeds)."""
    import torch
    L = pk.lib()
    h = ctypes.c_void_p()
    rp = np.array([0, 2, 3], dtype=np.int64)
    ci = np.array([0, 2, 1], dtype=np.int32)
    rc = L.ppcg_matrix_create(ctypes.byref(h), 2, 3, 3, rp.ctypes.data_as(ctypes.c_void_p),
                              ci.ctypes.data_as(ctypes.c_void_p), None, pk.MEM_HOST, None)
    if torch.cuda.is_available():
        assert rc == pk.OK
        assert L.ppcg_matrix_destroy(h) == pk.OK
    else:
        assert rc == pk.ENODEV


@needs_lib
def test_batch_entry_points_reject_bad_arguments():
    """Argument checks of the batch entry points happen before any device call."""
    L = pk.lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.ppcg_batch_create(ctypes.byref(h), 0, arr, pk.F64, None) == pk.EINVAL
    assert L.ppcg_batch_create(ctypes.byref(h), 2, arr, pk.F64, None) == pk.EINVAL  # NULL X
    assert L.ppcg_batch_create(ctypes.byref(h), 1, None, pk.F64, None) == pk.EINVAL
    assert L.ppcg_batch_create(None, 1, arr, pk.F64, None) == pk.EINVAL
    chains = (pk.Chain * 1)()
    assert L.ppcg_draw_batched(None, chains, None, None, None) == pk.EINVAL
    assert L.ppcg_solve_batched(None, chains, None, None, None) == pk.EINVAL
    assert L.ppcg_batch_destroy(None) == pk.OK


@needs_lib
def test_general_prior_entry_points_reject_bad_arguments():
    """NULL handle or NULL prior precision is rejected before any device call."""
    L = pk.lib()
    assert L.ppcg_solve_general(None, None, None, None, None, None, None, None, None,
                                None) == pk.EINVAL
    assert L.ppcg_draw_general(None, None, None, None, None, None, 0, 0, 0, None, None, None,
                               None) == pk.EINVAL
    assert L.ppcg_phi_diag(None, None, pk.F64, None, None, None) == pk.EINVAL


def test_warm_start_entry_points_reject_bad_arguments():
    """NULL arrays, p < 1, non-positive scales or an unknown dtype give
    PPCG_EINVAL before any launch."""
    L = pk.lib()
    one = ctypes.c_void_p(1)  # never dereferenced: every call below fails its checks first
    assert L.ppcg_warm_start_accumulate(None, one, one, 1.0, pk.F64, 4, None) == pk.EINVAL
    assert L.ppcg_warm_start_accumulate(one, one, one, 0.0, pk.F64, 4, None) == pk.EINVAL
    assert L.ppcg_warm_start_accumulate(one, one, one, 1.0, 7, 4, None) == pk.EINVAL
    assert L.ppcg_warm_start_accumulate(one, one, one, 1.0, pk.F64, 0, None) == pk.EINVAL
    assert L.ppcg_warm_start_vector(one, one, 0.0, one, 1.0, pk.F64, 4, None) == pk.EINVAL
    assert L.ppcg_warm_start_vector(one, one, 2.0, one, float("nan"), pk.F64, 4, None) == pk.EINVAL
    assert L.ppcg_warm_start_vector(one, None, 2.0, one, 1.0, pk.F32, 4, None) == pk.EINVAL


def test_gibbs_helpers_reject_bad_arguments():
    """Moments, unshrunk set-up, Jacobi and switch entry points check their
    arguments before any launch; a switch is created and destroyed without a
    device only when its arguments are bad."""
    L = pk.lib()
    one = ctypes.c_void_p(1)  # never dereferenced: every call below fails its checks first
    assert L.ppcg_moments_update(None, one, one, pk.F64, 3, 1, None) == pk.EINVAL
    assert L.ppcg_moments_update(one, one, one, pk.F64, 0, 1, None) == pk.EINVAL
    assert L.ppcg_moments_update(one, one, one, pk.F64, 3, 0, None) == pk.EINVAL
    assert L.ppcg_unshrunk_setup(one, one, one, one, 1, 2.0, one, 1.0, pk.F64, 2, 5,
                                 None) == pk.EINVAL  # count < 2
    assert L.ppcg_unshrunk_setup(one, one, one, one, 5, 0.0, one, 1.0, pk.F64, 2, 5,
                                 None) == pk.EINVAL  # c <= 0
    assert L.ppcg_unshrunk_setup(one, one, None, one, 5, 2.0, one, 1.0, pk.F64, 2, 5,
                                 None) == pk.EINVAL  # no sigma
    assert L.ppcg_unshrunk_setup(one, None, one, None, 5, 2.0, one, 1.0, pk.F64, 6, 5,
                                 None) == pk.EINVAL  # q1 > p
    assert L.ppcg_jacobi_precond(None, one, pk.F64, one, one, None) == pk.EINVAL
    h = ctypes.c_void_p()
    assert L.ppcg_switch_create(ctypes.byref(h), 0, 100) == pk.EINVAL
    assert L.ppcg_switch_create(ctypes.byref(h), 10, 0) == pk.EINVAL
    assert L.ppcg_switch_destroy(None) == pk.EINVAL
    assert L.ppcg_switch_state(None, None, None, None, None) == pk.EINVAL
    assert L.ppcg_draw_switch(None, None, None, None, None, None, None, 0, 0, 0, None, None,
                              None, None) == pk.EINVAL


def test_pg_entry_points_reject_bad_arguments():
    L = pk.lib()
    one = ctypes.c_void_p(1)  # never dereferenced: every call below fails its checks first
    assert L.ppcg_pg_update(None, one, one, 0, 0, 0, pk.F64, one, one, None) == pk.EINVAL
    assert L.ppcg_pg_sample(None, 5, 0, 0, 0, one, None) == pk.EINVAL
    assert L.ppcg_pg_sample(one, -1, 0, 0, 0, one, None) == pk.EINVAL


def _create_csc(n, p, cp, ri):
    L = pk.lib()
    h = ctypes.c_void_p()
    cp = np.ascontiguousarray(cp, dtype=np.int64)
    ri = np.ascontiguousarray(ri, dtype=np.int32)
    return L.ppcg_matrix_create_csc(ctypes.byref(h), n, p, int(ri.size),
                                    cp.ctypes.data_as(ctypes.c_void_p),
                                    ri.ctypes.data_as(ctypes.c_void_p) if ri.size else None,
                                    None, pk.MEM_HOST, None)


@needs_lib
@pytest.mark.parametrize("case", ["ok", "offset0", "tail", "range", "unsorted", "dup", "sizes"])
def test_create_csc_validates_columns(case):
    """Column-major input is checked as strictly as row-major: offsets from 0
    to nnz, rows in range and strictly increasing within a column; valid input
    stops at the device check without a GPU."""
    import torch
    cp, ri, n, p = [0, 1, 3, 3], [1, 0, 1], 2, 3
    if case == "offset0":
        cp = [1, 1, 3, 3]
    elif case == "tail":
        cp = [0, 1, 2, 2]
    elif case == "range":
        ri = [1, 0, 2]
    elif case == "unsorted":
        ri = [1, 1, 0]
    elif case == "dup":
        ri = [1, 0, 0]
    elif case == "sizes":
        n = 0
    rc = _create_csc(n, p, cp, ri)
    if case != "ok":
        assert rc == pk.EINVAL
    else:
        assert rc == (pk.OK if torch.cuda.is_available() else pk.ENODEV)
