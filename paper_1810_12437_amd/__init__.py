"""Prior-preconditioned CG sampler on MI355X: Python binding of libppcg.so.

Argument marshalling only: every step of the sampler runs in the HIP library
(``csrc/``) behind the C ABI declared in ``include/ppcg.h``.  There is no CPU
fallback; importing works without the library, but every call raises
``PPCGUnavailable`` when ``libppcg.so`` is missing.

Vectors are torch CUDA (HIP) tensors; PyTorch is used for device memory and
the current stream only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "F64", "F32", "REL_PRECOND", "RMS_PRECOND_ABS", "REL_PLAIN",
    "STREAM_ETA", "STREAM_DELTA", "Matrix", "Batch", "Options", "Info", "Chain",
    "phi_matvec", "normals", "rhs", "solve", "draw", "solve_backward",
    "solve_general", "draw_general", "phi_diag", "WarmStart", "moments_update",
    "unshrunk_setup", "jacobi_precond", "Switch", "PRECOND_PRIOR", "PRECOND_JACOBI",
    "pg_sample", "pg_update",
    "PPCGSolve", "PPCGError", "PPCGUnavailable", "lib", "LIB_PATH", "EXPORTED_SYMBOLS",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppcg.so")

F64, F32 = 0, 1
REL_PRECOND, RMS_PRECOND_ABS, REL_PLAIN = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
STREAM_ETA, STREAM_DELTA = 0, 1
OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EBREAKDOWN, ENODEV, ETOOBIG = 0, 1, 2, 3, 4, 5, 6, 7
_SOLVER_STATUS = (OK, ENOTCONV, EBREAKDOWN)

EXPORTED_SYMBOLS = (
    "ppcg_options_default", "ppcg_status_string", "ppcg_version",
    "ppcg_matrix_create", "ppcg_matrix_destroy", "ppcg_matrix_shape",
    "ppcg_phi_matvec", "ppcg_normals", "ppcg_rhs", "ppcg_solve", "ppcg_draw",
    "ppcg_solve_backward", "ppcg_matrix_profile", "ppcg_matrix_stats",
    "ppcg_matrix_pass_bytes", "ppcg_batch_create", "ppcg_batch_create_shared",
    "ppcg_batch_destroy",
    "ppcg_draw_batched", "ppcg_solve_batched",
    "ppcg_solve_general", "ppcg_draw_general", "ppcg_phi_diag",
    "ppcg_warm_start_accumulate", "ppcg_warm_start_vector",
    "ppcg_moments_update", "ppcg_unshrunk_setup", "ppcg_jacobi_precond",
    "ppcg_switch_create", "ppcg_switch_destroy", "ppcg_switch_state", "ppcg_draw_switch",
    "ppcg_pg_update", "ppcg_pg_sample", "ppcg_matrix_create_csc", "ppcg_phi_matvec_noalloc",
)


class PPCGError(RuntimeError):
    def __init__(self, what, code):
        super().__init__(f"{what}: {_status_string(code)} (code {code})")
        self.code = code


class PPCGUnavailable(ImportError):
    pass


class Options(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("criterion", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("refine", ctypes.c_int32),
        ("tol", ctypes.c_double), ("true_resid", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("loop_factor", ctypes.c_double),
        ("no_graph", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32), ("refined", ctypes.c_int32),
        ("resid_rec", ctypes.c_double), ("resid_true", ctypes.c_double),
        ("rms_precond", ctypes.c_double), ("bnorm_precond", ctypes.c_double),
        ("resid_true_first", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Chain(ctypes.Structure):
    _fields_ = [
        ("omega", ctypes.c_void_p), ("z", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("lambda_", ctypes.c_void_p), ("beta_out", ctypes.c_void_p), ("tau", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("chain", ctypes.c_uint64), ("draw_index", ctypes.c_uint64),
    ]


_lib = None
_vp, _i32, _i64, _u64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


def _declare(L):
    L.ppcg_options_default.argtypes = [ctypes.POINTER(Options), _i32]
    L.ppcg_options_default.restype = None
    L.ppcg_status_string.argtypes = [ctypes.c_int]
    L.ppcg_status_string.restype = ctypes.c_char_p
    L.ppcg_version.argtypes = []
    L.ppcg_version.restype = ctypes.c_char_p
    L.ppcg_matrix_create.argtypes = [ctypes.POINTER(_vp), _i64, _i64, _i64, _vp, _vp, _vp, _i32, _vp]
    L.ppcg_matrix_create_csc.argtypes = [ctypes.POINTER(_vp), _i64, _i64, _i64, _vp, _vp, _vp,
                                         _i32, _vp]
    L.ppcg_matrix_destroy.argtypes = [_vp]
    L.ppcg_matrix_shape.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    L.ppcg_phi_matvec.argtypes = [_vp, _vp, _vp, _dbl, _vp, _vp, _i32, _vp]
    L.ppcg_phi_matvec_noalloc.argtypes = [_vp, _vp, _vp, _dbl, _vp, _vp, _i32, _vp]
    L.ppcg_normals.argtypes = [_u64, _u64, _u64, _u64, _i64, _vp, _vp]
    L.ppcg_rhs.argtypes = [_vp, _vp, _vp, _vp, _dbl, _u64, _u64, _u64, _i32, _vp, _vp]
    L.ppcg_solve.argtypes = [_vp, _vp, _vp, _dbl, _vp, _vp, ctypes.POINTER(Options), _vp,
                             ctypes.POINTER(Info), _vp]
    L.ppcg_draw.argtypes = [_vp, _vp, _vp, _vp, _dbl, _u64, _u64, _u64, ctypes.POINTER(Options),
                            _vp, ctypes.POINTER(Info), _vp]
    L.ppcg_solve_general.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Options), _vp,
                                     ctypes.POINTER(Info), _vp]
    L.ppcg_draw_general.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _u64, _u64, _u64,
                                    ctypes.POINTER(Options), _vp, ctypes.POINTER(Info), _vp]
    L.ppcg_phi_diag.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp]
    L.ppcg_warm_start_accumulate.argtypes = [_vp, _vp, _vp, _dbl, _i32, _i64, _vp]
    L.ppcg_warm_start_vector.argtypes = [_vp, _vp, _dbl, _vp, _dbl, _i32, _i64, _vp]
    L.ppcg_moments_update.argtypes = [_vp, _vp, _vp, _i32, _i64, _i64, _vp]
    L.ppcg_unshrunk_setup.argtypes = [_vp, _vp, _vp, _vp, _i64, _dbl, _vp, _dbl, _i32, _i64,
                                      _i64, _vp]
    L.ppcg_jacobi_precond.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp]
    L.ppcg_switch_create.argtypes = [ctypes.POINTER(_vp), _i64, _i32]
    L.ppcg_switch_destroy.argtypes = [_vp]
    L.ppcg_switch_state.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                    ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
    L.ppcg_draw_switch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _u64, _u64, _vp,
                                   _vp, _vp, _vp]
    L.ppcg_pg_update.argtypes = [_vp, _vp, _vp, _u64, _u64, _u64, _i32, _vp, _vp, _vp]
    L.ppcg_pg_sample.argtypes = [_vp, _i64, _u64, _u64, _u64, _vp, _vp]
    L.ppcg_solve_backward.argtypes = [_vp, _vp, _vp, _dbl, _vp, _vp, ctypes.POINTER(Options),
                                      _vp, _vp, _vp, ctypes.POINTER(Info), _vp]
    L.ppcg_matrix_profile.argtypes = [_vp, _i32]
    L.ppcg_matrix_stats.argtypes = [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_i64),
                                    ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]
    L.ppcg_matrix_pass_bytes.argtypes = [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    L.ppcg_batch_create.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _i32, _vp]
    L.ppcg_batch_destroy.argtypes = [_vp]
    L.ppcg_batch_create_shared.argtypes = [ctypes.POINTER(_vp), _i32, _i64, _i64, _i64, _vp, _vp,
                                           _i32, _i32, _vp]
    L.ppcg_draw_batched.argtypes = [_vp, ctypes.POINTER(Chain), ctypes.POINTER(Options),
                                    ctypes.POINTER(Info), _vp]
    L.ppcg_solve_batched.argtypes = [_vp, ctypes.POINTER(Chain), ctypes.POINTER(Options),
                                     ctypes.POINTER(Info), _vp]
    for name in ("ppcg_batch_create", "ppcg_batch_create_shared", "ppcg_batch_destroy", "ppcg_draw_batched",
                 "ppcg_solve_batched", "ppcg_matrix_pass_bytes", "ppcg_matrix_profile", "ppcg_matrix_stats", "ppcg_matrix_create", "ppcg_matrix_destroy", "ppcg_matrix_shape",
                 "ppcg_matrix_create_csc", "ppcg_phi_matvec", "ppcg_normals", "ppcg_rhs", "ppcg_solve", "ppcg_draw",
                 "ppcg_solve_backward", "ppcg_solve_general", "ppcg_draw_general",
                 "ppcg_phi_diag", "ppcg_warm_start_accumulate", "ppcg_warm_start_vector",
                 "ppcg_moments_update", "ppcg_unshrunk_setup", "ppcg_jacobi_precond",
                 "ppcg_switch_create", "ppcg_switch_destroy", "ppcg_switch_state",
                 "ppcg_draw_switch", "ppcg_pg_update", "ppcg_pg_sample",
                 "ppcg_phi_matvec_noalloc"):
        getattr(L, name).restype = ctypes.c_int


def lib():
    """The loaded libppcg.so (raises PPCGUnavailable when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PPCGUnavailable(
                f"{LIB_PATH} is not built; build it with __graft_entry__.build(). "
                "The sampler has no CPU fallback.")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _status_string(code):
    try:
        return lib().ppcg_status_string(int(code)).decode()
    except Exception:  # pragma: no cover - library missing
        return "status"


def _check(rc, what, solver=False):
    if rc == OK or (solver and rc in _SOLVER_STATUS):
        return rc
    raise PPCGError(what, rc)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_TDTYPE = {}


def _tdtype(dtype):
    torch = _torch()
    return torch.float64 if dtype == F64 else torch.float32


def _dtype_of(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"vectors must be float32 or float64, got {t.dtype}")


def _dev(t, dtype, n, name):
    """Device pointer of a contiguous CUDA tensor of the given dtype and length."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != _tdtype(dtype):
        raise TypeError(f"{name} must be {_tdtype(dtype)}, got {t.dtype}")
    if t.dim() != 1 or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of length {n}")
    return ctypes.c_void_p(t.data_ptr())


class Matrix:
    """Handle of a binary design X (CSR index arrays, copied to the device)."""

    def __init__(self, n, p, row_ptr, col_idx):
        L = lib()
        torch = _torch()
        self.n, self.p = int(n), int(p)
        h = ctypes.c_void_p()
        if isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda:
            rp = row_ptr.to(torch.int64).contiguous()
            ci = col_idx.to(torch.int32).contiguous()
            nnz = int(ci.numel())
            rc = L.ppcg_matrix_create(ctypes.byref(h), self.n, self.p, nnz,
                                      ctypes.c_void_p(rp.data_ptr()),
                                      ctypes.c_void_p(ci.data_ptr() if nnz else 0), None,
                                      MEM_DEVICE, _stream())
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            nnz = int(ci.size)
            rc = L.ppcg_matrix_create(ctypes.byref(h), self.n, self.p, nnz,
                                      rp.ctypes.data_as(ctypes.c_void_p),
                                      ci.ctypes.data_as(ctypes.c_void_p) if nnz else None,
                                      None, MEM_HOST, _stream())
        _check(rc, "ppcg_matrix_create")
        self.nnz = nnz
        self._h = h

    @classmethod
    def from_csc(cls, n, p, col_ptr, row_idx):
        """The handle from host CSC index arrays (col_ptr int64 [p+1], row_idx
        int32 [nnz], rows strictly increasing within a column)."""
        self = cls.__new__(cls)
        self.n, self.p = int(n), int(p)
        cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
        ri = np.ascontiguousarray(row_idx, dtype=np.int32)
        nnz = int(ri.size)
        h = ctypes.c_void_p()
        rc = lib().ppcg_matrix_create_csc(ctypes.byref(h), self.n, self.p, nnz,
                                          cp.ctypes.data_as(ctypes.c_void_p),
                                          ri.ctypes.data_as(ctypes.c_void_p) if nnz else None,
                                          None, MEM_HOST, _stream())
        _check(rc, "ppcg_matrix_create_csc")
        self.nnz = nnz
        self._h = h
        return self

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("matrix handle is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ppcg_matrix_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable=True):
        """Start (and reset) or stop timing of the two X passes of the CG loop."""
        _check(lib().ppcg_matrix_profile(self.handle, 1 if enable else 0), "ppcg_matrix_profile")

    def stats(self):
        """{'csr_ms', 'csr_launches', 'csc_ms', 'csc_launches'} since profile(True)."""
        a, b = _dbl(), _dbl()
        na, nb = _i64(), _i64()
        _check(lib().ppcg_matrix_stats(self.handle, ctypes.byref(a), ctypes.byref(na),
                                       ctypes.byref(b), ctypes.byref(nb)), "ppcg_matrix_stats")
        return {"csr_ms": a.value, "csr_launches": na.value, "csc_ms": b.value,
                "csc_launches": nb.value}

    def pass_bytes(self, dtype):
        """(row pass, column pass) algorithmic bytes of one launch for `dtype`."""
        a, b = _i64(), _i64()
        _check(lib().ppcg_matrix_pass_bytes(self.handle, int(dtype), ctypes.byref(a),
                                            ctypes.byref(b)), "ppcg_matrix_pass_bytes")
        return a.value, b.value

    @classmethod
    def from_problem(cls, P):
        return cls(P.n, P.p, P.row_ptr, P.col_idx)


class _SharedDims:
    def __init__(self, n, p):
        self.n, self.p = n, p


class Batch:
    """Handle of C chains solved together (chain c on design matrices[c]; the
    same Matrix may serve several chains).  Each CG phase of all chains is one
    launch; a chain's result equals the single-chain call's."""

    def __init__(self, matrices, dtype=F64):
        L = lib()
        self.matrices = list(matrices)  # keeps the X handles alive
        if not self.matrices:
            raise ValueError("a batch needs at least one chain")
        self.dtype = int(dtype)
        arr = (ctypes.c_void_p * len(self.matrices))(*[m.handle.value for m in self.matrices])
        h = ctypes.c_void_p()
        _check(L.ppcg_batch_create(ctypes.byref(h), len(self.matrices), arr, self.dtype,
                                   _stream()), "ppcg_batch_create")
        self._h = h

    @classmethod
    def shared(cls, n, p, row_ptr, col_idx, nchains, dtype=F64):
        """nchains (1..8) chains on one design given as CSR arrays: each X
        pass reads the indices once for all chains."""
        L = lib()
        self = cls.__new__(cls)
        self.n, self.p = int(n), int(p)
        self.matrices = [_SharedDims(self.n, self.p)] * int(nchains)
        self.dtype = int(dtype)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.ppcg_batch_create_shared(ctypes.byref(h), int(nchains), self.n, self.p,
                                          int(ci.size), rp.ctypes.data_as(ctypes.c_void_p),
                                          ci.ctypes.data_as(ctypes.c_void_p) if ci.size else None,
                                          MEM_HOST, self.dtype, _stream()),
               "ppcg_batch_create_shared")
        self._h = h
        return self

    def __len__(self):
        return len(self.matrices)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch handle is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ppcg_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _run(self, fn, what, omegas, lams, taus, zs=None, bs=None, seeds=None, chains=None,
             draw_indices=None, **opts):
        torch = _torch()
        C = len(self.matrices)
        arr = (Chain * C)()
        outs = []
        for c, X in enumerate(self.matrices):
            dt = self.dtype
            beta = torch.empty(X.p, dtype=_tdtype(dt), device=omegas[c].device)
            outs.append(beta)
            ch = arr[c]
            ch.omega = _dev(omegas[c], dt, X.n, "omega")
            ch.lambda_ = _dev(lams[c], dt, X.p, "lambda")
            ch.beta_out = _dev(beta, dt, X.p, "beta")
            ch.tau = float(taus[c])
            if zs is not None:
                ch.z = _dev(zs[c], dt, X.n, "z")
                ch.seed = int(seeds[c])
                ch.chain = int(chains[c])
                ch.draw_index = int(draw_indices[c])
            if bs is not None:
                ch.b = _dev(bs[c], dt, X.p, "b")
        o = make_options(dtype=self.dtype, **opts)
        infos = (Info * C)()
        rc = fn(self.handle, arr, ctypes.byref(o), infos, _stream())
        _check(rc, what, solver=True)
        return outs, [i.as_dict() for i in infos]

    def draw(self, omegas, zs, lams, taus, seeds, chains, draw_indices, **opts):
        """One draw per chain (ppcg_draw of each); returns (betas, infos)."""
        return self._run(lib().ppcg_draw_batched, "ppcg_draw_batched", omegas, lams, taus, zs=zs,
                         seeds=seeds, chains=chains, draw_indices=draw_indices, **opts)

    def solve(self, omegas, lams, taus, bs, **opts):
        """Phi_c beta_c = b_c for every chain from zero; returns (betas, infos)."""
        return self._run(lib().ppcg_solve_batched, "ppcg_solve_batched", omegas, lams, taus,
                         bs=bs, **opts)


def make_options(dtype=F64, tol=1e-6, criterion=REL_PRECOND, max_iter=0, refine=-1,
                 true_resid=1, check_every=0, loop_factor=0.0, no_graph=0):
    o = Options()
    lib().ppcg_options_default(ctypes.byref(o), int(dtype))
    o.tol = float(tol)
    o.criterion = int(criterion)
    o.max_iter = int(max_iter)
    o.refine = int(refine)
    o.true_resid = int(true_resid)
    o.check_every = int(check_every)
    o.loop_factor = float(loop_factor)
    o.no_graph = int(no_graph)
    return o


def phi_matvec(X, omega, lam, tau, v):
    """out = Phi v (same dtype as v)."""
    torch = _torch()
    dt = _dtype_of(v)
    out = torch.empty(X.p, dtype=v.dtype, device=v.device)
    rc = lib().ppcg_phi_matvec(X.handle, _dev(omega, dt, X.n, "omega"), _dev(lam, dt, X.p, "lambda"),
                               float(tau), _dev(v, dt, X.p, "v"), _dev(out, dt, X.p, "out"), dt,
                               _stream())
    _check(rc, "ppcg_phi_matvec")
    return out


def phi_matvec_noalloc(X, omega, lam, tau, v, out):
    """out = Phi v into the caller's `out` through the entry point that
    allocates nothing (its scratch is a fixed per-device array); returns
    the status code (OK, or ETOOBIG when the fixed scratch is too small)."""
    dt = _dtype_of(v)
    rc = lib().ppcg_phi_matvec_noalloc(X.handle, _dev(omega, dt, X.n, "omega"),
                                       _dev(lam, dt, X.p, "lambda"), float(tau),
                                       _dev(v, dt, X.p, "v"), _dev(out, dt, X.p, "out"), dt,
                                       _stream())
    if rc not in (OK, ETOOBIG):
        raise PPCGError("ppcg_phi_matvec_noalloc", rc)
    return rc


def normals(seed, stream_id, chain, draw_index, count, device="cuda"):
    """FP64 normals of one generator stream (eta: 0, delta: 1)."""
    torch = _torch()
    out = torch.empty(int(count), dtype=torch.float64, device=device)
    rc = lib().ppcg_normals(int(seed), int(stream_id), int(chain), int(draw_index), int(count),
                            ctypes.c_void_p(out.data_ptr()), _stream())
    _check(rc, "ppcg_normals")
    return out


def rhs(X, omega, z, lam, tau, seed, chain, draw_index):
    """FP64 b of Prop 2.1 for draw (seed, chain, draw_index)."""
    torch = _torch()
    dt = _dtype_of(omega)
    b = torch.empty(X.p, dtype=torch.float64, device=omega.device)
    rc = lib().ppcg_rhs(X.handle, _dev(omega, dt, X.n, "omega"), _dev(z, dt, X.n, "z"),
                        _dev(lam, dt, X.p, "lambda"), float(tau), int(seed), int(chain),
                        int(draw_index), dt, ctypes.c_void_p(b.data_ptr()), _stream())
    _check(rc, "ppcg_rhs")
    return b


def solve(X, omega, lam, tau, b, beta0=None, **opts):
    """beta = Phi^-1 b by prior-preconditioned CG; returns (beta, info dict)."""
    torch = _torch()
    dt = _dtype_of(b)
    o = make_options(dtype=dt, **opts)
    beta = torch.empty(X.p, dtype=b.dtype, device=b.device)
    info = Info()
    rc = lib().ppcg_solve(X.handle, _dev(omega, dt, X.n, "omega"), _dev(lam, dt, X.p, "lambda"),
                          float(tau), _dev(b, dt, X.p, "b"),
                          None if beta0 is None else _dev(beta0, dt, X.p, "beta0"),
                          ctypes.byref(o), _dev(beta, dt, X.p, "beta"), ctypes.byref(info),
                          _stream())
    _check(rc, "ppcg_solve", solver=True)
    return beta, info.as_dict()


def draw(X, omega, z, lam, tau, seed, chain=0, draw_index=0, **opts):
    """One draw of beta ~ N(Phi^-1 X^T Omega z, Phi^-1); returns (beta, info dict)."""
    torch = _torch()
    dt = _dtype_of(omega)
    o = make_options(dtype=dt, **opts)
    beta = torch.empty(X.p, dtype=omega.dtype, device=omega.device)
    info = Info()
    rc = lib().ppcg_draw(X.handle, _dev(omega, dt, X.n, "omega"), _dev(z, dt, X.n, "z"),
                         _dev(lam, dt, X.p, "lambda"), float(tau), int(seed), int(chain),
                         int(draw_index), ctypes.byref(o), _dev(beta, dt, X.p, "beta"),
                         ctypes.byref(info), _stream())
    _check(rc, "ppcg_draw", solver=True)
    return beta, info.as_dict()


def _f64(v, n, name):
    """Device pointer of a float64 vector (prior precision, preconditioner)."""
    return _dev(v, F64, n, name)


def solve_general(X, omega, prior_prec, b, precond_inv=None, beta0=None, **opts):
    """beta = Phi^-1 b with Phi = X^T Omega X + diag(prior_prec) by CG with
    M^-1 = diag(precond_inv) (default 1 / prior_prec); prior_prec and
    precond_inv are float64 (Supplement S4.3).  Returns (beta, info dict)."""
    torch = _torch()
    dt = _dtype_of(b)
    o = make_options(dtype=dt, **opts)
    beta = torch.empty(X.p, dtype=b.dtype, device=b.device)
    info = Info()
    rc = lib().ppcg_solve_general(
        X.handle, _dev(omega, dt, X.n, "omega"), _f64(prior_prec, X.p, "prior_prec"),
        None if precond_inv is None else _f64(precond_inv, X.p, "precond_inv"),
        _dev(b, dt, X.p, "b"), None if beta0 is None else _dev(beta0, dt, X.p, "beta0"),
        ctypes.byref(o), _dev(beta, dt, X.p, "beta"), ctypes.byref(info), _stream())
    _check(rc, "ppcg_solve_general", solver=True)
    return beta, info.as_dict()


def draw_general(X, omega, z, prior_prec, seed, chain=0, draw_index=0, precond_inv=None,
                 beta0=None, **opts):
    """One draw of beta ~ N(Phi^-1 X^T Omega z, Phi^-1) with Phi = X^T Omega X +
    diag(prior_prec) (Prop 2.1 with that prior), CG preconditioned by
    M^-1 = diag(precond_inv), started from beta0.  Returns (beta, info dict)."""
    torch = _torch()
    dt = _dtype_of(omega)
    o = make_options(dtype=dt, **opts)
    beta = torch.empty(X.p, dtype=omega.dtype, device=omega.device)
    info = Info()
    rc = lib().ppcg_draw_general(
        X.handle, _dev(omega, dt, X.n, "omega"), _dev(z, dt, X.n, "z"),
        _f64(prior_prec, X.p, "prior_prec"),
        None if precond_inv is None else _f64(precond_inv, X.p, "precond_inv"),
        None if beta0 is None else _dev(beta0, dt, X.p, "beta0"), int(seed), int(chain),
        int(draw_index), ctypes.byref(o), _dev(beta, dt, X.p, "beta"), ctypes.byref(info),
        _stream())
    _check(rc, "ppcg_draw_general", solver=True)
    return beta, info.as_dict()


def phi_diag(X, omega, prior_prec):
    """diag(Phi) = X^T omega + prior_prec (float64); 1 / it is the Jacobi
    preconditioner's M^-1."""
    torch = _torch()
    dt = _dtype_of(omega)
    out = torch.empty(X.p, dtype=torch.float64, device=omega.device)
    rc = lib().ppcg_phi_diag(X.handle, _dev(omega, dt, X.n, "omega"), dt,
                             _f64(prior_prec, X.p, "prior_prec"),
                             ctypes.c_void_p(out.data_ptr()), _stream())
    _check(rc, "ppcg_phi_diag")
    return out


class WarmStart:
    """Rescaled running mean of the draws (Supplement S4.1): add(beta, lam, tau)
    after each draw with the scales it was drawn under; vector(lam, tau) gives
    beta0 for the next draw under its scales (None before the first add)."""

    def __init__(self, p, device="cuda"):
        torch = _torch()
        self.p = int(p)
        self.count = 0
        self.acc = torch.zeros(self.p, dtype=torch.float64, device=device)

    def add(self, beta, lam, tau):
        dt = _dtype_of(beta)
        rc = lib().ppcg_warm_start_accumulate(ctypes.c_void_p(self.acc.data_ptr()),
                                              _dev(beta, dt, self.p, "beta"),
                                              _dev(lam, dt, self.p, "lambda"), float(tau), dt,
                                              self.p, _stream())
        _check(rc, "ppcg_warm_start_accumulate")
        self.count += 1

    def vector(self, lam, tau):
        if self.count == 0:
            return None
        torch = _torch()
        dt = _dtype_of(lam)
        out = torch.empty(self.p, dtype=lam.dtype, device=lam.device)
        rc = lib().ppcg_warm_start_vector(_dev(out, dt, self.p, "beta0"),
                                          ctypes.c_void_p(self.acc.data_ptr()),
                                          float(self.count), _dev(lam, dt, self.p, "lambda"),
                                          float(tau), dt, self.p, _stream())
        _check(rc, "ppcg_warm_start_vector")
        return out


PRECOND_PRIOR, PRECOND_JACOBI = 0, 1


def moments_update(mean, m2, beta, count):
    """Welford update of the running mean / squared deviations of the leading
    len(mean) coefficients with the count-th draw (Supplement S4.3)."""
    dt = _dtype_of(beta)
    q1 = mean.numel()
    rc = lib().ppcg_moments_update(_f64(mean, q1, "mean"), _f64(m2, q1, "m2"),
                                   _dev(beta, dt, beta.numel(), "beta"), dt, q1, int(count),
                                   _stream())
    _check(rc, "ppcg_moments_update")


def unshrunk_setup(lam, tau, sigma_inv2=None, m2=None, count=0, c=1.0, want_precond=True):
    """(prior_prec, precond_inv) for ppcg_draw_general: the leading
    len(sigma_inv2) coefficients unshrunk with gamma_j^2 = c^2 m2_j/(count-1),
    the rest tau^-2 lambda^-2 and (tau lambda)^2 (Supplement S4.3)."""
    torch = _torch()
    dt = _dtype_of(lam)
    p = lam.numel()
    q1 = 0 if sigma_inv2 is None else sigma_inv2.numel()
    d = torch.empty(p, dtype=torch.float64, device=lam.device)
    m = torch.empty_like(d) if want_precond else None
    rc = lib().ppcg_unshrunk_setup(
        ctypes.c_void_p(d.data_ptr()), None if m is None else ctypes.c_void_p(m.data_ptr()),
        None if sigma_inv2 is None else _f64(sigma_inv2, q1, "sigma_inv2"),
        None if m2 is None else _f64(m2, q1, "m2"), int(count), float(c),
        _dev(lam, dt, p, "lambda"), float(tau), dt, q1, p, _stream())
    _check(rc, "ppcg_unshrunk_setup")
    return d, m


def jacobi_precond(X, omega, prior_prec):
    """M^-1 = 1 / diag(Phi), the Jacobi preconditioner (float64)."""
    torch = _torch()
    dt = _dtype_of(omega)
    out = torch.empty(X.p, dtype=torch.float64, device=omega.device)
    rc = lib().ppcg_jacobi_precond(X.handle, _dev(omega, dt, X.n, "omega"), dt,
                                   _f64(prior_prec, X.p, "prior_prec"),
                                   ctypes.c_void_p(out.data_ptr()), _stream())
    _check(rc, "ppcg_jacobi_precond")
    return out


class Switch:
    """Adaptive prior / Jacobi preconditioner choice (Supplement S5.3): every
    period-th draw solves the same draw under both and keeps the one with
    fewer CG iterations."""

    def __init__(self, p, period=100):
        self.handle = ctypes.c_void_p()
        _check(lib().ppcg_switch_create(ctypes.byref(self.handle), int(p), int(period)),
               "ppcg_switch_create")
        self.p = int(p)

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ppcg_switch_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self):
        c, n, ip, ij = _i32(), _i64(), _i32(), _i32()
        _check(lib().ppcg_switch_state(self.handle, ctypes.byref(c), ctypes.byref(n),
                                       ctypes.byref(ip), ctypes.byref(ij)), "ppcg_switch_state")
        return {"choice": "jacobi" if c.value == PRECOND_JACOBI else "prior", "draws": n.value,
                "iters_prior": ip.value, "iters_jacobi": ij.value}

    def draw(self, X, omega, z, prior_prec, seed, chain=0, draw_index=0, precond_inv=None,
             beta0=None, **opts):
        torch = _torch()
        dt = _dtype_of(omega)
        o = make_options(dtype=dt, **opts)
        beta = torch.empty(X.p, dtype=omega.dtype, device=omega.device)
        info = Info()
        rc = lib().ppcg_draw_switch(
            self.handle, X.handle, _dev(omega, dt, X.n, "omega"), _dev(z, dt, X.n, "z"),
            _f64(prior_prec, X.p, "prior_prec"),
            None if precond_inv is None else _f64(precond_inv, X.p, "precond_inv"),
            None if beta0 is None else _dev(beta0, dt, X.p, "beta0"), int(seed), int(chain),
            int(draw_index), ctypes.byref(o), _dev(beta, dt, X.p, "beta"), ctypes.byref(info),
            _stream())
        _check(rc, "ppcg_draw_switch", solver=True)
        return beta, info.as_dict()


def pg_sample(c, seed, chain=0, draw_index=0):
    """omega_i ~ PG(1, c_i) for a float64 CUDA vector of tilts (Supplement S1,
    step 3); float64 output."""
    torch = _torch()
    n = c.numel()
    out = torch.empty(n, dtype=torch.float64, device=c.device)
    rc = lib().ppcg_pg_sample(_f64(c, n, "c"), n, int(seed), int(chain), int(draw_index),
                              ctypes.c_void_p(out.data_ptr()), _stream())
    _check(rc, "ppcg_pg_sample")
    return out


def pg_update(X, beta, y, seed, chain=0, draw_index=0):
    """The Gibbs cycle's omega update: omega_i ~ PG(1, (X beta)_i) and the
    pseudo-response z_i = (y_i - 1/2) / omega_i, in beta's dtype; y is a
    uint8 CUDA vector of 0/1 outcomes.  Returns (omega, z)."""
    torch = _torch()
    dt = _dtype_of(beta)
    if not isinstance(y, torch.Tensor) or not y.is_cuda or y.dtype != torch.uint8 or \
            y.numel() != X.n or not y.is_contiguous():
        raise TypeError(f"y must be a contiguous uint8 CUDA vector of length {X.n}")
    omega = torch.empty(X.n, dtype=beta.dtype, device=beta.device)
    z = torch.empty_like(omega)
    rc = lib().ppcg_pg_update(X.handle, _dev(beta, dt, X.p, "beta"),
                              ctypes.c_void_p(y.data_ptr()), int(seed), int(chain),
                              int(draw_index), dt, ctypes.c_void_p(omega.data_ptr()),
                              ctypes.c_void_p(z.data_ptr()), _stream())
    _check(rc, "ppcg_pg_update")
    return omega, z


def solve_backward(X, omega, lam, tau, beta, grad_beta, **opts):
    """Adjoint of beta = Phi^-1 b: returns (grad_b, grad_loglambda, grad_logtau, info)."""
    torch = _torch()
    dt = _dtype_of(beta)
    o = make_options(dtype=dt, **opts)
    gb = torch.empty_like(beta)
    gl = torch.empty_like(beta)
    gt = torch.empty(1, dtype=torch.float64, device=beta.device)
    info = Info()
    rc = lib().ppcg_solve_backward(X.handle, _dev(omega, dt, X.n, "omega"),
                                   _dev(lam, dt, X.p, "lambda"), float(tau),
                                   _dev(beta, dt, X.p, "beta"), _dev(grad_beta, dt, X.p, "grad_beta"),
                                   ctypes.byref(o), _dev(gb, dt, X.p, "grad_b"),
                                   _dev(gl, dt, X.p, "grad_loglambda"),
                                   ctypes.c_void_p(gt.data_ptr()), ctypes.byref(info), _stream())
    _check(rc, "ppcg_solve_backward", solver=True)
    return gb, gl, gt, info.as_dict()


def _autograd_function():
    torch = _torch()

    class PPCGSolve(torch.autograd.Function):
        """beta = Phi(lambda, tau)^-1 b with lambda = exp(log_lambda), tau =
        exp(log_tau); gradients with respect to b, log_lambda and log_tau by
        the adjoint CG solve (no CG iterates are stored: the backward pass
        solves Phi a = dL/dbeta afresh)."""

        @staticmethod
        def forward(ctx, X, omega, b, log_lambda, log_tau, opts=None):
            opts = dict(opts or {})
            lam = torch.exp(log_lambda).contiguous()
            tau = float(torch.exp(log_tau.detach()).item())
            beta, info = solve(X, omega, lam, tau, b.contiguous(), **opts)
            ctx.X, ctx.tau, ctx.opts = X, tau, opts
            ctx.save_for_backward(omega, lam, beta)
            ctx.info = info
            return beta

        @staticmethod
        def backward(ctx, grad_beta):
            omega, lam, beta = ctx.saved_tensors
            gb, gl, gt, _ = solve_backward(ctx.X, omega, lam, ctx.tau, beta,
                                           grad_beta.contiguous(), **ctx.opts)
            gt = gt.reshape(()).to(beta.dtype)
            return None, None, gb, gl, gt, None

    return PPCGSolve


class _LazyAutograd:
    _fn = None

    def __getattr__(self, name):
        if _LazyAutograd._fn is None:
            _LazyAutograd._fn = _autograd_function()
        return getattr(_LazyAutograd._fn, name)


PPCGSolve = _LazyAutograd()
