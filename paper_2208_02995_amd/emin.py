"""ctypes binding of libemin.so (the C ABI in include/emin.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  Functions keep the C names; device arrays are
passed as torch tensors (their ``data_ptr()``), streams as the current torch
stream.  There is no CPU fallback: if the library is missing, importing this
module raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libemin.so")

EMIN_OK = 0
EMIN_ERR_ARG = -1
EMIN_ERR_SHAPE = -2
EMIN_ERR_CSR = -3
EMIN_ERR_PATTERN = -4
EMIN_ERR_DIAG = -5
EMIN_ERR_BREAKDOWN = -6
EMIN_ERR_HIP = -7
EMIN_ERR_OOM = -8
EMIN_ERR_UNSUPPORTED = -9
EMIN_WARN_RANK = 1
EMIN_MAX_M = 8

EMIN_FP64 = 0
EMIN_MIXED = 1
EMIN_JACOBI = 0
EMIN_BJACOBI = 1
EMIN_SGS = 2
EMIN_STOP_MAXIT = 0
EMIN_STOP_CONVERGED = 1
EMIN_STOP_TAU = 2
EMIN_STOP_BREAKDOWN = 3
STOP_NAMES = {0: "maxit", 1: "converged", 2: "tau", 3: "breakdown"}

# every symbol include/emin.h declares
EXPORTS = (
    "emin_opts_default", "emin_ctx_create", "emin_ctx_destroy", "emin_problem_create",
    "emin_problem_destroy", "emin_pattern_get", "emin_sgs_colours_get", "emin_solve", "emin_energy", "emin_energy_noalloc",
    "emin_constraint_error", "emin_masked_product", "emin_last_error",
    "emin_batch_create", "emin_batch_solve", "emin_batch_plan", "emin_batch_destroy",
    "emin_solve_taped", "emin_backward", "emin_tape_destroy", "emin_loss",
    "emin_problem_create_cf", "emin_ptent_setup", "emin_loss_forward", "emin_loss_backward",
)


class EminError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"emin status {status}: {msg}")
        self.status = status


class emin_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class emin_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("precond", ctypes.c_int), ("block", ctypes.c_int),
                ("maxit", ctypes.c_int), ("tau", ctypes.c_double), ("pattern_power", ctypes.c_int),
                ("profile", ctypes.c_int), ("k1_group", ctypes.c_int), ("k1_slots", ctypes.c_int)]


class emin_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("rank_deficient_rows", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nnz_pattern", ctypes.c_int64), ("gamma1", ctypes.c_double),
                ("dE_first", ctypes.c_double), ("dE_last", ctypes.c_double),
                ("k1_ms", ctypes.c_double), ("k1_launches", ctypes.c_int64),
                ("solve_ms", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libemin.so (raises OSError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run __graft_entry__.build() or "
                      "python paper_2208_02995_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.emin_opts_default.argtypes = [P(emin_opts)]
    lib.emin_opts_default.restype = None
    lib.emin_ctx_create.argtypes = [i32, vp, P(vp)]
    lib.emin_ctx_create.restype = i32
    lib.emin_ctx_destroy.argtypes = [vp]
    lib.emin_ctx_destroy.restype = None
    lib.emin_problem_create.argtypes = [vp, P(emin_csr), P(emin_csr), P(emin_csr), i32, vp, vp,
                                        P(emin_opts), P(vp)]
    lib.emin_problem_create.restype = i32
    lib.emin_problem_destroy.argtypes = [vp]
    lib.emin_problem_destroy.restype = None
    lib.emin_problem_create_cf.argtypes = [vp, P(emin_csr), P(emin_csr), P(emin_csr), vp, i32,
                                           vp, vp, P(emin_opts), P(vp)]
    lib.emin_problem_create_cf.restype = i32
    lib.emin_ptent_setup.argtypes = [vp, P(emin_csr), vp, i32, vp, i32, i32, P(i64), vp, vp, vp,
                                     vp]
    lib.emin_ptent_setup.restype = i32
    lib.emin_pattern_get.argtypes = [vp, P(i64), vp, vp]
    lib.emin_pattern_get.restype = i32
    lib.emin_sgs_colours_get.argtypes = [vp, P(i32), vp]
    lib.emin_sgs_colours_get.restype = i32
    lib.emin_solve.argtypes = [vp, vp, P(dbl), P(emin_stats)]
    lib.emin_solve.restype = i32
    lib.emin_energy.argtypes = [vp, vp, P(dbl)]
    lib.emin_energy.restype = i32
    lib.emin_energy_noalloc.argtypes = [vp, vp, P(dbl)]
    lib.emin_energy_noalloc.restype = i32
    lib.emin_constraint_error.argtypes = [vp, vp, P(dbl)]
    lib.emin_constraint_error.restype = i32
    lib.emin_masked_product.argtypes = [vp, vp, vp]
    lib.emin_masked_product.restype = i32
    lib.emin_last_error.argtypes = []
    lib.emin_last_error.restype = ctypes.c_char_p
    lib.emin_batch_create.argtypes = [vp, i32, P(vp), ctypes.c_char_p, P(vp)]
    lib.emin_batch_create.restype = i32
    lib.emin_batch_solve.argtypes = [vp, P(vp), P(emin_stats)]
    lib.emin_batch_solve.restype = i32
    lib.emin_batch_plan.argtypes = [vp, ctypes.c_char_p, i32]
    lib.emin_batch_plan.restype = i32
    lib.emin_batch_destroy.argtypes = [vp]
    lib.emin_batch_destroy.restype = None
    lib.emin_solve_taped.argtypes = [vp, vp, P(vp)]
    lib.emin_solve_taped.restype = i32
    lib.emin_backward.argtypes = [vp, vp, vp, vp]
    lib.emin_backward.restype = i32
    lib.emin_tape_destroy.argtypes = [vp]
    lib.emin_tape_destroy.restype = None
    lib.emin_loss.argtypes = [vp, vp, vp, dbl, dbl, P(dbl), vp, vp]
    lib.emin_loss.restype = i32
    lib.emin_loss_forward.argtypes = [vp, vp, vp, dbl, dbl, P(dbl)]
    lib.emin_loss_forward.restype = i32
    lib.emin_loss_backward.argtypes = [vp, vp, vp, dbl, dbl, vp, vp]
    lib.emin_loss_backward.restype = i32
    _lib = lib
    return lib


def _check(status: int, allow_warn: bool = False) -> int:
    if status == EMIN_OK or (allow_warn and status == EMIN_WARN_RANK):
        return status
    msg = _lib.emin_last_error().decode(errors="replace")
    raise EminError(status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------- C names ---

def emin_opts_default() -> emin_opts:
    o = emin_opts()
    load_library().emin_opts_default(ctypes.byref(o))
    return o


def emin_ctx_create(device: int = 0, stream=None) -> ctypes.c_void_p:
    import torch

    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    h = ctypes.c_void_p()
    _check(lib.emin_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    return h


def emin_ctx_destroy(ctx) -> None:
    load_library().emin_ctx_destroy(ctx)


def make_csr(n_rows: int, n_cols: int, rowptr, colind, vals=None) -> emin_csr:
    return emin_csr(n_rows, n_cols, int(colind.numel()), rowptr.data_ptr(), colind.data_ptr(),
                    vals.data_ptr() if vals is not None else None)


def emin_problem_create(ctx, A: emin_csr, P0: emin_csr, pattern, m: int, B, Bc,
                        opts: emin_opts):
    h = ctypes.c_void_p()
    _check(load_library().emin_problem_create(
        ctx, ctypes.byref(A), ctypes.byref(P0), ctypes.byref(pattern) if pattern is not None else None,
        m, _ptr(B), _ptr(Bc), ctypes.byref(opts), ctypes.byref(h)))
    return h


def emin_problem_create_cf(ctx, A: emin_csr, P0: emin_csr, pattern, cf, m: int, B, Bc,
                           opts: emin_opts):
    h = ctypes.c_void_p()
    _check(load_library().emin_problem_create_cf(
        ctx, ctypes.byref(A), ctypes.byref(P0), ctypes.byref(pattern) if pattern is not None else None,
        _ptr(cf), m, _ptr(B), _ptr(Bc), ctypes.byref(opts), ctypes.byref(h)))
    return h


def emin_ptent_setup(ctx, S: emin_csr, cf, nc: int, V, m: int, lmax: int, rowptr, colind, vals,
                     level=None) -> int:
    """Alg. 1 into device tensors (colind / vals of capacity n * m); returns nnz."""
    nnz = ctypes.c_int64()
    _check(load_library().emin_ptent_setup(ctx, ctypes.byref(S), _ptr(cf), nc, _ptr(V), m, lmax,
                                           ctypes.byref(nnz), _ptr(rowptr), _ptr(colind),
                                           _ptr(vals), _ptr(level)))
    return nnz.value


def emin_problem_destroy(prob) -> None:
    load_library().emin_problem_destroy(prob)


def emin_sgs_colours_get(prob, colour=None) -> int:
    """Number of sweep colours of an EMIN_SGS problem; fills the device
    tensor ``colour`` (n int32) when given."""
    nc = ctypes.c_int32()
    _check(load_library().emin_sgs_colours_get(prob, ctypes.byref(nc), _ptr(colour)))
    return nc.value


def emin_pattern_get(prob, rowptr=None, colind=None) -> int:
    nnz = ctypes.c_int64()
    _check(load_library().emin_pattern_get(prob, ctypes.byref(nnz), _ptr(rowptr), _ptr(colind)))
    return nnz.value


def emin_solve(prob, P_vals, maxit: int):
    """Returns (status, dE history (numpy), emin_stats)."""
    hist = (ctypes.c_double * max(maxit, 1))()
    st = emin_stats()
    status = _check(load_library().emin_solve(prob, _ptr(P_vals), hist, ctypes.byref(st)),
                    allow_warn=True)
    return status, np.array(hist[:maxit]), st


def emin_energy(prob, P_vals) -> float:
    e = ctypes.c_double()
    _check(load_library().emin_energy(prob, _ptr(P_vals), ctypes.byref(e)))
    return e.value


def emin_energy_noalloc(prob, P_vals) -> float:
    e = ctypes.c_double()
    _check(load_library().emin_energy_noalloc(prob, _ptr(P_vals), ctypes.byref(e)))
    return e.value


def emin_constraint_error(prob, P_vals) -> float:
    e = ctypes.c_double()
    _check(load_library().emin_constraint_error(prob, _ptr(P_vals), ctypes.byref(e)))
    return e.value


def emin_masked_product(prob, Y, Y_hat) -> None:
    _check(load_library().emin_masked_product(prob, _ptr(Y), _ptr(Y_hat)))


def emin_last_error() -> str:
    return load_library().emin_last_error().decode(errors="replace")


def emin_batch_create(ctx, probs, tune_cache=None):
    """probs: sequence of problem handles (c_void_p)."""
    arr = (ctypes.c_void_p * len(probs))(*[p.value if isinstance(p, ctypes.c_void_p) else p
                                           for p in probs])
    h = ctypes.c_void_p()
    _check(load_library().emin_batch_create(
        ctx, len(probs), arr, tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
    return h


def emin_batch_solve(batch, P_list):
    """P_list: device tensors (one per member).  Returns (status, [emin_stats])."""
    n = len(P_list)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in P_list])
    stats = (emin_stats * n)()
    status = _check(load_library().emin_batch_solve(batch, ptrs, stats), allow_warn=True)
    return status, list(stats)


def emin_batch_plan(batch) -> str:
    lib = load_library()
    need = lib.emin_batch_plan(batch, None, 0)
    buf = ctypes.create_string_buffer(max(need, 1))
    lib.emin_batch_plan(batch, buf, need)
    return buf.value.decode()


def emin_batch_destroy(batch) -> None:
    load_library().emin_batch_destroy(batch)


def emin_solve_taped(prob, P_vals):
    """Returns (status, tape handle)."""
    t = ctypes.c_void_p()
    status = _check(load_library().emin_solve_taped(prob, _ptr(P_vals), ctypes.byref(t)),
                    allow_warn=True)
    return status, t


def emin_backward(tape, dL_dP, dL_dA, dL_dP0) -> None:
    """Adds dL/dA into dL_dA, writes dL/dP0 into dL_dP0."""
    _check(load_library().emin_backward(tape, _ptr(dL_dP), _ptr(dL_dA), _ptr(dL_dP0)))


def emin_tape_destroy(tape) -> None:
    load_library().emin_tape_destroy(tape)


def emin_loss_forward(prob, P_vals, e, w_energy: float, w_twogrid: float) -> float:
    L = ctypes.c_double()
    _check(load_library().emin_loss_forward(prob, _ptr(P_vals), _ptr(e), float(w_energy),
                                            float(w_twogrid), ctypes.byref(L)))
    return L.value


def emin_loss_backward(prob, P_vals, e, w_energy: float, w_twogrid: float, dL_dP=None,
                       dL_dA=None) -> None:
    _check(load_library().emin_loss_backward(prob, _ptr(P_vals), _ptr(e), float(w_energy),
                                             float(w_twogrid), _ptr(dL_dP), _ptr(dL_dA)))


def emin_loss(prob, P_vals, e, w_energy: float, w_twogrid: float, dL_dP=None, dL_dA=None) -> float:
    L = ctypes.c_double()
    _check(load_library().emin_loss(prob, _ptr(P_vals), _ptr(e), float(w_energy), float(w_twogrid),
                                    ctypes.byref(L), _ptr(dL_dP), _ptr(dL_dA)))
    return L.value
