"""Convenience layer over the C ABI: moves a host problem (scipy CSR A and
P0, numpy B and B_c) into device tensors and drives one emin_problem.

Marshalling only -- pattern growth, set-up, iteration and assembly all run
in libemin.so.
"""

from __future__ import annotations

import numpy as np

from . import emin as _c


def _dev(x, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _dev_matrix(X):
    """A (rows x m) FP64 device tensor from a numpy array or device tensor."""
    import torch

    if isinstance(X, torch.Tensor) and X.is_cuda:
        if X.dtype != torch.float64:
            raise TypeError("B and B_c must be FP64")
        X = X if X.dim() == 2 else X[:, None]
        return X.contiguous()
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    return _dev(X, torch.float64)


class DeviceCSR:
    """A scipy CSR matrix held as device tensors (int32 indices, FP64 values)."""

    def __init__(self, M, with_values: bool = True):
        import torch

        self.shape = M.shape
        self.rowptr = _dev(M.indptr.astype(np.int32), torch.int32)
        self.colind = _dev(M.indices.astype(np.int32), torch.int32)
        self.vals = _dev(M.data.astype(np.float64), torch.float64) if with_values else None

    def c(self) -> _c.emin_csr:
        return _c.make_csr(self.shape[0], self.shape[1], self.rowptr, self.colind, self.vals)

    def to_scipy(self):
        import scipy.sparse as sp

        vals = (self.vals.cpu().numpy() if self.vals is not None
                else np.ones(self.colind.numel()))
        return sp.csr_matrix((vals, self.colind.cpu().numpy(), self.rowptr.cpu().numpy()),
                             shape=self.shape)


class Context:
    """A device context.  Problems and batches made on it are closed before
    the context itself (the native context must outlive them)."""

    def __init__(self, device: int = 0, stream=None):
        import weakref

        self.handle = _c.emin_ctx_create(device, stream)
        self._children = weakref.WeakSet()

    def _adopt(self, child):
        self._children.add(child)

    def close(self):
        if self.handle:
            for ch in [c for c in self._children if isinstance(c, Batch)]:
                ch.close()
            for ch in list(self._children):
                ch.close()
            _c.emin_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ptent_setup(ctx: Context, S, cf, V, lmax: int, nc=None):
    """Alg. 1 on the device: the tentative prolongation of a C/F splitting
    (``cf``: coarse index of every COARSE node, -1 FINE; ``V``: n x m near
    kernel; ``S``: scipy CSR or DeviceCSR strength graph).  Returns
    (DeviceCSR P0 with nc columns, level of every row as numpy)."""
    import torch

    S = S if isinstance(S, DeviceCSR) else DeviceCSR(S, with_values=False)
    n = S.shape[0]
    cf_d = cf if isinstance(cf, torch.Tensor) else _dev(np.asarray(cf, np.int32), torch.int32)
    V_d = _dev_matrix(V)
    m = V_d.shape[1]
    if nc is None:
        nc = int(cf_d.max().item()) + 1 if n else 0
    rp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.empty(max(n * m, 1), dtype=torch.int32, device="cuda")
    vals = torch.empty(max(n * m, 1), dtype=torch.float64, device="cuda")
    level = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    nnz = _c.emin_ptent_setup(ctx.handle, S.c(), cf_d, nc, V_d, m, lmax, rp, ci, vals, level)
    P0 = DeviceCSR.__new__(DeviceCSR)
    P0.shape = (n, nc)
    P0.rowptr = rp
    P0.colind = ci[:nnz].contiguous()
    P0.vals = vals[:nnz].contiguous()
    return P0, level[:n].cpu().numpy()


class Problem:
    """One energy-minimization problem on the device.

    ``A``, ``P0``: scipy CSR, or DeviceCSR already on the device; ``B``
    (n x m), ``Bc`` (nc x m): numpy arrays, or FP64 device tensors.
    ``pattern``: optional (rowptr, colind) host arrays; default S^k P0.
    """

    def __init__(self, ctx: Context, A, P0, B, Bc, *, pattern=None, precision="fp64",
                 precond="jacobi", block=1, maxit=10, tau=0.0, pattern_power=1, profile=False,
                 k1_group=0, k1_slots=0, cf=None):
        import torch

        self.ctx = ctx
        self.A = A if isinstance(A, DeviceCSR) else DeviceCSR(A)
        self.P0 = P0 if isinstance(P0, DeviceCSR) else DeviceCSR(P0)
        self.B = _dev_matrix(B)
        self.Bc = _dev_matrix(Bc)
        self.m = self.B.shape[1]
        self.pattern_in = None
        if pattern is not None:
            rp, ci = pattern
            self.pattern_in = (_dev(np.asarray(rp, np.int32), torch.int32),
                               _dev(np.asarray(ci, np.int32), torch.int32))
        o = _c.emin_opts_default()
        o.precision = _c.EMIN_MIXED if precision == "mixed" else _c.EMIN_FP64
        o.precond = {"jacobi": _c.EMIN_JACOBI, "bjacobi": _c.EMIN_BJACOBI,
                     "sgs": _c.EMIN_SGS}[precond]
        o.block = int(block)
        o.maxit = int(maxit)
        o.tau = float(tau)
        o.pattern_power = int(pattern_power)
        o.profile = 1 if profile else 0
        o.k1_group = int(k1_group)  # masked-product shape hints (0: automatic)
        o.k1_slots = int(k1_slots)
        self.opts = o
        pat_c = None
        if self.pattern_in is not None:
            pat_c = _c.make_csr(A.shape[0], P0.shape[1], self.pattern_in[0], self.pattern_in[1])
        if cf is None:
            self.handle = _c.emin_problem_create(ctx.handle, self.A.c(), self.P0.c(), pat_c,
                                                 self.m, self.B, self.Bc, o)
        else:  # the C/F form P = [W; I]
            self.cf = cf if isinstance(cf, torch.Tensor) else _dev(np.asarray(cf, np.int32),
                                                                   torch.int32)
            self.handle = _c.emin_problem_create_cf(ctx.handle, self.A.c(), self.P0.c(), pat_c,
                                                    self.cf, self.m, self.B, self.Bc, o)
        ctx._adopt(self)
        self.nnz = _c.emin_pattern_get(self.handle)
        import weakref

        self._tapes = weakref.WeakSet()

    @classmethod
    def from_input(cls, ctx, inp, **kw):
        """Build from a ``gen.EminInput``-like object (A, P0, B, Bc, pattern_power,
        maxit, precond, block, extra['pattern'])."""
        kw.setdefault("maxit", inp.maxit)
        kw.setdefault("precond", inp.precond)
        kw.setdefault("block", inp.block)
        if inp.pattern_power == 0:
            kw.setdefault("pattern", inp.extra["pattern"])
        else:
            kw.setdefault("pattern_power", inp.pattern_power)
        return cls(ctx, inp.A, inp.P0, inp.B, inp.Bc, **kw)

    def pattern(self):
        import torch

        n = self.A.shape[0]
        rp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        _c.emin_pattern_get(self.handle, rp, ci)
        return rp.cpu().numpy(), ci[: self.nnz].cpu().numpy()

    def sgs_colours(self):
        """(number of colours, colour of every row) of an SGS problem."""
        import torch

        n = self.A.shape[0]
        col = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        nc = _c.emin_sgs_colours_get(self.handle, col)
        return nc, col[:n].cpu().numpy()

    def new_values(self):
        import torch

        return torch.empty(max(self.nnz, 1), dtype=torch.float64, device="cuda")

    def solve(self, out=None):
        """Run the numeric phase; returns (P tensor, status, dE history, stats)."""
        if out is None:
            out = self.new_values()
        status, hist, st = _c.emin_solve(self.handle, out, self.opts.maxit)
        return out, status, hist, st

    def energy(self, P) -> float:
        return _c.emin_energy(self.handle, P)

    def constraint_error(self, P) -> float:
        return _c.emin_constraint_error(self.handle, P)

    def masked_product(self, Y, Y_hat) -> None:
        _c.emin_masked_product(self.handle, Y, Y_hat)

    def solve_taped(self, out=None):
        """Solve and record the reverse-sweep tape; returns (P tensor, status, Tape)."""
        if out is None:
            out = self.new_values()
        status, h = _c.emin_solve_taped(self.handle, out)
        t = Tape(self, h)
        return out, status, t

    def loss(self, P, e=None, w_energy=1.0, w_twogrid=0.0, grad=True):
        """(L, dL/dP, dL/dA) of w_E tr(P^T A P) + w_T ||e - P c||_A^2 (gradients
        None when grad is False)."""
        import torch

        gP = gA = None
        if grad:
            gP = self.new_values()
            gA = torch.zeros_like(self.A.vals)
        L = _c.emin_loss(self.handle, P, e, w_energy, w_twogrid, gP, gA)
        return L, gP, gA

    def close(self):
        if getattr(self, "handle", None):
            for t in list(self._tapes):
                t.close()
            _c.emin_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tape:
    """Reverse-sweep record of one solve (closed before its problem)."""

    def __init__(self, problem: Problem, handle):
        self.problem = problem
        self.handle = handle
        problem._tapes.add(self)

    def backward(self, dL_dP, dL_dA=None):
        """Returns (dL/dA values, dL/dP0 values); dL_dA, when given, is added to."""
        import torch

        p = self.problem
        gA = torch.zeros_like(p.A.vals) if dL_dA is None else dL_dA
        gP0 = torch.empty_like(p.P0.vals)
        _c.emin_backward(self.handle, dL_dP, gA, gP0)
        return gA, gP0

    def close(self):
        if getattr(self, "handle", None):
            _c.emin_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many problems solved together (block-diagonal form, one HIP graph)."""

    def __init__(self, ctx: Context, problems, tune_cache=None):
        self.ctx = ctx
        self.problems = list(problems)
        self.handle = _c.emin_batch_create(ctx.handle, [p.handle for p in self.problems],
                                           tune_cache)
        ctx._adopt(self)
        self.outs = [p.new_values() for p in self.problems]

    def plan(self) -> str:
        return _c.emin_batch_plan(self.handle)

    def solve(self):
        status, stats = _c.emin_batch_solve(self.handle, self.outs)
        return self.outs, status, stats

    def close(self):
        if getattr(self, "handle", None):
            _c.emin_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
