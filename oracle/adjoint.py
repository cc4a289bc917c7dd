"""Reverse-mode derivatives of the oracle RCG (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/rcg.py).  Hand-written reverse sweep
of the path of oracle.rcg: pattern and B_c fixed, every stored entry of A and
of P0 an independent input.  With B_c fixed, W_i and Q_i are constants, so
the whole map (A values, P0 values) -> P is a composition of sums, products
and divisions -- analytic -- and the complex-step derivative of the forward
oracle pins this sweep (tests/test_adjoint_oracle.py).

Forward, iteration k of Alg. 3 (aggregation form, Jacobi):
    Z_k = Pi D^{-1} R_k,  gamma_k = <R_k, Z_k>,  Y_k = Z_k + beta_k Y_{k-1},
    beta_k = gamma_k / gamma_{k-1},  Yh_k = Pi K(A) Y_k,  delta_k = <Y_k, Yh_k>,
    alpha_k = gamma_k / delta_k,  dP += alpha_k Y_k,  R_{k+1} = R_k - alpha_k Yh_k
with R_1 = -Pi K(A) p0', p0' = Pi p_hat + G W b (Alg. 2), P = p0' + dP, and
K(A) y = mask(A Y) (Sec. 4).  A is symmetric at the point of evaluation, so
K(A)^T = K(A).

Loss (the differentiation workload): L = w_E tr(P^T A P) + w_T ||u||_A^2 with
u = e - P c, c = (P^T A P)^{-1} P^T A e.  Gradients of the loss in P and A:
energy 2 mask(A P) and (P P^T)_il on A's pattern; two-grid -2 (A u) c^T
masked to the pattern and u_i u_l on A's pattern (c minimises ||e - P c||_A,
so its own variation does not enter -- the envelope theorem).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import rcg as orc


def sddmm(A: sp.csr_matrix, rowptr, colind, U: np.ndarray, V: np.ndarray, nc: int) -> np.ndarray:
    """For every stored entry (i, l) of A: sum_j U(i, j) V(l, j) over the
    pattern, i.e. (U V^T)_il with U, V the matrices carried on the pattern."""
    Um = orc.as_matrix(U, rowptr, colind, nc)
    Vm = orc.as_matrix(V, rowptr, colind, nc)
    return orc.values_on_pattern(Um @ Vm.T, A.indptr, A.indices)


def diag_positions(A: sp.csr_matrix) -> np.ndarray:
    pos = np.empty(A.shape[0], dtype=np.int64)
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        pos[i] = A.indptr[i] + int(np.nonzero(cols == i)[0][0])
    return pos


def p0_positions(P0: sp.csr_matrix, rowptr, colind) -> np.ndarray:
    """Position in the pattern of every stored entry of P0."""
    nc = P0.shape[1]
    key_pat = orc.row_ids(np.asarray(rowptr)) * nc + np.asarray(colind, dtype=np.int64)
    key_p0 = orc.row_ids(P0.indptr) * nc + P0.indices.astype(np.int64)
    return np.searchsorted(key_pat, key_p0)


# ------------------------------------------------------------------- loss ---

def twogrid_parts(A, rowptr, colind, P, nc, e):
    """c = (P^T A P)^{-1} P^T A e and u = e - P c."""
    Pm = orc.as_matrix(P, rowptr, colind, nc)
    Ac = (Pm.T @ A @ Pm).tocsc()
    rhs = Pm.T @ (A @ e)
    c = spla.spsolve(Ac, rhs)
    u = e - Pm @ c
    return c, u


def loss(A, rowptr, colind, P, nc, e=None, w_energy=1.0, w_twogrid=1.0):
    L = w_energy * orc.energy(A, rowptr, colind, P, nc)
    if e is not None and w_twogrid != 0.0:
        c, u = twogrid_parts(A, rowptr, colind, P, nc, e)
        L = L + w_twogrid * np.sum(u * (A @ u))
    return L


def loss_grad(A, rowptr, colind, P, nc, e=None, w_energy=1.0, w_twogrid=1.0):
    """(dL/dP on the pattern, dL/dA on A's stored entries) at fixed P."""
    Pbar = 2.0 * w_energy * orc.masked_product(A, rowptr, colind, P, nc)
    Abar = w_energy * sddmm(A, rowptr, colind, P, P, nc)
    if e is not None and w_twogrid != 0.0:
        c, u = twogrid_parts(A, rowptr, colind, P, nc, e)
        Au = A @ u
        rows = orc.row_ids(np.asarray(rowptr))
        Pbar = Pbar - 2.0 * w_twogrid * Au[rows] * c[np.asarray(colind)]
        Ar = orc.row_ids(A.indptr)
        Abar = Abar + w_twogrid * u[Ar] * u[A.indices]
    return Pbar, Abar


# ---------------------------------------------------------- reverse sweep ---

def rcg_backward(A, P0, st, res, nc, Pbar):
    """Gradient of <Pbar, P(A, P0)> with respect to A's stored values and
    P0's stored values, through Alg. 2 and the iterations recorded in
    ``res.tape`` (oracle.rcg with keep_tape=True, Jacobi)."""
    rowptr, colind = st.rowptr, st.colind
    rows = orc.row_ids(rowptr)
    d = A.diagonal()
    dinv = 1.0 / d[rows]
    dpos = diag_positions(A)
    K = lambda x: orc.masked_product(A, rowptr, colind, x, nc)
    Pi = lambda x: orc.project(st, x)
    tape = res.tape
    n_it = res.iterations
    Abar = np.zeros(A.nnz, dtype=np.result_type(Pbar, A.data))
    p0bar = Pbar.copy()
    Rbar_next = np.zeros_like(Pbar)
    Ybar_next = np.zeros_like(Pbar)   # beta_{k+1} * Ybar_{k+1}
    gbar_next = 0.0                   # from beta_{k+1} = gamma_{k+1} / gamma_k
    for k in range(n_it, 0, -1):
        Y, R, Z = tape["Y"][k - 1], tape["R"][k - 1], tape["Z"][k - 1]
        g, dl, a, b = res.gamma[k - 1], res.delta[k - 1], res.alpha[k - 1], res.beta[k - 1]
        Yh = Pi(K(Y))
        Ybar = Ybar_next + a * Pbar
        abar = np.sum(Pbar * Y) - np.sum(Rbar_next * Yh)
        Rbar = Rbar_next.copy()
        Yhbar = -a * Rbar_next
        gbar = gbar_next + abar / dl
        dbar = -abar * g / dl ** 2
        Ybar = Ybar + dbar * Yh
        Yhbar = Yhbar + dbar * Y
        U = Pi(Yhbar)
        Ybar = Ybar + K(U)
        Abar = Abar + sddmm(A, rowptr, colind, U, Y, nc)
        Zbar = Ybar.copy()
        if k > 1:
            Yprev = tape["Y"][k - 2]
            gprev = res.gamma[k - 2]
            bbar = np.sum(Ybar * Yprev)
            Ybar_next = b * Ybar
            gbar = gbar + bbar / gprev
            gbar_next = -bbar * g / gprev ** 2
        else:
            Ybar_next = np.zeros_like(Pbar)
            gbar_next = 0.0
        Rbar = Rbar + gbar * Z
        Zbar = Zbar + gbar * R
        W = Pi(Zbar)                       # Z = Pi D^{-1} R
        Rbar = Rbar + W * dinv
        Abar[dpos] -= _rowsum(rows, W * R * dinv ** 2, A.shape[0])   # d(R/A_ii)/dA_ii
        Rbar_next = Rbar
    # R_1 = -Pi K(A) p0'
    V = -Pi(Rbar_next)
    p0bar = p0bar + K(V)
    Abar = Abar + sddmm(A, rowptr, colind, V, st.p0, nc)
    # p0' = Pi p_hat + constant (Alg. 2 with B_c fixed)
    phatbar = Pi(p0bar)
    P0bar = phatbar[p0_positions(P0, rowptr, colind)]
    return Abar, P0bar


def _rowsum(rows, x, n):
    out = np.zeros(n, dtype=x.dtype)
    np.add.at(out, rows, x)
    return out


# ------------------------------------------------------------ whole path ---

def forward(inp, A_vals=None, P0_vals=None, maxit=None, e=None, w_energy=1.0, w_twogrid=1.0,
            keep_tape=False):
    """Loss of the whole path for A's and P0's values (possibly complex, for
    complex-step checks).  Returns (L, st, res, A, P0)."""
    A = inp.A.copy()
    P0 = inp.P0.copy()
    if A_vals is not None:
        A = sp.csr_matrix((A_vals, inp.A.indices, inp.A.indptr), shape=inp.A.shape)
    if P0_vals is not None:
        P0 = sp.csr_matrix((P0_vals, inp.P0.indices, inp.P0.indptr), shape=inp.P0.shape)
    if inp.pattern_power == 0:
        rowptr, colind = inp.extra["pattern"]
    else:
        rowptr, colind = orc.pattern_expand(inp.A, inp.P0, inp.pattern_power)
    st = orc.emin_setup(rowptr, colind, P0, inp.B, inp.Bc)
    res = orc.rcg(A, st, inp.nc, inp.maxit if maxit is None else maxit, "jacobi",
                  keep_tape=keep_tape)
    L = loss(A, st.rowptr, st.colind, res.P, inp.nc, e, w_energy, w_twogrid)
    return L, st, res, A, P0


def gradient(inp, maxit=None, e=None, w_energy=1.0, w_twogrid=1.0):
    """dL/d(A values), dL/d(P0 values) by the reverse sweep."""
    L, st, res, A, P0 = forward(inp, maxit=maxit, e=e, w_energy=w_energy, w_twogrid=w_twogrid,
                                keep_tape=True)
    Pbar, Abar_direct = loss_grad(A, st.rowptr, st.colind, res.P, inp.nc, e, w_energy, w_twogrid)
    Abar, P0bar = rcg_backward(A, P0, st, res, inp.nc, Pbar)
    return L, Abar + Abar_direct, P0bar
