"""CPU FP64 oracle of the energy-minimization RCG (arXiv 2208.02995).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library.  It is plain numpy/scipy, slow on
purpose and written to be checked against the paper by eye.

Notation (aggregation form of the paper's problem, every row of P free):

* ``A``       n x n SPD operator (scipy CSR).
* pattern     (rowptr, colind) of P, columns sorted ascending; J_i is the
              column set of row i (Sec. 3, eq. Constr).
* values      a flat array of length nnz(pattern), row-wise order -- the
              paper's p-tilde (Sec. 3, eq. Constr_Mat).
* ``B``       n x m fine near-kernel basis (the paper's V_f, rows v_i).
* ``Bc``      nc x m coarse basis (the paper's V_c); G_i = Bc[J_i, :] is the
              transpose of the paper's local block V_c(J_i,:)^T.

Readings where the paper is silent or garbled (listed with reasons in the
design notes): every row is free and f = 0, so the initial residual is
r = -Pi K w0; the local block is factored as the tall G_i (QR when
l_i >= m, else / on rank failure an SVD) with the min-norm correction
delta = Q R^{-T} r; the rank tolerance is max(l_i, m) * 2^-52 relative to the
largest |R_jj| or sigma_1; the first-iteration test reads "k = 1"; a relative
floor gamma_k <= 1e-26 gamma_1 ends the loop as converged; the energy stop,
when tau > 0, skips the update of the iteration that triggers it and then
assembles P.

Dot products use the bilinear form sum(x * y) (no conjugation) so every
function is analytic in its inputs and can be differentiated by complex step.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import sgs

EPS = 2.0 ** -52


# --------------------------------------------------------------------------
# helpers on a fixed pattern
# --------------------------------------------------------------------------

def row_ids(rowptr: np.ndarray) -> np.ndarray:
    """Row index of every pattern entry."""
    n = rowptr.shape[0] - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))


def _row_sum_matrix(rowptr: np.ndarray) -> sp.csr_matrix:
    """S (n x nnz) with S[i, s] = 1 when entry s lies in row i; S @ x sums
    entry-wise data per row."""
    n = rowptr.shape[0] - 1
    nnz = int(rowptr[-1])
    return sp.csr_matrix((np.ones(nnz), np.arange(nnz), rowptr.astype(np.int64)), shape=(n, nnz))


def values_on_pattern(M: sp.spmatrix, rowptr: np.ndarray, colind: np.ndarray) -> np.ndarray:
    """Entries of the sparse matrix M at the pattern positions (0 where M has
    no stored entry)."""
    M = sp.csr_matrix(M)
    M.sort_indices()
    ncol = M.shape[1]
    mk = row_ids(M.indptr).astype(np.int64) * ncol + M.indices.astype(np.int64)
    pk = row_ids(rowptr) * ncol + colind.astype(np.int64)
    pos = np.searchsorted(mk, pk)
    pos_c = np.minimum(pos, max(mk.shape[0] - 1, 0))
    found = (pos < mk.shape[0]) & (mk[pos_c] == pk) if mk.shape[0] else np.zeros(pk.shape, bool)
    out = np.zeros(pk.shape[0], dtype=M.dtype)
    out[found] = M.data[pos_c[found]]
    return out


def as_matrix(values: np.ndarray, rowptr: np.ndarray, colind: np.ndarray, nc: int) -> sp.csr_matrix:
    n = rowptr.shape[0] - 1
    return sp.csr_matrix((values, colind, rowptr), shape=(n, nc))


# --------------------------------------------------------------------------
# a1. Pattern growth  (Sec. 3, eq. enlPatt)
# --------------------------------------------------------------------------

def pattern_expand(A: sp.csr_matrix, P0: sp.csr_matrix, k: int):
    """Pattern of  S^k P0bar  with S = struct(A): the entries of A and of P0
    are replaced by ones and the product is taken in 0/1 arithmetic, so no
    entry can cancel (Sec. 3, eq. enlPatt).  Returns sorted CSR
    (rowptr, colind) as int32."""
    S = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    T = sp.csr_matrix((np.ones(P0.nnz), P0.indices, P0.indptr), shape=P0.shape)
    for _ in range(k):
        T = S @ T
    T = sp.csr_matrix(T)
    T.sort_indices()
    return T.indptr.astype(np.int32), T.indices.astype(np.int32)


def pattern_contains(rowptr, colind, P0: sp.csr_matrix) -> bool:
    """True when every stored entry of P0 lies in the pattern (P is grown from
    P0's pattern, Sec. 3)."""
    ones = sp.csr_matrix((np.ones(colind.shape[0]), colind, rowptr), shape=P0.shape)
    hit = values_on_pattern(ones, P0.indptr, P0.indices)
    return bool(np.all(hit == 1.0))


# --------------------------------------------------------------------------
# a2. Set-up of P0 and of the block projector  (Sec. 3.2, Alg. 2)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Setup:
    rowptr: np.ndarray
    colind: np.ndarray
    p0: np.ndarray         # final tentative prolongation values on the pattern
    Q: np.ndarray          # (nnz, m): row i's block holds an orthonormal basis of range(G_i)
    rank: np.ndarray       # (n,) rank used for each row
    used_svd: np.ndarray   # (n,) True where the SVD branch ran
    m: int


def rank_tol(l: int, m: int) -> float:
    return max(l, m) * EPS


def emin_setup(rowptr, colind, P0: sp.csr_matrix, B: np.ndarray, Bc: np.ndarray) -> Setup:
    """Alg. 2 (Energy Minimization Set-Up) row by row:

    gather G_i = Bc[J_i,:], b_i = B[i,:] and the starting row p_hat_i (P0's
    row placed on J_i); r_i = b_i - G_i^T p_hat_i.  When l_i >= m take the
    economy QR G_i = Q_i R_i; if R_i is full rank, delta_i = Q_i R_i^{-T} r_i
    (the min-norm solution of G_i^T delta = r_i).  When l_i < m or the rank
    test fails take the SVD G_i = U S V^T, keep the k_i singular values above
    the tolerance, Q_i = U(:, :k_i) and delta_i = U_k S_k^{-1} V_k^T r_i (the
    least-squares min-norm solution).  Then p0_i = p_hat_i + delta_i and the
    row's projector is I - Q_i Q_i^T.

    Rows are independent; rows of equal length are factored together
    (stacked LAPACK calls), which is the same per-row arithmetic."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    n = rowptr.shape[0] - 1
    m = Bc.shape[1]
    nnz = colind.shape[0]
    p_hat = values_on_pattern(P0, rowptr, colind)
    if not pattern_contains(rowptr.astype(np.int32), colind.astype(np.int32), P0):
        raise ValueError("pattern does not contain P0's pattern")
    G_all = np.asarray(Bc, dtype=np.float64)[colind, :]                    # (nnz, m)
    S = _row_sum_matrix(rowptr)
    r_all = B - S @ (G_all * p_hat[:, None])                               # (n, m)
    Q = np.zeros((nnz, m))
    delta = np.zeros(nnz, dtype=np.result_type(p_hat, r_all))
    rank = np.zeros(n, dtype=np.int64)
    used_svd = np.zeros(n, dtype=bool)
    lens = np.diff(rowptr)
    svd_rows = []
    for L in np.unique(lens):
        rows = np.nonzero(lens == L)[0]
        if L == 0:
            svd_rows.extend(rows.tolist())
            continue
        idx = rowptr[rows][:, None] + np.arange(L)[None, :]                # (cnt, L)
        if L < m:
            svd_rows.extend(rows.tolist())
            continue
        G = G_all[idx]                                                     # (cnt, L, m)
        Qb, Rb = np.linalg.qr(G)                                           # Householder (LAPACK)
        d = np.abs(np.diagonal(Rb, axis1=1, axis2=2))
        ok = d.min(axis=1) > rank_tol(int(L), m) * d.max(axis=1)
        for bad in rows[~ok]:
            svd_rows.append(int(bad))
        if np.any(ok):
            Rt = np.transpose(Rb[ok], (0, 2, 1))                           # R^T, lower triangular
            c = np.linalg.solve(Rt, r_all[rows[ok]][:, :, None])           # R^{-T} r
            dl = (Qb[ok] @ c)[:, :, 0]                                     # Q R^{-T} r
            delta[idx[ok]] = dl
            Q[idx[ok]] = Qb[ok]
            rank[rows[ok]] = m
    for i in svd_rows:
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        used_svd[i] = True
        if b == a:
            rank[i] = 0
            continue
        G = G_all[a:b]
        U, s, Vt = np.linalg.svd(G, full_matrices=False)
        k = int(np.sum(s > rank_tol(b - a, m) * s[0])) if s[0] > 0 else 0
        rank[i] = k
        if k == 0:
            continue
        Q[a:b, :k] = U[:, :k]
        delta[a:b] = U[:, :k] @ ((Vt[:k] @ r_all[i]) / s[:k])
    return Setup(rowptr.astype(np.int32), colind.astype(np.int32), p_hat + delta, Q, rank,
                 used_svd, m)


def project(st: Setup, X: np.ndarray) -> np.ndarray:
    """Pi_B X with Pi_B = I - Q Q^T applied block by block, one block per row
    of P (Sec. 3.1; block form Sec. 3.2)."""
    S = _row_sum_matrix(st.rowptr)
    coef = S @ (st.Q * X[:, None])                   # (n, m): Q_i^T x_i
    return X - np.sum(st.Q * coef[row_ids(st.rowptr)], axis=1)


# --------------------------------------------------------------------------
# a3. K y as the product A Y restricted to the fixed pattern  (Sec. 4)
# --------------------------------------------------------------------------

def masked_product(A: sp.csr_matrix, rowptr, colind, Y: np.ndarray, nc: int) -> np.ndarray:
    """K y: the values of A @ Y at the pattern positions, where Y is the
    matrix with values ``Y`` on the pattern (Sec. 3 eq. 11blk: K is block
    diagonal with blocks A(I_j, I_j), one per column j of P; Sec. 4: the
    product is the SpMM A P with a prescribed pattern)."""
    Ym = as_matrix(Y, rowptr, colind, nc)
    return values_on_pattern(A @ Ym, rowptr, colind)


def energy(A, rowptr, colind, P: np.ndarray, nc: int):
    """tr(P^T A P) = <P, mask(A P)>_F  (Sec. 3, eq. trace)."""
    return np.sum(P * masked_product(A, rowptr, colind, P, nc))


def constraint_error(rowptr, colind, P: np.ndarray, B, Bc) -> float:
    """||P B_c - B||_F / ||B||_F  (the range requirement, Sec. 3 eq. TSP)."""
    n = rowptr.shape[0] - 1
    Pm = as_matrix(np.real(P), rowptr, colind, Bc.shape[0])
    return float(np.linalg.norm(Pm @ Bc - B) / np.linalg.norm(B))


# --------------------------------------------------------------------------
# a5. Preconditioners  (Sec. 3.4)
# --------------------------------------------------------------------------

def jacobi(A: sp.csr_matrix, rowptr, X: np.ndarray) -> np.ndarray:
    """M_J^{-1} X with M_J = diag(K); the diagonal entry of K at position
    (i, j) is A(i, i) (proof of Theorem 3.1), so this scales row i of P by
    1 / A(i, i)."""
    d = A.diagonal()
    return X / d[row_ids(rowptr)]


def block_jacobi(A: sp.csr_matrix, rowptr, colind, X: np.ndarray, bs: int) -> np.ndarray:
    """Nodal block-Jacobi on K: for node a (rows bs*a .. bs*a+bs-1) and each
    column j of P, the entries of the node's rows in column j are multiplied
    by the inverse of the sub-block of A(rows, rows) restricted to the rows
    whose pattern holds j.  Not in the paper; the Pi M^{-1} Pi rule of
    Sec. 3.4.1 makes any such M admissible."""
    n = rowptr.shape[0] - 1
    assert n % bs == 0
    out = np.zeros_like(X)
    Ad = A.tocsr()
    for a in range(n // bs):
        rows = list(range(bs * a, bs * a + bs))
        Aaa = Ad[rows][:, rows].toarray()
        pos = {}
        for t, i in enumerate(rows):
            for s in range(rowptr[i], rowptr[i + 1]):
                pos.setdefault(int(colind[s]), []).append((t, s))
        for j, lst in pos.items():
            ts = [t for t, _ in lst]
            ss = [s for _, s in lst]
            out[ss] = np.linalg.solve(Aaa[np.ix_(ts, ts)], X[ss])
    return out


def block_jacobi_shared(A: sp.csr_matrix, rowptr, colind, X: np.ndarray, bs: int, nc: int) -> np.ndarray:
    """The same nodal block-Jacobi when every node's rows share one column
    set: then Z = mask(D^{-1} X) with D the block diagonal of A, and the
    per-column sub-blocks are the whole A(rows, rows)."""
    n = rowptr.shape[0] - 1
    nb = n // bs
    Ad = A.tocsr()
    blocks = np.zeros((nb, bs, bs))
    for r in range(bs):
        for c in range(bs):
            rr = np.arange(nb) * bs + r
            cc = np.arange(nb) * bs + c
            blocks[:, r, c] = np.asarray(Ad[rr, cc]).ravel()
    inv = np.linalg.inv(blocks)
    Dinv = sp.bsr_matrix((inv, np.arange(nb), np.arange(nb + 1)), shape=(n, n)).tocsr()
    return masked_product(Dinv, rowptr, colind, X, nc)


def rows_share_pattern(rowptr, colind, bs: int) -> bool:
    n = rowptr.shape[0] - 1
    if n % bs:
        return False
    lens = np.diff(rowptr).reshape(-1, bs)
    if np.any(lens != lens[:, :1]):
        return False
    for t in range(1, bs):
        a = np.concatenate([colind[rowptr[i]:rowptr[i + 1]] for i in range(t, n, bs)]) if n else colind[:0]
        b = np.concatenate([colind[rowptr[i]:rowptr[i + 1]] for i in range(0, n, bs)]) if n else colind[:0]
        if not np.array_equal(a, b):
            return False
    return True


# --------------------------------------------------------------------------
# a3-a6. Alg. 3: preconditioned restricted CG  (Sec. 3.4.1)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class RCGResult:
    P: np.ndarray            # final prolongation values w0 + dw on the pattern
    dw: np.ndarray
    iterations: int          # updates applied
    status: str              # "maxit", "converged", "tau", "breakdown"
    gamma: list
    delta: list
    alpha: list
    beta: list
    dE: list                 # gamma_k * alpha_k (Sec. 3.3, eq. CG_dEa)
    energies: Optional[list] = None   # E(P_k), k = 0..iterations, when requested
    tape: Optional[dict] = None


def _stop_reason(gamma, gamma1, gamma_floor):
    """Why the iteration must end before using gamma, or None: a negative
    <r, z> means the preconditioned operator is not positive (breakdown); a
    gamma at or below the relative floor means the residual has vanished to
    rounding (converged)."""
    if np.real(gamma) < 0:
        return "breakdown"
    if np.real(gamma) <= gamma_floor * np.real(gamma1):
        return "converged"
    return None


def rcg(A: sp.csr_matrix, st: Setup, nc: int, maxit: int, precond: str = "jacobi",
        bs: int = 1, tau: float = 0.0, record_energy: bool = False, keep_tape: bool = False,
        gamma_floor: float = 1e-26) -> RCGResult:
    """Alg. 3 of Sec. 3.4.1: conjugate gradients on the projected energy
    Hessian Pi K Pi with the preconditioner Pi M^{-1} Pi, started from the
    corrected tentative prolongation w0 of Alg. 2.

    This is the aggregation form: no row is fixed and the right-hand side f
    is zero, so the first residual is the projected negative half-gradient
    -Pi K w0.  The correction dw is kept apart from w0 and added at the end.
    Each iteration preconditions the residual, makes the new direction
    K-conjugate to the previous one, and steps along it by the exact line
    search.  The energy falls by gamma alpha per step (Sec. 3.3, eq. CG_dEa);
    with tau > 0 the step whose fall is below tau times the first one is not
    taken (Sec. 3.3, eq. relRed).  The first-step test reads "k = 1", and a
    relative floor on gamma ends the loop as converged."""
    rowptr, colind = st.rowptr, st.colind
    shared = precond == "bjacobi" and rows_share_pattern(rowptr, colind, bs)
    colour = sgs.jp_colours(A) if precond == "sgs" else None

    def Minv(x):
        if precond == "jacobi":
            return jacobi(A, rowptr, x)
        if precond == "sgs":  # projected SGS, M_2 of Sec. 3.4.1
            return sgs.sgs(A, rowptr, colind, x, colour)
        if precond == "bjacobi":
            if shared:
                return block_jacobi_shared(A, rowptr, colind, x, bs, nc)
            return block_jacobi(A, rowptr, colind, x, bs)
        if precond == "none":
            return x.copy()
        raise ValueError(precond)

    def K(x):
        return masked_product(A, rowptr, colind, x, nc)

    def PiK(x):
        return project(st, K(x))

    w0 = st.p0
    res = RCGResult(P=None, dw=None, iterations=0, status="maxit", gamma=[], delta=[], alpha=[],
                    beta=[], dE=[], energies=[energy(A, rowptr, colind, w0, nc)] if record_energy else None)
    tape = {"Y": [], "R": [], "Z": []} if keep_tape else None
    dw = np.zeros_like(w0)
    r = -PiK(w0)
    y = None              # current search direction
    gamma_prev = None     # <r, z> of the previous iteration
    for k in range(1, maxit + 1):
        z = project(st, Minv(r))
        gamma = np.sum(r * z)
        if k == 1:
            gamma1 = gamma
        reason = _stop_reason(gamma, gamma1, gamma_floor)
        if reason:
            res.status = reason
            break
        # conjugate direction: the first one is z itself
        beta = 0.0 if k == 1 else gamma / gamma_prev
        y = z.copy() if k == 1 else z + beta * y
        gamma_prev = gamma
        # exact line search along y
        yh = PiK(y)
        delta = np.sum(y * yh)
        if np.real(delta) <= 0:
            res.status = "breakdown"
            break
        alpha = gamma / delta
        dE = gamma * alpha
        if k == 1:
            dE1 = dE
        if tau > 0 and np.real(dE) < tau * np.real(dE1):
            res.status = "tau"
            break
        if keep_tape:
            tape["Y"].append(y.copy())
            tape["R"].append(r.copy())
            tape["Z"].append(z.copy())
        dw = dw + alpha * y
        r = r - alpha * yh
        for hist, v in ((res.gamma, gamma), (res.delta, delta), (res.alpha, alpha),
                        (res.beta, beta), (res.dE, dE)):
            hist.append(v)
        res.iterations = k
        if record_energy:
            res.energies.append(energy(A, rowptr, colind, w0 + dw, nc))
    res.P = w0 + dw
    res.dw = dw
    if keep_tape:
        tape["r_final"] = r
        res.tape = tape
    return res


# --------------------------------------------------------------------------
# whole path
# --------------------------------------------------------------------------

def solve(inp, maxit: Optional[int] = None, precond: Optional[str] = None, tau: float = 0.0,
          record_energy: bool = False, pattern=None, keep_tape: bool = False):
    """Pattern (eq. enlPatt) -> Alg. 2 -> Alg. 3 for an input from ``gen``.
    Returns (Setup, RCGResult)."""
    if pattern is None:
        if inp.pattern_power == 0:
            pattern = inp.extra["pattern"]
        else:
            pattern = pattern_expand(inp.A, inp.P0, inp.pattern_power)
    rowptr, colind = pattern
    st = emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    res = rcg(inp.A, st, inp.nc, inp.maxit if maxit is None else maxit,
              precond or inp.precond, bs=inp.block, tau=tau, record_energy=record_energy,
              keep_tape=keep_tape)
    return st, res
