"""Dense brute-force constructions used to pin the oracle.

These build the paper's objects as explicit dense matrices on tiny inputs
(K of Sec. 3 eq. 11blk in row-wise entry order, the block constraint matrix
of eq. Constr_Mat, the saddle-point system eq. sadsys, the Krylov space of
Sec. 3.1) and solve them with plain dense linear algebra: a route that shares
nothing with the oracle's sparse, iterative one.
"""

import numpy as np


def entry_rows_cols(rowptr, colind):
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    return rows, np.asarray(colind)


def dense_K(A, rowptr, colind):
    """K in row-wise entry order: K[s,t] = A[row(s), row(t)] when entries s
    and t lie in the same column of P, else 0 (no coupling between columns)."""
    Ad = A.toarray()
    rows, cols = entry_rows_cols(rowptr, colind)
    same = cols[:, None] == cols[None, :]
    return np.where(same, Ad[np.ix_(rows, rows)], 0.0)


def dense_constraint(rowptr, colind, Bc):
    """Btil (nnz x n*m): column i*m + c holds Bc[J_i, c] on row i's entries,
    so Btil^T p stacks G_i^T p_i (eq. Constr_Mat)."""
    n = len(rowptr) - 1
    m = Bc.shape[1]
    nnz = len(colind)
    Bt = np.zeros((nnz, n * m))
    rows, cols = entry_rows_cols(rowptr, colind)
    for s in range(nnz):
        for c in range(m):
            Bt[s, rows[s] * m + c] = Bc[cols[s], c]
    return Bt


def dense_projector(rowptr, colind, Bc):
    """Pi = I - Bt (Bt^T Bt)^+ Bt^T, via the pseudo-inverse."""
    Bt = dense_constraint(rowptr, colind, Bc)
    return np.eye(Bt.shape[0]) - Bt @ np.linalg.pinv(Bt.T @ Bt) @ Bt.T


def kkt_solution(A, rowptr, colind, B, Bc):
    """argmin p^T K p subject to Btil^T p = vec(B): the saddle-point system
    [[K, Bt], [Bt^T, 0]] [p; lam] = [0; g] (eq. sadsys with f = 0)."""
    K = dense_K(A, rowptr, colind)
    Bt = dense_constraint(rowptr, colind, Bc)
    nnz, nm = Bt.shape
    M = np.zeros((nnz + nm, nnz + nm))
    M[:nnz, :nnz] = K
    M[:nnz, nnz:] = Bt
    M[nnz:, :nnz] = Bt.T
    rhs = np.concatenate([np.zeros(nnz), np.asarray(B).reshape(-1)])
    sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
    return sol[:nnz]


def dense_energy(A, rowptr, colind, p, nc):
    n = len(rowptr) - 1
    P = np.zeros((n, nc))
    rows, cols = entry_rows_cols(rowptr, colind)
    P[rows, cols] = p
    return float(np.trace(P.T @ A.toarray() @ P))


def krylov_iterate(A, rowptr, colind, Bc, w0, Minv, k):
    """The k-th PCG iterate as the minimiser of E(w0 + x) over
    x in span{v, T v, ..., T^{k-1} v}, v = Pi M^{-1} Pi r0, T = Pi M^{-1} Pi K,
    r0 = -Pi K w0 (Sec. 3.1: CG on Pi K Pi with the Pi M^{-1} Pi
    preconditioner of Sec. 3.4.1).  ``Minv`` is the dense preconditioner."""
    K = dense_K(A, rowptr, colind)
    Pi = dense_projector(rowptr, colind, Bc)
    Mt = Pi @ Minv @ Pi
    r0 = -Pi @ K @ w0
    v = Mt @ r0
    basis = []
    for _ in range(k):
        basis.append(v)
        v = Mt @ (K @ v)
    V = np.stack(basis, axis=1)
    Qv, _ = np.linalg.qr(V)
    H = Qv.T @ K @ Qv
    c = np.linalg.solve(H, -Qv.T @ K @ w0)
    return w0 + Qv @ c


def dense_jacobi(A, rowptr, colind):
    rows, _ = entry_rows_cols(rowptr, colind)
    return np.diag(1.0 / A.diagonal()[rows])


def dense_block_jacobi(A, rowptr, colind, bs):
    """The nodal block-Jacobi preconditioner as an explicit matrix in
    row-wise entry order: M[s, t] = A[row(s), row(t)] when entries s and t lie
    in the same column of P and their rows belong to the same node of bs
    consecutive rows, else 0.  It is K (eq. 11blk) with every coupling
    between different nodes removed, so it is block diagonal with one block
    per (node, column) pair."""
    K = dense_K(A, rowptr, colind)
    rows, _ = entry_rows_cols(rowptr, colind)
    node = rows // bs
    return np.where(node[:, None] == node[None, :], K, 0.0)
