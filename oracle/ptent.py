"""CPU FP64 oracle of the tentative prolongation set-up (Alg. 1, Sec. 3.2)
and of the classical C/F form P = [W; I] (Sec. 2, eqs. CFspl and prol).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests and the smoke check do.  It shares no code with the HIP
library.  Plain Python loops over small dense blocks, in the order the text
describes, so each step can be checked by eye.

Alg. 1, for every FINE node i: for l = 1, 2, ..., l_max, take the COARSE
nodes within distance l of i in the strength graph S (N_i, ordered by
coarse index), select m of them with max vol on the rows of V_c(N_i, :),
solve B w = v_i for the selected block B = V_c(J, :)^T, and keep w as row i
of P_0 as soon as v_i - B w vanishes.  COARSE rows of P_0 are the identity
(P = [W; I]).

Readings where the paper is silent (listed with reasons in the design
notes):
* distance: hops in the graph of S's stored off-diagonal structure, i
  itself at distance 0;
* max vol: Gaussian elimination with partial (row) pivoting gives the
  starting rows (a column whose remaining entries are all below 1e-12 of the
  largest entry of the matrix gives none, so a rank-r set yields r rows
  spanning it); with m rows, while some coefficient of a row in the basis
  of the selected rows exceeds 1 + 1/20 in modulus, that row replaces the
  selected row of the coefficient (Goreinov et al.'s iteration); pivots and
  maxima go to the first row in order on ties;
* "residual = 0": ||v - B w||_2 <= 1e-10 ||v||_2 (an exact fit up to
  rounding); a row never fitted up to l_max stays empty (Alg. 2 then treats
  it by least squares on the grown pattern);
* w: the square system by Gaussian elimination with partial pivoting, a
  non-square one (fewer rows selected than m) through its normal equations.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MAXVOL_TOL = 1.05
MAXVOL_SWAPS = 64
PIVOT_TOL = 1e-12
FIT_TOL = 1e-10


def distance_sets(S: sp.csr_matrix, i: int, lmax: int):
    """Nodes at distance exactly 1..lmax from i (breadth-first levels)."""
    seen = {i}
    frontier = [i]
    levels = []
    for _ in range(lmax):
        nxt = []
        for u in frontier:
            for v in S.indices[S.indptr[u]:S.indptr[u + 1]]:
                v = int(v)
                if v not in seen:
                    seen.add(v)
                    nxt.append(v)
        levels.append(nxt)
        frontier = nxt
    return levels


def ge_solve(M, rhs):
    """Solve M x = rhs (M square, rhs a matrix) by Gaussian elimination with
    partial pivoting (first row on ties); None when a pivot is zero."""
    n = len(M)
    a = [list(map(float, row)) for row in M]
    b = [list(map(float, row)) for row in rhs]
    for j in range(n):
        p = j
        for r in range(j + 1, n):
            if abs(a[r][j]) > abs(a[p][j]):
                p = r
        if a[p][j] == 0.0:
            return None
        a[j], a[p] = a[p], a[j]
        b[j], b[p] = b[p], b[j]
        for r in range(j + 1, n):
            f = a[r][j] / a[j][j]
            for c in range(j, n):
                a[r][c] = a[r][c] - f * a[j][c]
            for c in range(len(b[r])):
                b[r][c] = b[r][c] - f * b[j][c]
    x = [[0.0] * len(b[0]) for _ in range(n)]
    for j in range(n - 1, -1, -1):
        for c in range(len(b[0])):
            s = b[j][c]
            for k in range(j + 1, n):
                s = s - a[j][k] * x[k][c]
            x[j][c] = s / a[j][j]
    return x


def maxvol(M) -> list:
    """Indices of (up to) m rows of the k x m matrix M with locally maximal
    volume (the readings above)."""
    k = len(M)
    m = len(M[0]) if k else 0
    U = [list(map(float, row)) for row in M]
    floor = PIVOT_TOL * max((abs(x) for row in U for x in row), default=0.0)
    sel, avail = [], list(range(k))
    for j in range(m):
        best, bv = -1, floor
        for r in avail:
            if abs(U[r][j]) > bv:
                best, bv = r, abs(U[r][j])
        if best < 0:
            continue                    # column j adds no direction: skip it
        sel.append(best)
        avail.remove(best)
        for r in avail:
            f = U[r][j] / U[best][j]
            for c in range(j, m):
                U[r][c] = U[r][c] - f * U[best][c]
    if len(sel) < m:
        return sel
    for _ in range(MAXVOL_SWAPS):
        # coefficients of every row in the basis of the selected rows:
        # C = M M_sel^{-1}, i.e. M_sel^T C^T = M^T
        Msel_T = [[M[sel[c]][r] for c in range(m)] for r in range(m)]
        Ct = ge_solve(Msel_T, [[M[q][r] for q in range(k)] for r in range(m)])
        if Ct is None:
            break
        best, bc, bv = -1, -1, MAXVOL_TOL
        for q in range(k):
            if q in sel:
                continue
            for c in range(m):
                if abs(Ct[c][q]) > bv:
                    best, bc, bv = q, c, abs(Ct[c][q])
        if best < 0:
            break
        sel[bc] = best
    return sel


def fit_row(Vsel, v):
    """w with B w = v, B = Vsel^T (m x s); (w, relative residual)."""
    s = len(Vsel)
    m = len(v)
    B = [[Vsel[c][x] for c in range(s)] for x in range(m)]
    if s == 0:
        sol = []
    elif s == m:
        sol = ge_solve(B, [[vx] for vx in v])
    else:   # normal equations B^T B w = B^T v
        BtB = [[sum(B[x][a] * B[x][b] for x in range(m)) for b in range(s)] for a in range(s)]
        Btv = [[sum(B[x][a] * v[x] for x in range(m))] for a in range(s)]
        sol = ge_solve(BtB, Btv)
    if sol is None:
        return None, np.inf
    w = [sol[a][0] for a in range(s)]  # (no entries when nothing was selected)
    res = [v[x] - sum(B[x][a] * w[a] for a in range(s)) for x in range(m)]
    nv = float(np.sqrt(sum(t * t for t in v)))
    nr = float(np.sqrt(sum(t * t for t in res)))
    return w, (nr / nv if nv > 0 else nr)


def ptent_setup(S: sp.csr_matrix, V: np.ndarray, cf: np.ndarray, lmax: int):
    """Alg. 1.  ``cf[i]`` is the coarse index of node i (>= 0) or -1 for a
    FINE node.  Returns (P_0 as CSR n x nc, level of every row: the distance
    at which it was fitted, 0 for COARSE rows, -1 when never fitted)."""
    S = sp.csr_matrix(S)
    V = np.asarray(V, dtype=np.float64)
    n, m = V.shape
    nc = int(cf.max()) + 1 if n else 0
    rows, cols, vals = [], [], []
    level = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        if cf[i] >= 0:
            rows.append(i)
            cols.append(int(cf[i]))
            vals.append(1.0)
            level[i] = 0
            continue
        near = []
        for l, ring in enumerate(distance_sets(S, i, lmax), start=1):
            near += [u for u in ring if cf[u] >= 0]
            N = sorted(near, key=lambda u: cf[u])
            if not N:
                continue
            M = [list(V[u]) for u in N]
            sel = sorted(maxvol(M))
            w, rel = fit_row([M[q] for q in sel], list(V[i]))
            if w is not None and rel <= FIT_TOL:
                for q, wq in zip(sel, w):
                    rows.append(i)
                    cols.append(int(cf[N[q]]))
                    vals.append(wq)
                level[i] = l
                break
    P0 = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
    P0.sort_indices()
    return P0, level


def cf_pattern(A: sp.csr_matrix, P0: sp.csr_matrix, cf: np.ndarray, k: int):
    """Pattern of P = [W; I]: rows of struct(A^k P0) (eq. enlPatt, the whole
    P0 including its identity rows) for FINE nodes; COARSE rows keep their
    single identity entry (they are not unknowns)."""
    from .rcg import pattern_expand

    rp, ci = pattern_expand(A, P0, k)
    rows = []
    for i in range(A.shape[0]):
        if cf[i] >= 0:
            rows.append(np.array([cf[i]], dtype=np.int32))
        else:
            rows.append(ci[rp[i]:rp[i + 1]])
    rp2 = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int32)
    ci2 = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return rp2, ci2
