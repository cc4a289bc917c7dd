"""CPU FP64 oracle of the projected symmetric Gauss-Seidel preconditioner
M_2 (Sec. 3.4.1, eq. SGS_prec with its second term dropped, as the paper
does): z = Pi M_SGS^{-1} r with M_SGS^{-1} = (L + D)^{-T} D (L + D)^{-1}.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library.

K is block diagonal with one block per column j of P (Sec. 3, eq. 11blk):
K_j = A(I_j, I_j) over the rows I_j whose pattern holds j.  So SGS on K is SGS
on every K_j separately; L is the strictly lower part of K_j and D its
diagonal, in the order the rows are swept.

The paper fixes no order.  The reading here: rows are swept colour by colour
(a colouring of A's graph in which no two coupled rows share a colour), by
index within a colour.  Rows of one colour are not coupled, so their order
does not change the result, and each colour's rows can be updated together.
The colouring is Jones and Plassmann's: in round r, every uncoloured row
whose priority exceeds that of all its uncoloured neighbours is picked (an
independent set), and takes the smallest colour not held by a neighbour
coloured in an earlier round.  The priority of row i is (h(i), i) compared
lexicographically, with h the 32-bit finalizer of MurmurHash3 (Appleby),
so the colouring is a fixed function of A's structure.  A's stored structure
(explicit zeros included) is the graph; it is assumed structurally
symmetric, as an SPD matrix stored whole is.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

_M32 = np.uint64(0xFFFFFFFF)


def fmix32(x) -> np.ndarray:
    """The 32-bit finalizer of MurmurHash3 on each element (uint32 result)."""
    h = np.asarray(x, dtype=np.uint64) & _M32
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & _M32
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & _M32
    h ^= h >> np.uint64(16)
    return h


def priorities(n: int) -> np.ndarray:
    """Row priority as one unsigned 64-bit key: h(i) in the high half, i in
    the low half (so no two rows tie)."""
    i = np.arange(n, dtype=np.uint64)
    return (fmix32(i) << np.uint64(32)) | i


def jp_rounds(A: sp.csr_matrix):
    """(round, colour) of every row.  Round r picks every uncoloured row whose
    priority exceeds that of all its uncoloured neighbours (an independent
    set); each picked row takes the smallest colour that none of its
    neighbours coloured in earlier rounds holds (first fit)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    key = priorities(n)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    off = rows != cols                      # graph edges (the diagonal is no edge)
    er, ec = rows[off], cols[off]
    rnd = np.full(n, -1, dtype=np.int64)
    colour = np.full(n, -1, dtype=np.int64)
    r = 0
    while np.any(rnd < 0):
        active = rnd < 0
        # the largest priority among each row's uncoloured neighbours
        live = active[ec]
        nb = np.zeros(n, dtype=np.uint64)
        np.maximum.at(nb, er[live], key[ec[live]])
        has = np.zeros(n, dtype=bool)
        has[er[live]] = True
        pick = np.flatnonzero(active & (~has | (key > nb)))
        for i in pick:
            nbr = A.indices[A.indptr[i]:A.indptr[i + 1]]
            used = set(colour[k] for k in nbr if k != i and rnd[k] >= 0)
            c = 0
            while c in used:
                c += 1
            colour[i] = c
        rnd[pick] = r
        r += 1
    return rnd, colour


def jp_colours(A: sp.csr_matrix) -> np.ndarray:
    """Colour of every row (Jones-Plassmann rounds, first-fit colours)."""
    return jp_rounds(A)[1]


def sweep_order(colour: np.ndarray) -> np.ndarray:
    """Position of every row in the sweep: by colour, then by index."""
    n = colour.shape[0]
    order = np.lexsort((np.arange(n), colour))
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    return pos


def sgs(A: sp.csr_matrix, rowptr, colind, X: np.ndarray, colour: np.ndarray) -> np.ndarray:
    """M_SGS^{-1} X on the pattern: for every column j of P, the entries of
    X in column j (rows I_j, in sweep order) go through a forward triangular
    solve with L + D, a scaling by D and a backward solve with (L + D)^T."""
    A = sp.csr_matrix(A)
    rowptr = np.asarray(rowptr)
    colind = np.asarray(colind)
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    pos = sweep_order(colour)
    # entries grouped by column, each group in sweep order of its rows
    ent = np.lexsort((pos[rows], colind))
    bounds = np.flatnonzero(np.diff(colind[ent])) + 1
    out = np.zeros_like(X)
    for grp in np.split(ent, bounds):
        if grp.size == 0:
            continue
        I = rows[grp]
        Kj = A[I][:, I].toarray()
        LD = np.tril(Kj)
        u = sla.solve_triangular(LD, X[grp], lower=True)
        out[grp] = sla.solve_triangular(LD.T, np.diag(Kj) * u, lower=False)
    return out
